// Perfect spatial hash construction (host) and the inrf_build_psh* entry
// points.
//
// Hash of Sec. 4.1, Eq. 1: h(p) = h0(p) + Phi(h1(p)) with h0(p) = p mod mbar,
// h1(p) = p mod rbar (component-wise) and the sum taken mod mbar, so that the
// table of mbar^3 slots holds every occupied vertex without collision.  The
// paper's offsets come from a heuristic that prefers mapping neighbouring
// points to neighbouring slots; this is the deterministic greedy used here:
//
//   sizes    mbar: smallest with load_pct*mbar^3 >= 100*n and
//            1024*mbar >= N+1.
//            rbar: smallest >= 2 with bucket_keys*rbar^3 >= n, then grown
//            until gcd(mbar, rbar) = 1 and mbar*rbar >= N+1; by the Chinese
//            remainder theorem the keys of one bucket then differ mod mbar.
//   order    buckets {p : p mod rbar = q}, largest first, ties by linear q.
//   offsets  per bucket, the first that puts every key on a free slot among
//            (i) the offsets already held by its 6 face neighbours in offset
//            space (-x,+x,-y,+y,-z,+z, wrapping, duplicates skipped), (ii)
//            n_random values r_k = splitmix64(splitmix64(seed) + 256 q + k)
//            mapped to (r mod mbar, (r>>21) mod mbar, (r>>42) mod mbar),
//            (iii) every offset that puts the bucket's first key on a free
//            slot, free slots in ascending order.
//   failure  rbar grows (same conditions) and the level restarts; after
//            max_restarts restarts mbar grows by one.
// Offsets are packed x | y<<10 | z<<20; empty buckets hold 0.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>

#include "brick_layout.hpp"
#include "host_common.hpp"
#include "host_internal.hpp"

namespace inrf {

namespace {

thread_local std::string g_error;

uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int64_t icbrt_ceil(int64_t n, int64_t mult) {
    int64_t r = std::max<int64_t>(1, int64_t(std::llround(std::cbrt(double(n) / double(mult)))) - 2);
    while (mult * r * r * r < n) ++r;
    while (r > 1 && mult * (r - 1) * (r - 1) * (r - 1) >= n) --r;
    return r;
}

int64_t fix_rbar(int64_t r, int64_t mbar, int64_t N) {
    while (std::gcd(mbar, r) != 1 || mbar * r < N + 1) ++r;
    return r;
}

struct Bits {
    std::vector<uint64_t> w;
    explicit Bits(int64_t n) : w(size_t((n + 63) / 64), 0) {}
    bool get(int64_t i) const { return (w[size_t(i >> 6)] >> (i & 63)) & 1; }
    void set(int64_t i) { w[size_t(i >> 6)] |= uint64_t(1) << (i & 63); }
    // first clear bit >= i, or -1 (bits at or beyond `limit` are ignored)
    int64_t next_clear(int64_t i, int64_t limit) const {
        while (i < limit) {
            const uint64_t inv = ~w[size_t(i >> 6)] >> (i & 63);
            if (inv) {
                const int64_t j = i + __builtin_ctzll(inv);
                return j < limit ? j : -1;
            }
            i = (i | 63) + 1;
        }
        return -1;
    }
};

constexpr uint32_t kUnset = 0xFFFFFFFFu;

inline uint32_t pack(int64_t x, int64_t y, int64_t z) { return uint32_t(x | (y << 10) | (z << 20)); }

bool try_build(PshLevel& L, int64_t mbar, int64_t rbar, const inrf_psh_params& p) {
    const int64_t n = int64_t(L.keys.size()), M = int64_t(L.res) + 1;
    const int64_t R3 = rbar * rbar * rbar, M3 = mbar * mbar * mbar;
    std::vector<int32_t> h0(size_t(n) * 3);
    std::vector<int64_t> qlin(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
        const int64_t key = L.keys[size_t(i)];
        const int64_t x = key % M, y = (key / M) % M, z = key / (M * M);
        h0[size_t(i) * 3 + 0] = int32_t(x % mbar);
        h0[size_t(i) * 3 + 1] = int32_t(y % mbar);
        h0[size_t(i) * 3 + 2] = int32_t(z % mbar);
        qlin[size_t(i)] = ((z % rbar) * rbar + (y % rbar)) * rbar + (x % rbar);
    }
    // stable counting sort of keys into buckets (canonical key order kept)
    std::vector<int64_t> start(size_t(R3) + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++start[size_t(qlin[size_t(i)]) + 1];
    for (int64_t q = 0; q < R3; ++q) start[size_t(q) + 1] += start[size_t(q)];
    std::vector<int32_t> member(static_cast<size_t>(n));
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) member[size_t(fill[size_t(qlin[size_t(i)])]++)] = int32_t(i);
    }
    // bucket order: size descending, linear q ascending
    int64_t max_size = 0;
    for (int64_t q = 0; q < R3; ++q) max_size = std::max(max_size, start[size_t(q) + 1] - start[size_t(q)]);
    std::vector<int64_t> by_size(size_t(max_size) + 2, 0);
    for (int64_t q = 0; q < R3; ++q) ++by_size[size_t(start[size_t(q) + 1] - start[size_t(q)])];
    std::vector<int64_t> sz_start(size_t(max_size) + 2, 0);  // position of size s in the order
    {
        int64_t pos = 0;
        for (int64_t s = max_size; s >= 1; --s) {
            sz_start[size_t(s)] = pos;
            pos += by_size[size_t(s)];
        }
    }
    std::vector<int64_t> order;
    {
        int64_t nonempty = 0;
        for (int64_t s = 1; s <= max_size; ++s) nonempty += by_size[size_t(s)];
        order.resize(size_t(nonempty));
        for (int64_t q = 0; q < R3; ++q) {
            const int64_t s = start[size_t(q) + 1] - start[size_t(q)];
            if (s > 0) order[size_t(sz_start[size_t(s)]++)] = q;
        }
    }
    Bits used(M3);
    std::vector<uint32_t> phi(size_t(R3), kUnset);
    const uint64_t s0 = splitmix64(p.seed);
    std::vector<int64_t> chosen, trial;
    auto fits = [&](int64_t b, int64_t e, int64_t ox, int64_t oy, int64_t oz, std::vector<int64_t>& out) {
        out.clear();
        for (int64_t k = b; k < e; ++k) {
            const int32_t* h = &h0[size_t(member[size_t(k)]) * 3];
            int64_t sx = h[0] + ox, sy = h[1] + oy, sz = h[2] + oz;
            if (sx >= mbar) sx -= mbar;
            if (sy >= mbar) sy -= mbar;
            if (sz >= mbar) sz -= mbar;
            const int64_t s = (sz * mbar + sy) * mbar + sx;
            if (used.get(s)) return false;
            out.push_back(s);
        }
        return true;
    };
    for (const int64_t q : order) {
        const int64_t b = start[size_t(q)], e = start[size_t(q) + 1];
        const int64_t qx = q % rbar, qy = (q / rbar) % rbar, qz = q / (rbar * rbar);
        uint32_t cands[6];
        int nc = 0;
        static const int d6[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
        for (const auto& d : d6) {
            const int64_t nx = (qx + d[0] + rbar) % rbar, ny = (qy + d[1] + rbar) % rbar, nz = (qz + d[2] + rbar) % rbar;
            const uint32_t v = phi[size_t((nz * rbar + ny) * rbar + nx)];
            if (v == kUnset) continue;
            bool dup = false;
            for (int i = 0; i < nc; ++i) dup |= cands[i] == v;
            if (!dup) cands[nc++] = v;
        }
        bool ok = false;
        uint32_t off = 0;
        for (int i = 0; i < nc && !ok; ++i) {
            off = cands[i];
            ok = fits(b, e, off & 1023, (off >> 10) & 1023, (off >> 20) & 1023, chosen);
        }
        for (int k = 0; k < p.n_random && !ok; ++k) {
            const uint64_t r = splitmix64(s0 + uint64_t(q) * 256u + uint64_t(k));
            const int64_t ox = int64_t(r % uint64_t(mbar)), oy = int64_t((r >> 21) % uint64_t(mbar)),
                          oz = int64_t((r >> 42) % uint64_t(mbar));
            off = pack(ox, oy, oz);
            ok = fits(b, e, ox, oy, oz, chosen);
        }
        if (!ok) {
            const int32_t* h = &h0[size_t(member[size_t(b)]) * 3];
            for (int64_t s = used.next_clear(0, M3); s >= 0 && !ok; s = used.next_clear(s + 1, M3)) {
                const int64_t sx = s % mbar, sy = (s / mbar) % mbar, sz = s / (mbar * mbar);
                const int64_t ox = (sx - h[0] + mbar) % mbar, oy = (sy - h[1] + mbar) % mbar,
                              oz = (sz - h[2] + mbar) % mbar;
                off = pack(ox, oy, oz);
                ok = fits(b, e, ox, oy, oz, chosen);
            }
        }
        if (!ok) return false;
        phi[size_t(q)] = off;
        for (const int64_t s : chosen) used.set(s);
    }
    L.slots.resize(size_t(n));
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t o = phi[size_t(qlin[size_t(i)])];
        const int32_t* h = &h0[size_t(i) * 3];
        const int64_t sx = (h[0] + int64_t(o & 1023)) % mbar, sy = (h[1] + int64_t((o >> 10) & 1023)) % mbar,
                      sz = (h[2] + int64_t((o >> 20) & 1023)) % mbar;
        L.slots[size_t(i)] = int32_t((sz * mbar + sy) * mbar + sx);
    }
    for (auto& v : phi)
        if (v == kUnset) v = 0;
    L.phi.swap(phi);
    return true;
}

void check_params(const inrf_psh_params& p) {
    require(p.load_pct >= 1 && p.load_pct <= 100, "load_pct must be in [1, 100]");
    require(p.bucket_keys >= 1 && p.bucket_keys <= 1024, "bucket_keys must be in [1, 1024]");
    require(p.n_random >= 0 && p.n_random <= 256, "n_random must be in [0, 256]");
    require(p.max_restarts >= 0 && p.max_restarts <= 64, "max_restarts must be in [0, 64]");
    require(p.dilate >= 0 && p.dilate <= 8, "dilate must be in [0, 8]");
    require(p.n_threads >= 0, "n_threads must be >= 0");
}

}  // namespace

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
const char* last_error() { return g_error.c_str(); }

int resolve_threads(int requested) {
    if (requested > 0) return requested;
    const unsigned h = std::thread::hardware_concurrency();
    return h ? int(std::min(h, 64u)) : 1;
}

void build_psh_level(PshLevel& L, const inrf_psh_params& p) {
    const int64_t n = int64_t(L.keys.size()), N = L.res;
    // mbar * 1024 >= N + 1 keeps rbar <= 1024 for any key count
    int64_t mbar = std::max(icbrt_ceil(100 * std::max<int64_t>(n, 1), p.load_pct), (N + 1 + 1023) / 1024);
    int64_t rbar = fix_rbar(std::max<int64_t>(2, icbrt_ceil(std::max<int64_t>(n, 1), p.bucket_keys)), mbar, N);
    int restarts = 0;
    for (;;) {
        for (int r = 0; r <= p.max_restarts; ++r) {
            if (mbar > 1024) fail(INRF_E_BUILD, "offset components would exceed 10 bits (mbar > 1024)");
            if (try_build(L, mbar, rbar, p)) {
                L.mbar = int32_t(mbar);
                L.rbar = int32_t(rbar);
                L.restarts = restarts;
                return;
            }
            ++restarts;
            rbar = fix_rbar(rbar + 1, mbar, N);
        }
        mbar += 1;
        rbar = fix_rbar(rbar, mbar, N);
    }
}

}  // namespace inrf

using namespace inrf;

extern "C" {

const char* inrf_last_error(void) { return inrf::last_error(); }

int32_t inrf_version(void) { return 100; }

void inrf_psh_params_default(inrf_psh_params* p) {
    if (!p) return;
    p->seed = 1;
    p->dilate = 1;
    p->load_pct = 80;
    p->bucket_keys = 2;
    p->n_random = 32;
    p->max_restarts = 4;
    p->n_threads = 0;
}

inrf_status inrf_build_psh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           int32_t n_levels, const int32_t* res, const inrf_psh_params* params, inrf_psh** out) {
    return guarded("inrf_build_psh", [&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(params != nullptr, "params is NULL");
        check_params(*params);
        require(n_verts >= 0 && n_tris >= 0, "negative sizes");
        require(n_verts == 0 || verts, "verts is NULL");
        require(n_tris == 0 || tris, "tris is NULL");
        require(n_levels >= 1 && n_levels <= INRF_MAX_LEVELS, "n_levels must be in [1, 32]");
        require(res != nullptr, "res is NULL");
        for (int64_t i = 0; i < n_tris * 3; ++i)
            require(tris[i] >= 0 && tris[i] < n_verts, "triangle vertex index out of range");
        const int threads = resolve_threads(params->n_threads);
        auto* obj = new inrf_psh();
        try {
            obj->levels.resize(size_t(n_levels));
            for (int l = 0; l < n_levels; ++l)
                require(res[l] >= 1 && res[l] <= 4096, "resolution must be in [1, 4096]");
            // occupancy level by level (each voxelisation is itself parallel),
            // then the sequential offset searches of all levels side by side
            for (int l = 0; l < n_levels; ++l) {
                PshLevel& L = obj->levels[size_t(l)];
                L.res = res[l];
                L.keys = shell_keys(verts, n_verts, tris, n_tris, res[l], params->dilate, threads);
            }
            std::vector<Error> errs(size_t(n_levels), Error{INRF_OK, ""});
            std::vector<std::thread> pool;
            std::atomic<int> next{0};
            const int workers = std::min(threads, int(n_levels));
            for (int w = 0; w < workers; ++w)
                pool.emplace_back([&] {
                    // largest levels first so the longest search starts first
                    for (int i = next.fetch_add(1); i < n_levels; i = next.fetch_add(1)) {
                        const int l = n_levels - 1 - i;
                        try {
                            build_psh_level(obj->levels[size_t(l)], *params);
                        } catch (const Error& e) {
                            errs[size_t(l)] = e;
                        } catch (const std::bad_alloc&) {
                            errs[size_t(l)] = Error{INRF_E_BUILD, "host out of memory"};
                        }
                    }
                });
            for (auto& t : pool) t.join();
            for (int l = 0; l < n_levels; ++l)
                if (errs[size_t(l)].code != INRF_OK)
                    fail(errs[size_t(l)].code, "level " + std::to_string(l) + ": " + errs[size_t(l)].msg);
        } catch (...) {
            delete obj;
            throw;
        }
        *out = obj;
    });
}

inrf_status inrf_build_psh_keys(int32_t res, const int64_t* keys, int64_t n_keys, const inrf_psh_params* params,
                                inrf_psh** out) {
    return guarded("inrf_build_psh_keys", [&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(params != nullptr, "params is NULL");
        check_params(*params);
        require(res >= 1 && res <= 4096, "resolution must be in [1, 4096]");
        require(n_keys >= 0 && (n_keys == 0 || keys), "bad keys");
        const int64_t M = int64_t(res) + 1;
        for (int64_t i = 0; i < n_keys; ++i) {
            require(keys[i] >= 0 && keys[i] < M * M * M, "key out of range");
            require(i == 0 || keys[i] > keys[i - 1], "keys must be strictly ascending");
        }
        auto* obj = new inrf_psh();
        try {
            obj->levels.resize(1);
            PshLevel& L = obj->levels[0];
            L.res = res;
            L.keys.assign(keys, keys + n_keys);
            build_psh_level(L, *params);
        } catch (...) {
            delete obj;
            throw;
        }
        *out = obj;
    });
}

int32_t inrf_psh_levels(const inrf_psh* psh) { return psh ? int32_t(psh->levels.size()) : 0; }

inrf_status inrf_psh_level(const inrf_psh* psh, int32_t level, inrf_psh_level_info* info, int64_t* keys,
                           uint32_t* phi, int32_t* slots) {
    return guarded("inrf_psh_level", [&] {
        require(psh != nullptr && info != nullptr, "NULL argument");
        require(level >= 0 && level < int32_t(psh->levels.size()), "level out of range");
        const PshLevel& L = psh->levels[size_t(level)];
        info->res = L.res;
        info->mbar = L.mbar;
        info->rbar = L.rbar;
        info->restarts = L.restarts;
        info->n_keys = int64_t(L.keys.size());
        info->n_slots = int64_t(L.mbar) * L.mbar * L.mbar;
        info->n_phi = int64_t(L.phi.size());
        if (keys) std::memcpy(keys, L.keys.data(), L.keys.size() * sizeof(int64_t));
        if (phi) std::memcpy(phi, L.phi.data(), L.phi.size() * sizeof(uint32_t));
        if (slots) std::memcpy(slots, L.slots.data(), L.slots.size() * sizeof(int32_t));
    });
}

void inrf_psh_free(inrf_psh* psh) { delete psh; }

int64_t inrf_brick_entries(int32_t side) {
    if (side < 1 || side > 1024) return -1;
    return inrf::brick_entries(side);
}

inrf_status inrf_brick_index(int32_t side, const int64_t* linear, int64_t n, int64_t* out) {
    return guarded("inrf_brick_index", [&] {
        require(side >= 1 && side <= 1024, "side must be in [1, 1024]");
        require(n >= 0, "n must be >= 0");
        require(n == 0 || (linear && out), "NULL buffer");
        const int64_t s = side, cells = s * s * s;
        for (int64_t i = 0; i < n; ++i) require(linear[i] >= 0 && linear[i] < cells, "linear index out of range");
        const uint32_t row = inrf::brick_row(side), plane = inrf::brick_plane(side);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t v = linear[i];
            const int x = int(v % s), y = int((v / s) % s), z = int(v / (s * s));
            out[i] = int64_t(inrf::brick_x(x)) + inrf::brick_y(y, row) + inrf::brick_z(z, plane);
        }
    });
}

}  // extern "C"
