// Exact shell voxelisation of a triangle proxy into the occupied vertices of
// one grid level.
//
// The paper keeps features only for voxels around the possible hit points
// (Sec. 4.2, "Implementation with PSH encoding") and derives the hash from an
// occupancy field (Sec. 4.1).  For a mesh proxy at resolution N:
//   surface cell  : closed box [p/N, (p+1)/N] meets a triangle;
//   occupied cell : within Chebyshev distance `dilate` of a surface cell;
//   key           : a corner of an occupied cell (vertex coordinates 0..N).
// Vertices are multiples of 2^-16, so 2*N*2^16*v is an integer and the
// separating-axis test runs on integers (int64 / __int128): no rounding.
// Sets are bitmaps with one 64-bit word per 64 cells along x; dilation and
// the corner expansion are separable word operations.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "host_common.hpp"
#include "host_internal.hpp"

namespace inrf {

namespace {

constexpr int kFrac = 16;  // vertex lattice: multiples of 2^-16

struct Bitmap3 {
    int64_t nx, ny, nz, words;  // words per row
    std::vector<uint64_t> w;
    Bitmap3(int64_t x, int64_t y, int64_t z) : nx(x), ny(y), nz(z), words((x + 63) / 64), w(size_t(words * y * z), 0) {}
    uint64_t* row(int64_t y, int64_t z) { return w.data() + (z * ny + y) * words; }
    const uint64_t* row(int64_t y, int64_t z) const { return w.data() + (z * ny + y) * words; }
};

template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
    if (n <= 0) return;
    threads = int(std::max<int64_t>(1, std::min<int64_t>(threads, n)));
    if (threads == 1) {
        f(int64_t(0), n, 0);
        return;
    }
    std::vector<std::thread> pool;
    std::atomic<int64_t> next{0};
    const int64_t chunk = std::max<int64_t>(1, n / (int64_t(threads) * 8));
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            for (;;) {
                int64_t s = next.fetch_add(chunk);
                if (s >= n) break;
                f(s, std::min(n, s + chunk), t);
            }
        });
    for (auto& th : pool) th.join();
}

inline int64_t iabs(int64_t a) { return a < 0 ? -a : a; }
inline __int128 iabs128(__int128 a) { return a < 0 ? -a : a; }

// Mark the surface cells of one triangle (integer corners in doubled units,
// where a cell spans S = 2^17 and has half-size H = 2^16).
void mark_triangle(const int64_t X[3][3], int64_t N, Bitmap3& S) {
    const int64_t CS = int64_t(1) << (kFrac + 1), H = int64_t(1) << kFrac;
    int64_t lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        int64_t mn = std::min({X[0][k], X[1][k], X[2][k]}), mx = std::max({X[0][k], X[1][k], X[2][k]});
        // cells p with [p*CS, (p+1)*CS] meeting [mn, mx]: ceil(mn/CS)-1 <= p <= floor(mx/CS)
        // (coordinates are >= 0, so integer division floors)
        lo[k] = std::max<int64_t>((mn + CS - 1) / CS - 1, 0);
        hi[k] = std::min<int64_t>(mx / CS, N - 1);
        if (lo[k] > hi[k]) return;
    }
    int64_t f[3][3];
    for (int k = 0; k < 3; ++k) {
        f[0][k] = X[1][k] - X[0][k];
        f[1][k] = X[2][k] - X[1][k];
        f[2][k] = X[0][k] - X[2][k];
    }
    // triangle normal (|component| < 2^60)
    const int64_t n0 = f[0][1] * (-f[2][2]) - f[0][2] * (-f[2][1]);
    const int64_t n1 = f[0][2] * (-f[2][0]) - f[0][0] * (-f[2][2]);
    const int64_t n2 = f[0][0] * (-f[2][1]) - f[0][1] * (-f[2][0]);
    const __int128 rn = __int128(H) * (__int128(iabs(n0)) + iabs(n1) + iabs(n2));
    const __int128 nx0 = __int128(n0) * X[0][0] + __int128(n1) * X[0][1] + __int128(n2) * X[0][2];
    for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int64_t cy = lo[1]; cy <= hi[1]; ++cy) {
            uint64_t* row = S.row(cy, cz);
            for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                const int64_t C[3] = {(2 * cx + 1) * H, (2 * cy + 1) * H, (2 * cz + 1) * H};
                // plane axis: |n.(X0 - C)| <= H * |n|_1
                const __int128 d = nx0 - (__int128(n0) * C[0] + __int128(n1) * C[1] + __int128(n2) * C[2]);
                if (iabs128(d) > rn) continue;
                int64_t w[3][3];
                for (int v = 0; v < 3; ++v)
                    for (int k = 0; k < 3; ++k) w[v][k] = X[v][k] - C[k];
                bool sep = false;
                // nine axes e_ax x f_j: components (a[b1], a[b2]) = (-f[b2], f[b1])
                for (int j = 0; j < 3 && !sep; ++j)
                    for (int ax = 0; ax < 3 && !sep; ++ax) {
                        const int b1 = (ax + 1) % 3, b2 = (ax + 2) % 3;
                        const int64_t a1 = -f[j][b2], a2 = f[j][b1];
                        int64_t pmin = INT64_MAX, pmax = INT64_MIN;
                        for (int v = 0; v < 3; ++v) {
                            const int64_t p = w[v][b1] * a1 + w[v][b2] * a2;
                            pmin = std::min(pmin, p);
                            pmax = std::max(pmax, p);
                        }
                        const int64_t r = H * (iabs(a1) + iabs(a2));
                        sep = pmin > r || pmax < -r;
                    }
                if (sep) continue;
                __atomic_fetch_or(&row[cx >> 6], uint64_t(1) << (cx & 63), __ATOMIC_RELAXED);
            }
        }
}

void dilate_x(Bitmap3& B, int threads) {
    const int64_t W = B.words, nx = B.nx;
    const uint64_t last_mask = (nx & 63) ? ((uint64_t(1) << (nx & 63)) - 1) : ~uint64_t(0);
    parallel_for(B.ny * B.nz, threads, [&](int64_t s, int64_t e, int) {
        std::vector<uint64_t> tmp(W);
        for (int64_t r = s; r < e; ++r) {
            uint64_t* row = B.w.data() + r * W;
            for (int64_t i = 0; i < W; ++i) {
                uint64_t v = row[i] | (row[i] << 1) | (row[i] >> 1);
                if (i > 0) v |= row[i - 1] >> 63;
                if (i + 1 < W) v |= row[i + 1] << 63;
                tmp[i] = v;
            }
            tmp[W - 1] &= last_mask;
            std::memcpy(row, tmp.data(), W * sizeof(uint64_t));
        }
    });
}

void dilate_y(Bitmap3& B, int threads) {
    const int64_t W = B.words;
    parallel_for(B.nz, threads, [&](int64_t s, int64_t e, int) {
        std::vector<uint64_t> prev(W), cur(W);
        for (int64_t z = s; z < e; ++z) {
            std::fill(prev.begin(), prev.end(), 0);
            for (int64_t y = 0; y < B.ny; ++y) {
                uint64_t* row = B.row(y, z);
                std::memcpy(cur.data(), row, W * sizeof(uint64_t));
                const uint64_t* next = (y + 1 < B.ny) ? B.row(y + 1, z) : nullptr;
                for (int64_t i = 0; i < W; ++i) row[i] = cur[i] | prev[i] | (next ? next[i] : 0);
                std::swap(prev, cur);
            }
        }
    });
}

void dilate_z(Bitmap3& B, int threads) {
    const int64_t W = B.words, slice = B.ny * W;
    // rows of a slice are independent: parallel over y
    parallel_for(B.ny, threads, [&](int64_t s, int64_t e, int) {
        std::vector<uint64_t> prev(W), cur(W);
        for (int64_t y = s; y < e; ++y) {
            std::fill(prev.begin(), prev.end(), 0);
            for (int64_t z = 0; z < B.nz; ++z) {
                uint64_t* row = B.row(y, z);
                std::memcpy(cur.data(), row, W * sizeof(uint64_t));
                const uint64_t* next = (z + 1 < B.nz) ? row + slice : nullptr;
                for (int64_t i = 0; i < W; ++i) row[i] = cur[i] | prev[i] | (next ? next[i] : 0);
                std::swap(prev, cur);
            }
        }
    });
}

}  // namespace

std::vector<int64_t> shell_keys(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, int N,
                                int dilate, int threads) {
    require(N >= 1 && N <= 4096, "resolution must be in [1, 4096]");
    require(dilate >= 0 && dilate <= 8, "dilate must be in [0, 8]");
    // integer vertices in doubled units: 2 * N * (v * 2^16)
    std::vector<int64_t> X(size_t(n_verts) * 3);
    for (int64_t i = 0; i < n_verts * 3; ++i) {
        const double v = verts[i];
        require(std::isfinite(v) && v >= 0.0 && v <= 1.0, "vertex coordinates must lie in [0, 1]");
        const double s = v * double(1 << kFrac);
        require(s == std::floor(s), "vertex coordinates must be multiples of 2^-16");
        X[i] = int64_t(s) * 2 * N;
    }
    Bitmap3 S(N, N, N);
    parallel_for(n_tris, threads, [&](int64_t s, int64_t e, int) {
        for (int64_t t = s; t < e; ++t) {
            int64_t T[3][3];
            for (int v = 0; v < 3; ++v) {
                const int64_t id = tris[t * 3 + v];
                for (int k = 0; k < 3; ++k) T[v][k] = X[size_t(id) * 3 + k];
            }
            mark_triangle(T, N, S);
        }
    });
    for (int r = 0; r < dilate; ++r) dilate_x(S, threads);
    for (int r = 0; r < dilate; ++r) dilate_y(S, threads);
    for (int r = 0; r < dilate; ++r) dilate_z(S, threads);
    // corners: vertex v is a key iff a cell in v - {0,1}^3 is occupied
    const int64_t M = int64_t(N) + 1, WK = (M + 63) / 64;
    std::vector<int64_t> counts(size_t(M), 0);
    std::vector<std::vector<int64_t>> per_slice(static_cast<size_t>(M));
    parallel_for(M, threads, [&](int64_t s, int64_t e, int) {
        std::vector<uint64_t> acc(WK);
        for (int64_t vz = s; vz < e; ++vz) {
            std::vector<int64_t>& out = per_slice[size_t(vz)];
            for (int64_t vy = 0; vy < M; ++vy) {
                std::fill(acc.begin(), acc.end(), 0);
                bool any = false;
                for (int64_t cz = vz - 1; cz <= vz; ++cz) {
                    if (cz < 0 || cz >= N) continue;
                    for (int64_t cy = vy - 1; cy <= vy; ++cy) {
                        if (cy < 0 || cy >= N) continue;
                        const uint64_t* row = S.row(cy, cz);
                        for (int64_t i = 0; i < S.words; ++i) {
                            if (!row[i]) continue;
                            any = true;
                            acc[i] |= row[i] | (row[i] << 1);
                            if (i + 1 < WK) acc[i + 1] |= row[i] >> 63;
                        }
                    }
                }
                if (!any) continue;
                const int64_t base = (vz * M + vy) * M;
                for (int64_t i = 0; i < WK; ++i) {
                    uint64_t w = acc[i];
                    while (w) {
                        const int b = __builtin_ctzll(w);
                        w &= w - 1;
                        const int64_t vx = i * 64 + b;
                        if (vx <= N) out.push_back(base + vx);
                    }
                }
            }
        }
    });
    int64_t total = 0;
    for (auto& v : per_slice) total += int64_t(v.size());
    std::vector<int64_t> keys;
    keys.reserve(size_t(total));
    for (auto& v : per_slice) {
        keys.insert(keys.end(), v.begin(), v.end());
        std::vector<int64_t>().swap(v);
    }
    return keys;
}

}  // namespace inrf
