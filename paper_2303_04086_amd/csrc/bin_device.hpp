// Closest hit of a camera frame through screen-space bins of the proxy's
// triangles.  Every primary ray of a pinhole camera starts at the camera
// centre, so the triangles a ray can hit are those whose projection covers
// its pixel.  Each frame therefore sorts the triangles into lists per 8x8
// pixel quadrant (the pixels one wave traces): a triangle goes into every
// quadrant its padded screen bounding box touches, less those the edge test
// below rules out.  A wave then runs the
// same watertight test on the same FP32 rays against its quadrant's list
// instead of walking the BVH, and keeps the nearest hit (ties to the lower
// triangle index) -- the result the BVH gives, since every triangle a ray
// can hit is in its quadrant's list.  Included by render.hip after the
// BVH traversal.
//
// Conservative projection.  The camera maps a world point q (relative to
// the centre) to coefficients (X, Y, lambda) = A q, A the inverse of the
// basis [right up forward]; the pixel ray through (s_x, s_y) is the
// direction of (s_x, s_y, 1) in that basis, so the point lies on the ray of
// s_x = X / lambda, s_y = Y / lambda, and a ray at t > 0 only meets points
// with lambda > 0.  A triangle whose three vertices all have lambda >= 0.05
// |q| (within 87 degrees of the view axis) projects to the triangle of the
// projected vertices; its bounding box, widened by one pixel, covers every
// pixel whose FP32 ray the FP32 test can report a hit for (the rounding of
// the projection and of the ray directions is far below a pixel).  A
// triangle whose vertices all have lambda <= -0.05 |q| lies behind the
// camera and is never hit.  Any other triangle (crossing the camera plane)
// goes into a global list that every quadrant tests.
//
// Edge test.  Within its bounding box, a triangle skips every quadrant whose
// pixel centres all lie more than kBinPad from the projected triangle: some
// edge line, moved out by kBinPad, has them all on its outer side (the
// padded triangle lies inside the three moved half-planes).  A sliver whose
// projected area is too small for the rounding of its vertices to leave the
// winding certain keeps its whole box.
//
// Lists.  Each quadrant has kBinCap slots, filled in one pass (k_bin):
// facing triangles from the start up, the others from the end down, each
// side counted by its own atomic counter, which keeps counting past the
// capacity.  The counts are therefore exact, and a quadrant whose two counts
// add up to more than kBinCap (its two sides then overlap) gets a list of
// exactly that size in a shared spill area (k_spill_alloc), filled by a
// second pass over the triangles (k_bin_spill) that does nothing when no
// quadrant overflowed.  A quadrant whose list does not fit the spill area,
// or every quadrant when the global list overflows, walks the BVH instead.
//
// Depth skip.  A quadrant's list holds the triangles facing the camera
// first, then the others, each with a lower bound on the distance t at which
// any camera ray can meet it: a point p of the triangle lies at t = |p - o|
// >= lambda(p) / |a_f| >= min_i lambda(v_i) / |a_f| (a_f the lambda row of
// A, unit rays), widened by 1e-4 for the FP32 rounding of lambda and of the
// test's t.  After the facing triangles, a wave skips every further
// triangle whose bound exceeds the largest closest hit among its rays: such
// a triangle can only be met farther than every ray's hit, so skipping it
// changes nothing.  On a closed proxy seen from outside this skips most of
// the triangles facing away.
#pragma once

namespace inrf {
namespace dev {

constexpr int kQuad = 8;            // bin side in pixels (one wave's quadrant of a tile)
constexpr int kBinCap = 256;        // slots of a quadrant's list
constexpr int kBinGlobal = 256;     // capacity of the global list
constexpr float kBinPad = 1.0f;     // bounding box widening, pixels
constexpr float kBinFront = 0.05f;  // lambda / |q| of a vertex safely in front (or behind)
constexpr float kBinSliver = 0.05f; // |twice the projected area| / perimeter below which the edge test is off

struct BinsC {
    float a[9];                // rows of the inverse camera basis: X (0..2), Y (3..5), lambda (6..8)
    float o[3];                // camera centre
    float sjx, sjb, siy, sib;  // pixel column j = X / lambda * sjx + sjb, row i = Y / lambda * siy + sib
    int32_t W, H, QX, QY;      // image and quadrant grid sizes
    int32_t* cnt;              // [QX * QY] entries of triangles not facing the camera, per quadrant
    int32_t* fcnt;             // [QX * QY] entries of facing triangles, per quadrant
    int32_t* total;            // the global list: total[1] = its count, total[2 ..] records
    int2* entries;             // [QX * QY][kBinCap] (triangle record, bits of its distance bound)
    int32_t* base;             // [QX * QY] start of an overflowing quadrant's spill list, -1: none
    int32_t* sfcnt;            // [QX * QY] spill fill counters: facing entries
    int32_t* scnt;             // [QX * QY] spill fill counters: the others
    unsigned long long* top;   // spill entries handed out
    int2* spill;               // [spill_cap] spill lists
    int32_t spill_cap;
    float tscale;              // (1 - 1e-4) / |a_f|: distance bound per unit of lambda
};

// Quadrant range of triangle record k: 0 = no pixel can hit it, 1 = the
// range [qx0, qx1] x [qy0, qy1], 2 = the global list.
__device__ __forceinline__ int bin_range(const BinsC& b, const BvhTri* __restrict__ tris, int64_t k, int& qx0,
                                         int& qx1, int& qy0, int& qy1, bool* facing = nullptr,
                                         float* lam_min = nullptr, float* pj = nullptr, float* pi = nullptr) {
#pragma clang fp contract(off)  // k_bin and k_bin_spill must classify every triangle identically
    const float4* p = reinterpret_cast<const float4*>(tris + k);
    const float4 v[3] = {p[0], p[1], p[2]};
    float jlo = INFINITY, jhi = -INFINITY, ilo = INFINITY, ihi = -INFINITY, lmin = INFINITY;
    int front = 0, behind = 0;
    float qv[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float qx = v[c].x - b.o[0], qy = v[c].y - b.o[1], qz = v[c].z - b.o[2];
        qv[c][0] = qx;
        qv[c][1] = qy;
        qv[c][2] = qz;
        const float X = b.a[0] * qx + b.a[1] * qy + b.a[2] * qz;
        const float Y = b.a[3] * qx + b.a[4] * qy + b.a[5] * qz;
        const float lam = b.a[6] * qx + b.a[7] * qy + b.a[8] * qz;
        const float lim = kBinFront * sqrtf(qx * qx + qy * qy + qz * qz);
        front += lam >= lim && lim > 0.f;
        behind += lam <= -lim && lim > 0.f;
        const float il = 1.f / lam;
        const float j = X * il * b.sjx + b.sjb, i = Y * il * b.siy + b.sib;
        if (pj) pj[c] = j;
        if (pi) pi[c] = i;
        jlo = fminf(jlo, j);
        jhi = fmaxf(jhi, j);
        ilo = fminf(ilo, i);
        ihi = fmaxf(ihi, i);
        lmin = fminf(lmin, lam);
    }
    if (lam_min) *lam_min = lmin;
    if (facing) {  // normal (v1 - v0) x (v2 - v0) against the view from the centre
        const float e1[3] = {qv[1][0] - qv[0][0], qv[1][1] - qv[0][1], qv[1][2] - qv[0][2]};
        const float e2[3] = {qv[2][0] - qv[0][0], qv[2][1] - qv[0][1], qv[2][2] - qv[0][2]};
        const float n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        *facing = n[0] * qv[0][0] + n[1] * qv[0][1] + n[2] * qv[0][2] <= 0.f;
    }
    if (behind == 3) return 0;
    if (front != 3) return 2;
    jlo = floorf(jlo - kBinPad);
    jhi = ceilf(jhi + kBinPad);
    ilo = floorf(ilo - kBinPad);
    ihi = ceilf(ihi + kBinPad);
    if (!(jhi >= 0.f && ihi >= 0.f && jlo <= float(b.W - 1) && ilo <= float(b.H - 1))) return 0;
    qx0 = int(fmaxf(jlo, 0.f)) / kQuad;
    qx1 = int(fminf(jhi, float(b.W - 1))) / kQuad;
    qy0 = int(fmaxf(ilo, 0.f)) / kQuad;
    qy1 = int(fminf(ihi, float(b.H - 1))) / kQuad;
    return 1;
}

// Edge functions of a projected triangle (column j, row i of its vertices),
// each moved out by kBinPad and oriented so that e(x, y) = a x + b y + c >= 0
// holds on the padded triangle's side.
struct BinEdges {
    float a[3], b[3], c[3];
    bool use;  // false: a sliver, test the whole bounding box
};

__device__ __forceinline__ BinEdges bin_edges(const float* pj, const float* pi) {
#pragma clang fp contract(off)  // k_bin and k_bin_spill must agree on every quadrant
    BinEdges E;
    const float A = (pj[1] - pj[0]) * (pi[2] - pi[0]) - (pj[2] - pj[0]) * (pi[1] - pi[0]);
    const float s = A > 0.f ? 1.f : -1.f;
    float per = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = k == 2 ? 0 : k + 1;
        const float ej = pj[k1] - pj[k], ei = pi[k1] - pi[k];
        const float len = sqrtf(ej * ej + ei * ei);
        per += len;
        E.a[k] = -s * ei;
        E.b[k] = s * ej;
        E.c[k] = s * (ei * pj[k] - ej * pi[k]) + kBinPad * len;
    }
    E.use = fabsf(A) > kBinSliver * per && isfinite(A) && isfinite(per);
    return E;
}

// Whether quadrant (qx, qy) has a pixel centre on the inner side of all
// three moved edges: each edge is tested at the corner of the quadrant's
// pixel-centre square where it is largest.
__device__ __forceinline__ bool bin_touches(const BinEdges& E, int qx, int qy) {
#pragma clang fp contract(off)
    if (!E.use) return true;
    const float x0 = float(kQuad * qx), y0 = float(kQuad * qy);
    const float x1 = x0 + float(kQuad - 1), y1 = y0 + float(kQuad - 1);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (E.a[k] * (E.a[k] > 0.f ? x1 : x0) + E.b[k] * (E.b[k] > 0.f ? y1 : y0) + E.c[k] < 0.f) return false;
    return true;
}

// Clears the quadrant counts, the global list and the spill area's
// counters (one thread per quadrant).
__global__ void k_bin_clear(BinsC b) {
    const int q = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < b.QX * b.QY) {
        b.cnt[q] = 0;
        b.fcnt[q] = 0;
        b.scnt[q] = 0;
        b.sfcnt[q] = 0;
    }
    if (q == 0) {
        b.total[1] = 0;
        *b.top = 0;
    }
}

// One thread per triangle record: the triangle's entry goes into every
// quadrant of its range that the edge test keeps, facing triangles from the start of the list up,
// the others from the end down; slots past kBinCap are counted but not
// written.
__global__ __launch_bounds__(256) void k_bin(BinsC b, const BvhTri* __restrict__ tris, int64_t n_tris) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_tris) return;
    int qx0, qx1, qy0, qy1;
    bool facing = true;
    float lmin = 0.f, pj[3], pi[3];
    const int r = bin_range(b, tris, k, qx0, qx1, qy0, qy1, &facing, &lmin, pj, pi);
    const int2 rec = make_int2(int32_t(k), __float_as_int(lmin * b.tscale));
    if (r == 0) return;
    if (r == 2) {
        const int g = atomicAdd(b.total + 1, 1);
        if (g < kBinGlobal) b.total[2 + g] = int32_t(k);
        return;
    }
    const BinEdges E = bin_edges(pj, pi);
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            if (!bin_touches(E, qx, qy)) continue;
            const int64_t q = int64_t(qy) * b.QX + qx;
            const int slot = atomicAdd((facing ? b.fcnt : b.cnt) + q, 1);
            if (slot < kBinCap) b.entries[q * kBinCap + (facing ? slot : kBinCap - 1 - slot)] = rec;
        }
}

// One thread per quadrant: a quadrant whose list overflowed gets a spill
// list of its exact size, or -1 when the spill area has no room for it.
__global__ void k_spill_alloc(BinsC b) {
    const int q = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= b.QX * b.QY) return;
    const int64_t n = int64_t(b.fcnt[q]) + b.cnt[q];
    int32_t at = -1;
    if (n > kBinCap) {
        const unsigned long long s = atomicAdd(b.top, (unsigned long long)n);
        if (s + (unsigned long long)n <= (unsigned long long)b.spill_cap) at = int32_t(s);
    }
    b.base[q] = at;
}

// The fill pass again for the quadrants that have a spill list: facing
// entries from the start of the list up, the others from its end down.
// Returns at once when no quadrant overflowed.
__global__ __launch_bounds__(256) void k_bin_spill(BinsC b, const BvhTri* __restrict__ tris, int64_t n_tris) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_tris || *b.top == 0) return;
    int qx0, qx1, qy0, qy1;
    bool facing = true;
    float lmin = 0.f, pj[3], pi[3];
    if (bin_range(b, tris, k, qx0, qx1, qy0, qy1, &facing, &lmin, pj, pi) != 1) return;
    const int2 rec = make_int2(int32_t(k), __float_as_int(lmin * b.tscale));
    const BinEdges E = bin_edges(pj, pi);
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            if (!bin_touches(E, qx, qy)) continue;
            const int64_t q = int64_t(qy) * b.QX + qx;
            const int32_t at = b.base[q];
            if (at < 0) continue;
            const int nf = b.fcnt[q], nb = b.cnt[q];
            const int slot = atomicAdd((facing ? b.sfcnt : b.scnt) + q, 1);
            if (slot < (facing ? nf : nb)) b.spill[int64_t(at) + (facing ? slot : nf + nb - 1 - slot)] = rec;
        }
}

// One triangle record against a lane's ray: keep the nearer hit, equal
// distances to the lower triangle index (the rule of the BVH leaves).
__device__ __forceinline__ void bin_test(const RayPre& R, const BvhTri* __restrict__ tris, int32_t rec, bool active,
                                         float& best_t, int32_t& best_i) {
    const float4* p = reinterpret_cast<const float4*>(tris + rec);
    const float4 a = p[0], b = p[1], c = p[2];
    const float t = hit_triangle(R, make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z), make_float3(c.x, c.y, c.z));
    const int32_t idx = __float_as_int(a.w);
    const bool better = active && (t < best_t || (t == best_t && t != INFINITY && idx < best_i));
    best_t = better ? t : best_t;
    best_i = better ? idx : best_i;
}

// Largest closest-hit distance over the wave's active rays (+inf if one of
// them has no hit yet).
__device__ __forceinline__ float wave_max_best(bool active, float best_t) {
    float m = active ? best_t : -INFINITY;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m)));  // the same in every lane
}

// Entries [s, e) of a quadrant's list against the wave's rays, with the axes
// of the watertight test given by Ax, four at a time: the four records, then
// their triangles, are requested before any test waits on them (past e, the
// first of the four is requested again but not tested).  With SKIP, entries
// whose distance bound exceeds tmax are not tested.
template <bool SKIP, class Ax>
__device__ __forceinline__ void bin_walk(const RayPre& R, const Ax& ax, const int2* __restrict__ ent,
                                         const float4* __restrict__ tv, int s, int e, float tmax, bool active,
                                         float& best_t, int32_t& best_i) {
    for (int k = s; k < e; k += 4) {
        int32_t r[4];
        bool go[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int2 en = ent[k + u < e ? k + u : k];
            r[u] = __builtin_amdgcn_readfirstlane(en.x);
            go[u] = k + u < e && (!SKIP || !(__int_as_float(__builtin_amdgcn_readfirstlane(en.y)) > tmax));
        }
        if (SKIP && !(go[0] || go[1] || go[2] || go[3])) continue;
        float4 v[12];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[3 * u + c] = tv[3 * int64_t(r[u]) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!go[u]) continue;  // wave-uniform
            const float t = hit_triangle_ax(R, ax, make_float3(v[3 * u].x, v[3 * u].y, v[3 * u].z),
                                            make_float3(v[3 * u + 1].x, v[3 * u + 1].y, v[3 * u + 1].z),
                                            make_float3(v[3 * u + 2].x, v[3 * u + 2].y, v[3 * u + 2].z));
            const int32_t idx = __float_as_int(v[3 * u].w);
            const bool better = active && (t < best_t || (t == best_t && t != INFINITY && idx < best_i));
            best_t = better ? t : best_t;
            best_i = better ? idx : best_i;
        }
    }
}

// The facing part [s, f) of a quadrant's list, then the rest [s2, e) with
// the depth skip (entry indices relative to ent).
template <class Ax>
__device__ __forceinline__ void bin_walk_list(const RayPre& R, const Ax& ax, const int2* __restrict__ ent,
                                              const float4* __restrict__ tv, int s, int f, int s2, int e, bool active,
                                              float& best_t, int32_t& best_i) {
    bin_walk<false>(R, ax, ent, tv, s, f, INFINITY, active, best_t, best_i);
    if (s2 < e) bin_walk<true>(R, ax, ent, tv, s2, e, wave_max_best(active, best_t), active, best_t, best_i);
}

// Closest hit of a wave of camera rays in quadrant (qx, qy) through its
// list and the global list; the BVH packet walk where a list is missing.
// The quadrant, its list bounds and every record are wave-uniform (read into
// scalar registers), so the list walk is a scalar loop whose loads go
// through the scalar cache.  Neighbouring camera rays almost always share
// the watertight test's axis permutation; a wave whose active rays all do
// runs the test with that permutation fixed at compile time.
template <class B>
__device__ void closest_hit_binned(const B& m, const BinsC& b, int qx, int qy, const RayPre& R, bool active, int* wst,
                                   float& best_t, int32_t& best_i) {
    if (m.n_tris == 0 || __ballot(active) == 0) return;
    const int q = __builtin_amdgcn_readfirstlane(qy * b.QX + qx);
    const int nf = __builtin_amdgcn_readfirstlane(b.fcnt[q]), nb = __builtin_amdgcn_readfirstlane(b.cnt[q]);
    const int g = __builtin_amdgcn_readfirstlane(b.total[1]);
    const bool fits = int64_t(nf) + nb <= kBinCap;
    const int at = fits ? 0 : __builtin_amdgcn_readfirstlane(b.base[q]);
    if (at < 0 || g > kBinGlobal) {  // a spill list that did not fit, or a full global list
        closest_hit_packet(m, R, active, wst, best_t, best_i);
        return;
    }
    // the global list first: its triangles have no distance bound
    for (int k = 0; k < g; ++k) bin_test(R, m.tris, __builtin_amdgcn_readfirstlane(b.total[2 + k]), active, best_t, best_i);
    // facing entries [0, nf) of the quadrant's slots and the others
    // [kBinCap - nb, kBinCap), or the spill list [0, nf) and [nf, nf + nb)
    const int s = 0, f = nf, s2 = fits ? kBinCap - nb : nf, e = fits ? kBinCap : nf + nb;
    const int2* __restrict__ ent = fits ? b.entries + int64_t(q) * kBinCap : b.spill + at;
    const float4* __restrict__ tv = reinterpret_cast<const float4*>(m.tris);
    // permutation id: kz (0..2) and whether kx, ky were swapped
    const int perm = 2 * R.kz + (R.kx == (R.kz + 1) % 3 ? 0 : 1);
    const int lead = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(active)));
    const int pu = __builtin_amdgcn_readlane(perm, lead);
    if (__ballot(active && perm != pu) == 0) {
        switch (pu) {
            case 0: bin_walk_list(R, AxisC<1, 2, 0>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
            case 1: bin_walk_list(R, AxisC<2, 1, 0>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
            case 2: bin_walk_list(R, AxisC<2, 0, 1>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
            case 3: bin_walk_list(R, AxisC<0, 2, 1>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
            case 4: bin_walk_list(R, AxisC<0, 1, 2>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
            default: bin_walk_list(R, AxisC<1, 0, 2>(), ent, tv, s, f, s2, e, active, best_t, best_i); break;
        }
    } else {
        bin_walk_list(R, AxisR{R.kx, R.ky, R.kz}, ent, tv, s, f, s2, e, active, best_t, best_i);
    }
}

}  // namespace dev
}  // namespace inrf
