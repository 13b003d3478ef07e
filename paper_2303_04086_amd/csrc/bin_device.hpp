// Closest hit of a camera frame through screen-space bins of the proxy's
// triangles.  Every primary ray of a pinhole camera starts at the camera
// centre, so the triangles a ray can hit are those whose projection covers
// its pixel.  Each frame therefore sorts the triangles into lists per 8x8
// pixel quadrant (the pixels one wave traces): a triangle goes into every
// quadrant its padded screen bounding box touches.  A wave then runs the
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
// goes into a global list that every quadrant tests.  A quadrant whose list
// did not fit the workspace, or every quadrant when the global list
// overflows, walks the BVH instead.
#pragma once

namespace inrf {
namespace dev {

constexpr int kQuad = 8;            // bin side in pixels (one wave's quadrant of a tile)
constexpr int kBinGlobal = 256;     // capacity of the global list
constexpr float kBinPad = 1.0f;     // bounding box widening, pixels
constexpr float kBinFront = 0.05f;  // lambda / |q| of a vertex safely in front (or behind)

struct BinsC {
    float a[9];                // rows of the inverse camera basis: X (0..2), Y (3..5), lambda (6..8)
    float o[3];                // camera centre
    float sjx, sjb, siy, sib;  // pixel column j = X / lambda * sjx + sjb, row i = Y / lambda * siy + sib
    int32_t W, H, QX, QY;      // image and quadrant grid sizes
    int32_t* cnt;              // [QX * QY] entries per quadrant (the fill pass counts them back to 0)
    int32_t* off;              // [QX * QY] exclusive offsets within scan runs
    int32_t* runs;             // scan run carries
    int32_t* total;            // total entries, then the global list: total[1] = its count, total[2 ..] records
    int32_t* entries;          // [E] triangle records, quadrant after quadrant
    int64_t E;
    int32_t clamp;             // the scan adds min(count, clamp) per quadrant, so sums fit 31 bits
    int32_t pad;
};

// Quadrant q's list [s, e) and whether it holds every record of the quadrant:
// its count was not clamped by the scan and the list lies inside [0, E).
__device__ __forceinline__ bool bin_list(const BinsC& b, int q, int64_t& s, int64_t& e) {
    const int nq = b.QX * b.QY;
    s = int64_t(b.off[q]) + b.runs[q / kScanRun];
    e = q + 1 < nq ? int64_t(b.off[q + 1]) + b.runs[(q + 1) / kScanRun] : int64_t(b.total[0]);
    return e - s < b.clamp && e <= b.E;
}

// Quadrant range of triangle record k: 0 = no pixel can hit it, 1 = the
// range [qx0, qx1] x [qy0, qy1], 2 = the global list.
__device__ __forceinline__ int bin_range(const BinsC& b, const BvhTri* __restrict__ tris, int64_t k, int& qx0,
                                         int& qx1, int& qy0, int& qy1) {
#pragma clang fp contract(off)  // the count and fill passes must classify every triangle identically
    const float4* p = reinterpret_cast<const float4*>(tris + k);
    const float4 v[3] = {p[0], p[1], p[2]};
    float jlo = INFINITY, jhi = -INFINITY, ilo = INFINITY, ihi = -INFINITY;
    int front = 0, behind = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float qx = v[c].x - b.o[0], qy = v[c].y - b.o[1], qz = v[c].z - b.o[2];
        const float X = b.a[0] * qx + b.a[1] * qy + b.a[2] * qz;
        const float Y = b.a[3] * qx + b.a[4] * qy + b.a[5] * qz;
        const float lam = b.a[6] * qx + b.a[7] * qy + b.a[8] * qz;
        const float lim = kBinFront * sqrtf(qx * qx + qy * qy + qz * qz);
        front += lam >= lim && lim > 0.f;
        behind += lam <= -lim && lim > 0.f;
        const float il = 1.f / lam;
        const float j = X * il * b.sjx + b.sjb, i = Y * il * b.siy + b.sib;
        jlo = fminf(jlo, j);
        jhi = fmaxf(jhi, j);
        ilo = fminf(ilo, i);
        ihi = fmaxf(ihi, i);
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

// Clears the quadrant counts and the global list (one thread per quadrant).
__global__ void k_bin_clear(BinsC b) {
    const int q = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < b.QX * b.QY) b.cnt[q] = 0;
    if (q == 0) b.total[1] = 0;
}

// Count pass (FILL = false) and fill pass (FILL = true), one thread per
// triangle record.  The fill pass counts each quadrant back down to zero and
// stores records only in quadrants whose whole list was kept (bin_list).
template <bool FILL>
__global__ __launch_bounds__(256) void k_bin(BinsC b, const BvhTri* __restrict__ tris, int64_t n_tris) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n_tris) return;
    int qx0, qx1, qy0, qy1;
    const int r = bin_range(b, tris, k, qx0, qx1, qy0, qy1);
    if (r == 0) return;
    if (r == 2) {
        if (!FILL) {
            const int g = atomicAdd(b.total + 1, 1);
            if (g < kBinGlobal) b.total[2 + g] = int32_t(k);
        }
        return;
    }
    for (int qy = qy0; qy <= qy1; ++qy)
        for (int qx = qx0; qx <= qx1; ++qx) {
            const int q = qy * b.QX + qx;
            if (!FILL) {
                atomicAdd(b.cnt + q, 1);
            } else {
                int64_t s, e;
                const bool whole = bin_list(b, q, s, e);
                const int slot = atomicSub(b.cnt + q, 1) - 1;
                if (whole && slot >= 0 && s + slot < e) b.entries[s + slot] = int32_t(k);
            }
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

// Records [s, e) of a quadrant's list against the wave's rays, with the
// axes of the watertight test given by Ax.  Four records, then their four
// triangles, are requested before any test waits on them.
template <class Ax>
__device__ __forceinline__ void bin_walk(const RayPre& R, const Ax& ax, const int32_t* __restrict__ ent,
                                         const float4* __restrict__ tv, int s, int e, bool active, float& best_t,
                                         int32_t& best_i) {
    for (int k = s; k < e; k += 4) {
        int32_t r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = __builtin_amdgcn_readfirstlane(ent[k + u < e ? k + u : k]);
        float4 v[12];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) v[3 * u + c] = tv[3 * int64_t(r[u]) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
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
    int64_t s64, e64;
    const bool whole = bin_list(b, q, s64, e64);
    const int g = __builtin_amdgcn_readfirstlane(b.total[1]);
    if (!__builtin_amdgcn_readfirstlane(int(whole)) || g > kBinGlobal) {
        closest_hit_packet(m, R, active, wst, best_t, best_i);
        return;
    }
    // lists lie in [0, E) with E < 2^31 records, so 32-bit bounds suffice
    const int s = __builtin_amdgcn_readfirstlane(int(s64)), e = __builtin_amdgcn_readfirstlane(int(e64));
    const int32_t* __restrict__ ent = b.entries;
    const float4* __restrict__ tv = reinterpret_cast<const float4*>(m.tris);
    // permutation id: kz (0..2) and whether kx, ky were swapped
    const int perm = 2 * R.kz + (R.kx == (R.kz + 1) % 3 ? 0 : 1);
    const int lead = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(active)));
    const int pu = __builtin_amdgcn_readlane(perm, lead);
    if (__ballot(active && perm != pu) == 0) {
        switch (pu) {
            case 0: bin_walk(R, AxisC<1, 2, 0>(), ent, tv, s, e, active, best_t, best_i); break;
            case 1: bin_walk(R, AxisC<2, 1, 0>(), ent, tv, s, e, active, best_t, best_i); break;
            case 2: bin_walk(R, AxisC<2, 0, 1>(), ent, tv, s, e, active, best_t, best_i); break;
            case 3: bin_walk(R, AxisC<0, 2, 1>(), ent, tv, s, e, active, best_t, best_i); break;
            case 4: bin_walk(R, AxisC<0, 1, 2>(), ent, tv, s, e, active, best_t, best_i); break;
            default: bin_walk(R, AxisC<1, 0, 2>(), ent, tv, s, e, active, best_t, best_i); break;
        }
    } else {
        bin_walk(R, AxisR{R.kx, R.ky, R.kz}, ent, tv, s, e, active, best_t, best_i);
    }
    for (int k = 0; k < g; ++k) bin_test(R, m.tris, __builtin_amdgcn_readfirstlane(b.total[2 + k]), active, best_t, best_i);
}

}  // namespace dev
}  // namespace inrf
