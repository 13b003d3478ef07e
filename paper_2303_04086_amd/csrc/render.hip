// Device entry points of libinrf: closest-hit trace, position encoding, the
// network alone, and the fused per-ray path (inrf_render / inrf_forward).
//
// A camera frame is nine launches on the caller's stream:
//   k_bin_clear, k_bin, k_spill_alloc, k_bin_spill  sort the proxy's
//             triangles into lists per 8x8-pixel quadrant of the frame
//             (bin_device.hpp);
//   k_trace   one ray per lane, tiles in strip order: generate (camera) or
//             load (batch) the ray, closest hit with a watertight triangle
//             test against the wave's quadrant list (camera; the BVH where a
//             list is missing) or through the BVH (batch), write depth /
//             triangle / zero colour for misses, and write the hit records
//             (hit point, unit direction, output index) of each tile in lane
//             order;
//   k_scan_local, k_scan_runs, k_compact  pack the records into one list in
//             tile order (deterministic) and count them;
//   k_shade   persistent waves over the packed hits: multi-level PSH gather
//             with trilinear blend, SH16 of the direction, the MLP on matrix
//             cores, sigmoid, colour write.
// Each ray's colour depends only on that ray; the packed order fixes which
// rays share a wave (it matters only to sums over rays, e.g. gradients).
// The same kernels serve batches of cameras (inrf_render_batch), ray batches
// (inrf_forward), scenes of several objects (scene_device.hpp) and the
// gradient (backward_device.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bvh_layout.hpp"
#include "device_common.hpp"
#include "host_common.hpp"
#include "inrf.h"
#include "mlp_device.hpp"

namespace inrf {
namespace dev {

constexpr int kTile = 16;      // camera tiles of 16x16 pixels
constexpr int kThreads = 256;  // 4 waves
// prefix sums: workgroup size, and counts each k_scan_local workgroup sums
constexpr int kScanThreads = 1024, kScanRun = 2 * kScanThreads;

struct alignas(16) HitRec {
    float x, y, z;
    int32_t out;  // output (pixel) index
    float dx, dy, dz;
    int32_t pad;
};

// The hit record of a single camera's frame: the shading kernel derives the
// direction from the pixel again (camera_dir, unit_of), so the record is
// half the size of a HitRec.
struct alignas(16) CamHit {
    float x, y, z;
    int32_t out;  // output (pixel) index
};

struct CamC {
    float o[3], r[3], u[3], f[3];
    float tan_y, tan_x;  // tan(fov_y/2) and tan(fov_y/2)*W/H
    int32_t W, H, tiles_x;
    int32_t tile0;       // first tile of this camera in a batch of cameras
    int64_t pix0;        // first output pixel of this camera in a batch
};

// Order in which a frame's tiles are traced, and so in which their hits are
// packed and shaded: strips of kStrip tile rows, each strip column after
// column (top to bottom inside a column).  Rays in flight together then
// cover a compact patch of the image rather than a band of whole rows, so
// the corners that neighbouring tiles share (above and below as well as
// left and right) are read while they are still cached.
constexpr int kStrip = 8;

__host__ __device__ __forceinline__ void tile_at(int t, int tiles_x, int tiles_y, int& tx, int& ty) {
    const int strip = t / (kStrip * tiles_x);
    const int rows = min(kStrip, tiles_y - strip * kStrip);
    const int r = t - strip * kStrip * tiles_x;
    tx = r / rows;
    ty = strip * kStrip + r % rows;
}

// Unit direction of the ray through the centre of pixel (row, col):
// normalize(f + s_x r + s_y u) with s_x = (2(col + 1/2)/W - 1) tan_x and
// s_y = (1 - 2(row + 1/2)/H) tan_y.  Every kernel that generates camera
// rays (and inrf_camera_rays) calls this one function, so their rays are
// bit-identical.
__device__ __forceinline__ float3 camera_dir(const CamC& cam, int row, int col) {
#pragma clang fp contract(off)  // the same rounding in every kernel that inlines it
    const float sx = ((2.f * (float(col) + 0.5f)) / float(cam.W) - 1.f) * cam.tan_x;
    const float sy = (1.f - (2.f * (float(row) + 0.5f)) / float(cam.H)) * cam.tan_y;
    const float3 v = make_float3(cam.f[0] + sx * cam.r[0] + sy * cam.u[0], cam.f[1] + sx * cam.r[1] + sy * cam.u[1],
                                 cam.f[2] + sx * cam.r[2] + sy * cam.u[2]);
    const float inv = 1.f / sqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
    return make_float3(v.x * inv, v.y * inv, v.z * inv);
}

// d / |d|, the direction a hit record holds (the trace and the shading of
// compact camera records both take it from here).
__device__ __forceinline__ float3 unit_of(float3 d) {
#pragma clang fp contract(off)
    const float inv = 1.f / sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
    return make_float3(d.x * inv, d.y * inv, d.z * inv);
}

// Cameras traced by one launch: tiles of camera j are [c[j].tile0, c[j+1].tile0).
constexpr int kMaxCameras = INRF_MAX_CAMERAS;
template <int NCAM>
struct CamSet {
    int32_t n, pad;
    CamC c[NCAM];
};

struct TraceArgs {
    const float* ray_o;  // batch mode
    const float* ray_d;
    int64_t n;
    float* rgba;    // nullable
    float* depth;   // nullable
    int32_t* tri;   // nullable
    void* tmp;      // nullable: no records (trace only); else hit records of workgroup b at blk[b].y
                    // (CamHit for a single camera's frame, else HitRec)
    int2* blk;      // per workgroup: (hit count, first record index in tmp)
};

// ------------------------------------------------------------- tracing ----

__device__ __forceinline__ float comp(const float3& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

struct RayPre {
    float3 o, d, inv;
    int kx, ky, kz;
    float Sx, Sy, Sz;
};

__device__ __forceinline__ RayPre ray_setup(float3 o, float3 d) {
    RayPre R;
    R.o = o;
    R.d = d;
    // slab reciprocals: a zero component becomes +-1e-30 so that a ray lying
    // in a slab's boundary plane gives 0 * 1e30 = 0 instead of 0 * inf = NaN
    const float tiny = 1e-30f;
    R.inv = make_float3(__builtin_amdgcn_rcpf(fabsf(d.x) < tiny ? copysignf(tiny, d.x) : d.x),
                        __builtin_amdgcn_rcpf(fabsf(d.y) < tiny ? copysignf(tiny, d.y) : d.y),
                        __builtin_amdgcn_rcpf(fabsf(d.z) < tiny ? copysignf(tiny, d.z) : d.z));
    const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    if (ay > ax) kz = 1;
    if (az > fmaxf(ax, ay)) kz = 2;
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (comp(d, kz) < 0.f) {
        const int t = kx;
        kx = ky;
        ky = t;
    }
    R.kx = kx;
    R.ky = ky;
    R.kz = kz;
    const float rz = __builtin_amdgcn_rcpf(comp(d, kz));  // the shear only needs to be the same for every triangle
    R.Sx = comp(d, kx) * rz;
    R.Sy = comp(d, ky) * rz;
    R.Sz = rz;
    return R;
}

// Component of v along axis k of the ray's permutation: a run-time axis
// (AxisR: the ray's own kx, ky, kz) or compile-time axes (AxisC, for a wave
// whose rays all share one permutation).  Both select the same value, so
// the test below is bit-identical either way.
struct AxisR {
    int kx, ky, kz;
    __device__ float x(const float3& v) const { return comp(v, kx); }
    __device__ float y(const float3& v) const { return comp(v, ky); }
    __device__ float z(const float3& v) const { return comp(v, kz); }
};
template <int KX, int KY, int KZ>
struct AxisC {
    __device__ static float pick(const float3& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
    __device__ float x(const float3& v) const { return pick(v, KX); }
    __device__ float y(const float3& v) const { return pick(v, KY); }
    __device__ float z(const float3& v) const { return pick(v, KZ); }
};

// Watertight ray/triangle test of Woop, Benthin and Wald (JCGT 2013),
// two-sided.  Returns t > 0 of the hit or +inf.  Products are not fused so
// that an edge shared by two triangles gets exactly opposite edge values.
template <class Ax>
__device__ __forceinline__ float hit_triangle_ax(const RayPre& R, const Ax& ax, const float3 v0, const float3 v1,
                                                 const float3 v2) {
#pragma clang fp contract(off)
    const float3 A = make_float3(v0.x - R.o.x, v0.y - R.o.y, v0.z - R.o.z);
    const float3 B = make_float3(v1.x - R.o.x, v1.y - R.o.y, v1.z - R.o.z);
    const float3 C = make_float3(v2.x - R.o.x, v2.y - R.o.y, v2.z - R.o.z);
    const float Akz = ax.z(A), Bkz = ax.z(B), Ckz = ax.z(C);
    const float Ax_ = ax.x(A) - R.Sx * Akz, Ay = ax.y(A) - R.Sy * Akz;
    const float Bx = ax.x(B) - R.Sx * Bkz, By = ax.y(B) - R.Sy * Bkz;
    const float Cx = ax.x(C) - R.Sx * Ckz, Cy = ax.y(C) - R.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax_ * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax_;
    if (U == 0.f || V == 0.f || W == 0.f) {  // rare: redo the edge tests exactly
        U = float(double(Cx) * double(By) - double(Cy) * double(Bx));
        V = float(double(Ax_) * double(Cy) - double(Ay) * double(Cx));
        W = float(double(Bx) * double(Ay) - double(By) * double(Ax_));
    }
    // the rest is select-based: no divergent branches inside a packet
    const bool outside = (U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f);
    const float det = U + V + W;
    const float Az = R.Sz * Akz, Bz = R.Sz * Bkz, Cz = R.Sz * Ckz;
    const float T0 = U * Az + V * Bz + W * Cz;
    const float T = det < 0.f ? -T0 : T0;
    const bool ok = !outside && det != 0.f && T > 0.f;
    return ok ? T * __builtin_amdgcn_rcpf(fabsf(det)) : INFINITY;
}

__device__ __forceinline__ float hit_triangle(const RayPre& R, const float3 v0, const float3 v1, const float3 v2) {
    return hit_triangle_ax(R, AxisR{R.kx, R.ky, R.kz}, v0, v1, v2);
}

// Slab test of one child box for t in [0, tmax]; conservative so that
// rounding never rejects a box a ray touches: each slab distance
// (l - o) * rcp(d) carries a relative error below 2^-22 (one rounding of the
// difference, the reciprocal's 1 ulp, one rounding of the product), so
// comparing t_near <= t_far * (1 + 2^-20) is safe (cf. Ize 2013).
__device__ __forceinline__ bool hit_box(const RayPre& R, float lx, float ly, float lz, float hx, float hy, float hz,
                                        float tmax, float& tnear) {
    const float t0x = (lx - R.o.x) * R.inv.x, t1x = (hx - R.o.x) * R.inv.x;
    const float t0y = (ly - R.o.y) * R.inv.y, t1y = (hy - R.o.y) * R.inv.y;
    const float t0z = (lz - R.o.z) * R.inv.z, t1z = (hz - R.o.z) * R.inv.z;
    const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.f));
    const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tnear = tn;
    return tn <= tf * 1.00000095f;
}

__device__ __forceinline__ void leaf(const RayPre& R, const BvhTri* __restrict__ tris, int32_t ref, float& best_t,
                                     int32_t& best_i, bool active = true) {
    const int32_t code = ~ref;
    const int32_t first = code >> 3, count = code & 7;
    for (int32_t k = 0; k < count; ++k) {
        const float4* p = reinterpret_cast<const float4*>(tris + first + k);
        const float4 a = p[0], b = p[1], c = p[2];
        const float t = hit_triangle(R, make_float3(a.x, a.y, a.z), make_float3(b.x, b.y, b.z),
                                     make_float3(c.x, c.y, c.z));
        const int32_t idx = __float_as_int(a.w);
        const bool better = active && (t < best_t || (t == best_t && t != INFINITY && idx < best_i));
        best_t = better ? t : best_t;
        best_i = better ? idx : best_i;
    }
}

// Closest hit through the four-wide BVH.  At a node, hit leaves are
// intersected at once; of the hit interior children the nearest (by entry
// distance) is visited next and the others are pushed farthest first.
// `stack` is this lane's column of an LDS stack with stride kThreads and
// m.stack_depth entries (the image's bound).
__device__ void closest_hit(const ModelC& m, const RayPre& R, int* stack, float& best_t, int32_t& best_i) {
    best_t = INFINITY;
    best_i = -1;
    if (m.n_tris == 0) return;
    int node = 0, sp = 0;
    // a valid image visits each node at most once; the cap only guarantees
    // termination for a corrupt one
    for (int visits = 0; visits < (1 << 20); ++visits) {
        const float4* p = reinterpret_cast<const float4*>(m.nodes + node);
        const float4 lx = p[0], ly = p[1], lz = p[2], hx = p[3], hy = p[4], hz = p[5];
        const int4 ch = *reinterpret_cast<const int4*>(p + 6);
        const int32_t ref[4] = {ch.x, ch.y, ch.z, ch.w};
        float tn[4];
        bool h[4];
        h[0] = hit_box(R, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, best_t, tn[0]);
        h[1] = hit_box(R, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, best_t, tn[1]);
        h[2] = hit_box(R, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, best_t, tn[2]);
        h[3] = hit_box(R, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, best_t, tn[3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h[c] = h[c] && ref[c] != kBvhEmpty;
            if (h[c] && ref[c] < 0) {
                leaf(R, m.tris, ref[c], best_t, best_i);
                h[c] = false;
            }
        }
        // order the hit interior children by entry distance (misses sort last)
        float d[4];
        int32_t r[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            d[c] = h[c] ? tn[c] : INFINITY;
            r[c] = h[c] ? ref[c] : kBvhEmpty;
        }
#define INRF_CSWAP(a, b)                                     \
    if (d[b] < d[a]) {                                       \
        const float td = d[a]; d[a] = d[b]; d[b] = td;       \
        const int32_t tr = r[a]; r[a] = r[b]; r[b] = tr;     \
    }
        INRF_CSWAP(0, 1)
        INRF_CSWAP(2, 3)
        INRF_CSWAP(0, 2)
        INRF_CSWAP(1, 3)
        INRF_CSWAP(1, 2)
#undef INRF_CSWAP
        // push the farther ones, farthest first, then visit the nearest
#pragma unroll
        for (int c = 3; c >= 1; --c)
            if (r[c] != kBvhEmpty && sp < m.stack_depth) stack[(sp++) * kThreads] = r[c];
        if (r[0] != kBvhEmpty) {
            node = r[0];
        } else {
            if (sp == 0) break;
            node = stack[(--sp) * kThreads];
        }
    }
}

// Closest hit of a wave of camera rays (one shared origin, neighbouring
// directions) traversed as one packet: the wave walks a single node
// sequence, visiting a child if any of its active lanes hits it within that
// lane's current closest distance, so every lane still tests every triangle
// it could hit and gets the same closest hit as a traversal of its own.
// Nodes and triangles are read at wave-uniform addresses; the stack of
// deferred nodes is wave-uniform (`wst`, m.stack_depth entries in LDS).
// Children are ordered by the entry distance of the lowest lane that hits
// them.
// B is any view with the members nodes, tris, n_tris and stack_depth (a
// model, or one object of a scene).  best_t / best_i come in as the lane's
// current closest hit (INFINITY / -1 for none) and are only improved.
template <class B>
__device__ void closest_hit_packet(const B& m, const RayPre& R, bool active, int* wst, float& best_t,
                                   int32_t& best_i) {
    if (m.n_tris == 0 || __ballot(active) == 0) return;
    int node = 0, sp = 0;
    for (int visits = 0; visits < (1 << 20); ++visits) {
        const float4* p = reinterpret_cast<const float4*>(m.nodes + node);
        const float4 lx = p[0], ly = p[1], lz = p[2], hx = p[3], hy = p[4], hz = p[5];
        const int4 ch = *reinterpret_cast<const int4*>(p + 6);
        const int32_t ref[4] = {ch.x, ch.y, ch.z, ch.w};
        float tn[4];
        bool h[4];
        h[0] = hit_box(R, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, best_t, tn[0]);
        h[1] = hit_box(R, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, best_t, tn[1]);
        h[2] = hit_box(R, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, best_t, tn[2]);
        h[3] = hit_box(R, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, best_t, tn[3]);
        uint64_t any[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h[c] = h[c] && active && ref[c] != kBvhEmpty;
            any[c] = __ballot(h[c]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (ref[c] < 0 && any[c]) leaf(R, m.tris, ref[c], best_t, best_i, h[c]);  // wave-uniform branch
        float d[4];
        int32_t r[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bool go = ref[c] >= 0 && any[c] != 0;
            const int rep = go ? int(__builtin_ctzll(any[c])) : 0;
            d[c] = go ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tn[c]), rep)) : INFINITY;
            r[c] = go ? ref[c] : kBvhEmpty;
        }
#define INRF_CSWAP(a, b)                                     \
    if (d[b] < d[a]) {                                       \
        const float td = d[a]; d[a] = d[b]; d[b] = td;       \
        const int32_t tr = r[a]; r[a] = r[b]; r[b] = tr;     \
    }
        INRF_CSWAP(0, 1)
        INRF_CSWAP(2, 3)
        INRF_CSWAP(0, 2)
        INRF_CSWAP(1, 3)
        INRF_CSWAP(1, 2)
#undef INRF_CSWAP
#pragma unroll
        for (int c = 3; c >= 1; --c)
            if (r[c] != kBvhEmpty && sp < m.stack_depth) wst[sp++] = r[c];
        if (r[0] != kBvhEmpty) {
            node = r[0];
        } else {
            if (sp == 0) break;
            node = __builtin_amdgcn_readfirstlane(wst[--sp]);
        }
    }
}

}  // namespace dev
}  // namespace inrf

#include "bin_device.hpp"

namespace inrf {
namespace dev {

// One workgroup per 16x16 camera tile (each wave an 8x8 quadrant, so that a
// packet is compact) or per 256 batch rays.  Writes depth / triangle / zero
// colour of misses and, if records are requested, the hit records of the
// workgroup in lane order to tmp[base ..], base = the index of the
// workgroup's first ray in the output (tiles of a row band are laid out
// one after another), with blk[b] = (hits, base).
template <bool CAMERA, int NCAM, bool BINNED = false>
__global__ __launch_bounds__(kThreads) void k_trace(ModelC m, CamSet<NCAM> cams, TraceArgs a, BinsC bins) {
    extern __shared__ int stack[];  // batch: [m.stack_depth][kThreads] per-lane stacks
    __shared__ int wst[(kThreads / 64) * kBvhMaxStack];
    __shared__ int s_cnt[kThreads / 64];
    const int lane = __lane_id(), wave = int(threadIdx.x) / 64;
    int64_t ray, base;
    bool valid;
    float3 o, d;
    int qx = 0, qy = 0;  // the wave's quadrant (camera)
    bool empty = false;  // binned: the wave's quadrant has no triangle to test (wave-uniform)
    if (CAMERA) {
        int j = 0;  // the camera of this tile (wave-uniform)
        for (int k = 1; k < NCAM && k < cams.n; ++k)
            if (int(blockIdx.x) >= cams.c[k].tile0) j = k;
        const CamC& cam = cams.c[j];
        const int tile = int(blockIdx.x) - cam.tile0;
        int tx, ty;
        tile_at(tile, cam.tiles_x, (cam.H + kTile - 1) / kTile, tx, ty);
        const int row = ty * kTile + 8 * (wave >> 1) + (lane >> 3), col = tx * kTile + 8 * (wave & 1) + (lane & 7);
        qx = 2 * tx + (wave & 1);
        qy = 2 * ty + (wave >> 1);
        valid = row < cam.H && col < cam.W;
        ray = cam.pix0 + int64_t(row) * cam.W + col;
        base = cam.pix0 + int64_t(ty) * kTile * cam.W + int64_t(tx) * kTile * min(kTile, cam.H - ty * kTile);
        if constexpr (BINNED) {
            if (qx < bins.QX && qy < bins.QY) {
                const int q = __builtin_amdgcn_readfirstlane(qy * bins.QX + qx);
                empty = (bins.fcnt[q] | bins.cnt[q] | bins.total[1]) == 0;
            } else {
                empty = true;  // every pixel of the quadrant is outside the image
            }
        }
        if (empty) d = make_float3(0.f, 0.f, 1.f);  // no ray to set up: every lane misses
        else d = camera_dir(cam, row, col);
        o = make_float3(cam.o[0], cam.o[1], cam.o[2]);
    } else {
        ray = int64_t(blockIdx.x) * kThreads + threadIdx.x;
        base = int64_t(blockIdx.x) * kThreads;
        valid = ray < a.n;
        if (valid) {
            o = make_float3(a.ray_o[3 * ray], a.ray_o[3 * ray + 1], a.ray_o[3 * ray + 2]);
            d = make_float3(a.ray_d[3 * ray], a.ray_d[3 * ray + 1], a.ray_d[3 * ray + 2]);
        } else {
            o = d = make_float3(0.f, 0.f, 1.f);
        }
    }
    const bool finite = isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(d.x) && isfinite(d.y) &&
                        isfinite(d.z) && (d.x != 0.f || d.y != 0.f || d.z != 0.f);
    float t = INFINITY;
    int32_t tri = -1;
    const bool active = valid && finite;
    if (CAMERA) {
        if constexpr (BINNED) {
            if (!empty) {
                const RayPre R = ray_setup(o, active ? d : make_float3(0.f, 0.f, 1.f));
                closest_hit_binned(m, bins, qx, qy, R, active, wst + wave * kBvhMaxStack, t, tri);
            }
        } else {
            const RayPre R = ray_setup(o, active ? d : make_float3(0.f, 0.f, 1.f));
            closest_hit_packet(m, R, active, wst + wave * kBvhMaxStack, t, tri);
        }
    } else if (active) {
        const RayPre R = ray_setup(o, d);
        closest_hit(m, R, stack + threadIdx.x, t, tri);
    }
    const bool hit = active && tri >= 0;
    if (valid) {
        if (a.depth) a.depth[ray] = t;
        if (a.tri) a.tri[ray] = tri;
        if (a.rgba && !hit) reinterpret_cast<float4*>(a.rgba)[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (a.tmp) {
        const uint64_t mask = __ballot(hit);
        if (lane == 0) s_cnt[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            before += w < wave ? s_cnt[w] : 0;
            total += s_cnt[w];
        }
        if (hit) {
            const int64_t pos = base + before + __popcll(mask & ((uint64_t(1) << lane) - 1));
            const float x = clamp01(o.x + t * d.x), y = clamp01(o.y + t * d.y), z = clamp01(o.z + t * d.z);
            if constexpr (CAMERA && NCAM == 1) {
                static_cast<CamHit*>(a.tmp)[pos] = CamHit{x, y, z, int32_t(ray)};
            } else {
                const float3 u = unit_of(d);
                static_cast<HitRec*>(a.tmp)[pos] = HitRec{x, y, z, int32_t(ray), u.x, u.y, u.z, 0};
            }
        }
        if (threadIdx.x == 0) a.blk[blockIdx.x] = make_int2(total, int(base));
    }
}

// Exclusive prefix sum of the per-tile hit counts in two levels: k_scan_local
// scans runs of kScanRun counts (one workgroup each) and writes each run's
// total; k_scan_runs scans those totals (one workgroup) and writes the grand
// total to the counter.  k_compact adds the two.

// Inclusive sum of v over the lanes of a wave up to this one.
__device__ __forceinline__ int wave_scan(int v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive block-wide prefix of v (kScanThreads threads); *total gets the sum.
__device__ __forceinline__ int block_exclusive(int v, int* s_wave, int* total) {
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int inc = wave_scan(v);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const int w = lane < kScanThreads / 64 ? s_wave[lane] : 0;
        const int wi = wave_scan(w);
        if (lane < kScanThreads / 64) s_wave[lane] = wi - w;  // exclusive over waves
        if (lane == kScanThreads / 64 - 1) s_wave[kScanThreads / 64] = wi;
    }
    __syncthreads();
    *total = s_wave[kScanThreads / 64];
    return s_wave[wave] + inc - v;
}

// cnt: counts at cnt[i * stride] (stride 2: the .x of per-tile (count, base)
// pairs), each taken as min(count, clamp).
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t* __restrict__ cnt, int stride, int n_blk,
                                                             int32_t* __restrict__ offsets, int32_t* __restrict__ runs,
                                                             int clamp) {
    __shared__ int s_wave[kScanThreads / 64 + 1];
    const int i0 = blockIdx.x * kScanRun + 2 * threadIdx.x;
    const int c0 = i0 < n_blk ? min(cnt[int64_t(i0) * stride], clamp) : 0,
              c1 = i0 + 1 < n_blk ? min(cnt[int64_t(i0 + 1) * stride], clamp) : 0;
    int total;
    const int ex = block_exclusive(c0 + c1, s_wave, &total);
    if (i0 < n_blk) offsets[i0] = ex;
    if (i0 + 1 < n_blk) offsets[i0 + 1] = ex + c0;
    if (threadIdx.x == 0) runs[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_runs(int32_t* __restrict__ runs, int n_runs,
                                                            int32_t* __restrict__ counter,
                                                            int32_t* __restrict__ clear, int n_clear) {
    __shared__ int s_wave[kScanThreads / 64 + 1];
    int carry = 0;
    for (int r0 = 0; r0 < n_runs; r0 += kScanThreads) {  // n_runs is small: usually one pass
        const int i = r0 + threadIdx.x;
        const int v = i < n_runs ? runs[i] : 0;
        int total;
        const int ex = block_exclusive(v, s_wave, &total);
        if (i < n_runs) runs[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *counter = carry;
    if (int(threadIdx.x) < n_clear) clear[threadIdx.x] = 0;  // the header's other counters
}

// Packs the workgroups' records into one list in workgroup order (tile
// order for a camera), so the list does not depend on timing.  Workgroup b
// moves the record runs b, b + stride, ... (n_groups of them): one run per
// workgroup for a single object, every object's run of tile b for a scene
// (runs stored [object][tile]), so a scene launches one workgroup per tile
// rather than one per (object, tile).
template <class Rec>
__global__ __launch_bounds__(kThreads) void k_compact(const int2* __restrict__ blk, const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ runs, const Rec* __restrict__ tmp,
                                                      Rec* __restrict__ recs, int n_groups, int stride) {
    constexpr int kWords = int(sizeof(Rec) / sizeof(float4));
    // the runs' (count, source) and destinations, all requested at once (n_groups <= kThreads)
    __shared__ int3 s_run[kThreads];
    if (int(threadIdx.x) < n_groups) {
        const int j = int(threadIdx.x) * stride + int(blockIdx.x);
        const int2 b = blk[j];
        s_run[threadIdx.x] = make_int3(b.x, b.y, offsets[j] + runs[j / kScanRun]);
    }
    __syncthreads();
    for (int k = 0; k < n_groups; ++k) {
        const int3 r = s_run[k];
        for (int i = threadIdx.x; i < r.x; i += kThreads) {
            const float4* src = reinterpret_cast<const float4*>(tmp + r.y + i);
            float4* dst = reinterpret_cast<float4*>(recs + r.z + i);
#pragma unroll
            for (int w = 0; w < kWords; ++w) dst[w] = src[w];
        }
    }
}

// k_compact for a single object: one wave per workgroup run of the trace
// (a camera tile or a block of rays), four runs per workgroup, so a frame's
// many empty tiles cost one wave each rather than one workgroup.
template <class Rec>
__global__ __launch_bounds__(kThreads) void k_compact_runs(const int2* __restrict__ blk,
                                                           const int32_t* __restrict__ offsets,
                                                           const int32_t* __restrict__ runs, const Rec* __restrict__ tmp,
                                                           Rec* __restrict__ recs, int n_blk) {
    constexpr int kWords = int(sizeof(Rec) / sizeof(float4));
    const int j = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * (kThreads / 64) + int(threadIdx.x) / 64);
    if (j >= n_blk) return;
    const int2 b = blk[j];
    if (b.x == 0) return;
    const int dst = offsets[j] + runs[j / kScanRun];
    for (int i = __lane_id(); i < b.x; i += 64) {
        const float4* src = reinterpret_cast<const float4*>(tmp + b.y + i);
        float4* out = reinterpret_cast<float4*>(recs + dst + i);
#pragma unroll
        for (int w = 0; w < kWords; ++w) out[w] = src[w];
    }
}

// ------------------------------------------------------------- shading ----

// Network kernels are declared to fit in at most 256 registers per lane (at
// least two waves per SIMD), which those of up to 16 levels do anyway (the
// shading kernel's larger instantiations keep the full register file, as they
// would spill in 256); with that bound the
// compiler keeps matrix-instruction results in ordinary vector registers
// instead of accumulation registers that must be copied out before the
// ReLU and the next layer.  (k_mlp on FP32 rows keeps the accumulation
// registers: in vector registers its 20- to 32-level instantiations were
// given a destination partially overlapping the accumulator input, which the
// build's assembly check refuses.)
#ifndef INRF_MFMA_VGPR
#define INRF_MFMA_VGPR __attribute__((amdgpu_waves_per_eu(2)))
#endif

template <class P>
struct TileElem {
    typedef P type;  // FP16/BF16 tiles hold the MMA operand type
};
template <>
struct TileElem<float> {
    typedef float type;
};

// Encoded features of levels L .. LMAX-1 of one point into e[2L ..], two
// levels at a time so that the offset loads of both are in flight before
// either is waited on.  Written as a recursion rather than a loop so that
// every level index stays a compile-time constant (the features stay in
// registers) at any level count.
template <class TableT, int L, int LMAX, int F, class M>
__device__ __forceinline__ void gather_levels(const M& m, float x, float y, float z, float (&e)[F]) {
    if constexpr (L < LMAX) {
        float2 ea = make_float2(0.f, 0.f), eb = make_float2(0.f, 0.f);
        if (L + 1 < m.n_levels) encode_level_pair<TableT>(m, m.lv[L], m.lv[L + 1], x, y, z, ea, eb);
        else if (L < m.n_levels) ea = encode_level<TableT>(m, m.lv[L], x, y, z, nullptr);
        e[2 * L] = ea.x;
        e[2 * L + 1] = ea.y;
        e[2 * L + 2] = eb.x;
        e[2 * L + 3] = eb.y;
        __builtin_amdgcn_sched_barrier(0);  // one pair of levels in flight at a time
        gather_levels<TableT, L + 2, LMAX>(m, x, y, z, e);
    }
}

// Geometry of the per-wave LDS tile: 16 rows (rays) of F feature slots.  X
// extra network inputs (0, or 1 for the coarse opacity of the i-NOLF form).
template <class P, int LPG, int X = 0>
struct ShadeShape {
    static constexpr int V = Mfma<P>::V;
    static constexpr int LMAX = 4 * LPG;  // levels the instantiation handles
    static constexpr int F = feature_slots(LMAX, V);
    // a row: F feature slots, 16 SH values, padding that keeps rows 16-byte aligned
    static constexpr int STRIDE = F + INRF_SH_DIM + (V == 1 ? 4 : 8);
    static constexpr int S1 = l1_steps(F, V, X);
    static constexpr size_t tile_bytes = 16 * STRIDE * sizeof(typename TileElem<P>::type);
    static constexpr size_t lds_bytes = size_t(weight_bytes(F, V, X)) + (kThreads / 64) * tile_bytes;
};

// One wave step of the shading kernel: the records [base, base + 64) of
// [.., n), one per lane.  Each lane gathers every level of its own hit (a
// level's loads then cover 64 neighbouring rays, and level parameters are
// wave-uniform), two levels at a time so their offset loads are in flight
// together, and computes the SH values of its own ray.  The network then runs
// on four blocks of 16 rays; each block's features and SH values pass
// through the wave's LDS tile into the matrix-core B-operand layout.
// NOLF (the paper's own i-NOLF form): the record's pad holds the ray's
// coarse opacity, a further network input, and the colour buffer holds the
// diffuse colour and tint of the hit, which the outputs complete as
// (c_d + t c_s, alpha).  With cam.W > 0 the records are the CamHit records
// of that camera's frame.
template <class TableT, class P, int LPG, bool NOLF, class M>
__device__ __forceinline__ void shade_step(const M& m, const typename Mfma<P>::vec* W,
                                           typename TileElem<P>::type* tile, const void* __restrict__ recs,
                                           const CamC& cam, int64_t base, int64_t n, float* __restrict__ rgba) {
    constexpr int X = NOLF ? 1 : 0;
    typedef Mfma<P> Mf;
    typedef typename Mf::vec Vec;
    typedef ShadeShape<P, LPG, X> S;
    typedef typename TileElem<P>::type T;
    const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
    const int64_t i = base + lane;
    const bool act = i < n;
    HitRec h;
    if (cam.W > 0) {  // wave-uniform
        const CamHit c = act ? static_cast<const CamHit*>(recs)[i] : CamHit{0.f, 0.f, 0.f, int32_t(cam.pix0)};
        const int p = c.out - int(cam.pix0);  // a single camera: pix0 = 0, pixels < 2^31
        const int row = p / cam.W, col = p - row * cam.W;
        const float3 u = unit_of(camera_dir(cam, row, col));
        h = HitRec{c.x, c.y, c.z, c.out, u.x, u.y, u.z, 0};
    } else if (act) {
        h = static_cast<const HitRec*>(recs)[i];
    } else {
        h = HitRec{0.f, 0.f, 0.f, 0, 0.f, 0.f, 1.f, 0};
    }
    float e[S::F];
#pragma unroll
    for (int k = 2 * S::LMAX; k < S::F; ++k) e[k] = 0.f;
    gather_levels<TableT, 0, S::LMAX>(m, h.x, h.y, h.z, e);
    float sh[INRF_SH_DIM];  // of the lane's own ray (unit direction)
    sh16(h.dx, h.dy, h.dz, sh);
    const int nb = int(min<int64_t>(4, (n - base + 15) / 16));
    for (int b = 0; b < nb; ++b) {
        if (g == b) {
            T* row = tile + r * S::STRIDE;
#pragma unroll
            for (int k = 0; k < S::F; ++k) row[k] = T(e[k]);
#pragma unroll
            for (int k = 0; k < INRF_SH_DIM; ++k) row[S::F + k] = T(sh[k]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int src = 16 * b + r;
        Vec b1[S::S1];
        const float extra = NOLF ? __shfl(__int_as_float(h.pad), src) : 0.f;
        load_inputs_row<P, S::F, X>(tile + r * S::STRIDE, b1, extra);
        const int out = __shfl(h.out, src);
        const f32x4 o = mlp_block<P, S::F, X>(W, b1);
        if (g == 0 && base + src < n) {
            float4* px = reinterpret_cast<float4*>(rgba) + out;
            if constexpr (NOLF) {
                const float4 dt = *px;  // diffuse RGB and tint
                *px = make_float4(dt.x + dt.w * sigmoidf(o[0]), dt.y + dt.w * sigmoidf(o[1]),
                                  dt.z + dt.w * sigmoidf(o[2]), sigmoidf(o[3]));
            } else {
                *px = make_float4(sigmoidf(o[0]), sigmoidf(o[1]), sigmoidf(o[2]), sigmoidf(o[3]));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the tile is rewritten by the next block
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Persistent waves over the packed hit list [first, counter), 64 hits per
// wave step (shade_step); CamHit records of camera `cam` when cam.W > 0,
// else HitRec records.
template <class TableT, class P, int LPG, bool NOLF = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LPG <= 4 ? 2 : 1)))
void k_shade(ModelC m, const void* __restrict__ recs, CamC cam, const int32_t* __restrict__ first,
             const int32_t* __restrict__ counter, float* __restrict__ rgba) {
    constexpr int X = NOLF ? 1 : 0;
    typedef typename Mfma<P>::vec Vec;
    typedef ShadeShape<P, LPG, X> S;
    typedef typename TileElem<P>::type T;
    const int lo = first ? *first : 0, n = *counter;  // records [lo, n)
    // a workgroup with no records to shade (few hits: a small frame) leaves
    // before staging the weights
    if (lo + int64_t(blockIdx.x) * kThreads >= n) return;
    extern __shared__ float4 lds_v[];
    Vec* W = reinterpret_cast<Vec*>(lds_v);
    stage_weights<P, X>(m.weights, m.n_levels, S::F, W);
    T* tile = reinterpret_cast<T*>(reinterpret_cast<char*>(lds_v) + weight_bytes(S::F, S::V, X) +
                                   (threadIdx.x / 64) * S::tile_bytes);
    __syncthreads();
    for (int64_t base = lo + (int64_t(blockIdx.x) * (kThreads / 64) + threadIdx.x / 64) * 64; base < n;
         base += int64_t(gridDim.x) * kThreads)
        shade_step<TableT, P, LPG, NOLF>(m, W, tile, recs, cam, base, n, rgba);
}

// The shading view of one object of a scene: its tables, weights and level
// parameters (at most 12 levels), small enough that a whole scene's set
// travels as one kernel argument.
constexpr int kSceneShadeLevels = 12;
struct ShadeModel {
    int32_t n_levels, pad;
    const uint32_t* phi;
    const void* table;
    const float* weights;
    LevelC lv[kSceneShadeLevels];
};
struct ShadeSet {
    int32_t n, pad;
    ShadeModel m[INRF_MAX_OBJECTS];
};

// Every object of a scene in one launch.  The packed records are grouped by
// object (object o's records are [seg[o], seg[o+1])); each object's run is
// cut into chunks of one workgroup step (256 records), and workgroup b takes
// chunks b, b + G, b + 2G, ... (G workgroups) of all objects in order, so the
// rays in flight at any moment are neighbours in the list, as in k_shade.
// A workgroup restages the weights in LDS when its chunk's object changes.
// All objects share the table type and precision; LPG covers the largest
// level count.  (Measured against giving each object its own share of the
// workgroups, staged once: slower, 0.97 against 0.92 ms for the 12-object
// 4K frame.)
template <class TableT, class P, int LPG>
__global__ __launch_bounds__(kThreads) INRF_MFMA_VGPR void k_shade_scene(ShadeSet ss, const HitRec* __restrict__ recs,
                                                                         const int32_t* __restrict__ seg,
                                                                         float* __restrict__ rgba) {
    typedef typename Mfma<P>::vec Vec;
    typedef ShadeShape<P, LPG> S;
    typedef typename TileElem<P>::type T;
    // chunks per object and in all (the same sums in every workgroup)
    int total = 0;
    for (int o = 0; o < ss.n; ++o) total += (seg[o + 1] - seg[o] + kThreads - 1) / kThreads;
    if (int(blockIdx.x) >= total) return;
    extern __shared__ float4 lds_v[];
    Vec* W = reinterpret_cast<Vec*>(lds_v);
    T* tile = reinterpret_cast<T*>(reinterpret_cast<char*>(lds_v) + weight_bytes(S::F, S::V) +
                                   (threadIdx.x / 64) * S::tile_bytes);
    int staged = -1, o = 0, first_chunk = 0;  // object of chunk c: first_chunk <= c < first_chunk + its chunks
    for (int c = blockIdx.x; c < total; c += gridDim.x) {
        while (c >= first_chunk + (seg[o + 1] - seg[o] + kThreads - 1) / kThreads) {
            first_chunk += (seg[o + 1] - seg[o] + kThreads - 1) / kThreads;
            ++o;
        }
        const int obj = __builtin_amdgcn_readfirstlane(o);
        if (obj != staged) {
            __syncthreads();  // every wave is done with the previous object's weights
            stage_weights<P>(ss.m[obj].weights, ss.m[obj].n_levels, S::F, W);
            __syncthreads();
            staged = obj;
        }
        const int64_t base = seg[obj] + int64_t(c - first_chunk) * kThreads + (threadIdx.x / 64) * 64;
        const int64_t n = seg[obj + 1];
        if (base < n) shade_step<TableT, P, LPG, false>(ss.m[obj], W, tile, recs, CamC{}, base, n, rgba);
    }
}

// ------------------------------------------------------------ camera rays --

// Origin and unit direction of every pixel ray of one camera, row-major
// (the rays the camera kernels generate, through camera_dir).
__global__ __launch_bounds__(kThreads) void k_camera_rays(CamC cam, float* __restrict__ ray_o,
                                                          float* __restrict__ ray_d) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= int64_t(cam.W) * cam.H) return;
    const int row = int(i / cam.W), col = int(i % cam.W);
    const float3 d = camera_dir(cam, row, col);
    if (ray_o) {
        ray_o[3 * i] = cam.o[0];
        ray_o[3 * i + 1] = cam.o[1];
        ray_o[3 * i + 2] = cam.o[2];
    }
    ray_d[3 * i] = d.x;
    ray_d[3 * i + 1] = d.y;
    ray_d[3 * i + 2] = d.z;
}

// --------------------------------------------------- encoder and network --

template <class TableT>
__global__ __launch_bounds__(kThreads) void k_encode(ModelC m, const float* __restrict__ x, int64_t n,
                                                     float* __restrict__ enc, int32_t* __restrict__ slots) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const float px = clamp01(x[3 * i]), py = clamp01(x[3 * i + 1]), pz = clamp01(x[3 * i + 2]);
    for (int l = 0; l < m.n_levels; ++l) {
        const float2 e = encode_level<TableT>(m, m.lv[l], px, py, pz, slots ? slots + (i * m.n_levels + l) * 8 : nullptr);
        enc[i * 2 * m.n_levels + 2 * l] = e.x;
        enc[i * 2 * m.n_levels + 2 * l + 1] = e.y;
    }
}

// a[k .. k+3] with entries at index >= limit read as zero (and all zero for
// an inactive lane); one 16-byte load when the four lie below the limit and
// `vec` says that a + k is 16-byte aligned.
__device__ __forceinline__ f32x4 load_inputs4(const float* a, int k, int limit, bool act, bool vec) {
    if (!act || k >= limit) return f32x4{0.f, 0.f, 0.f, 0.f};
    if (vec && k + 4 <= limit) return *reinterpret_cast<const f32x4*>(a + k);
    f32x4 v;
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = k + t < limit ? a[k + t] : 0.f;
    return v;
}

// The network alone on caller inputs [n][d_in] in natural order: lane
// (g, r) loads exactly its B operands of ray r straight from memory.
template <class P, int LPG>
__global__ __launch_bounds__(kThreads) void k_mlp(ModelC m, const float* __restrict__ x, int64_t n,
                                                  float* __restrict__ rgba, bool vec) {
    typedef Mfma<P> M;
    typedef typename M::vec Vec;
    typedef ShadeShape<P, LPG> S;
    extern __shared__ float4 lds_v[];
    Vec* W = reinterpret_cast<Vec*>(lds_v);
    stage_weights<P>(m.weights, m.n_levels, S::F, W);
    __syncthreads();
    const int L2 = 2 * m.n_levels, d_in = L2 + INRF_SH_DIM;
    const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
    for (int64_t blk = int64_t(blockIdx.x) * (kThreads / 64) + threadIdx.x / 64; blk * 16 < n;
         blk += int64_t(gridDim.x) * (kThreads / 64)) {
        const int64_t ray = blk * 16 + r;
        const bool act = ray < n;
        const float* row = x + (act ? ray : 0) * d_in;
        Vec b1[S::S1];
        if constexpr (S::V == 1) {
#pragma unroll
            for (int j = 0; j < S::F / 16; ++j) {
                const f32x4 v = load_inputs4(row, 16 * j + 4 * g, L2, act, vec);
#pragma unroll
                for (int t = 0; t < 4; ++t) b1[4 * j + t] = v[t];
            }
            const f32x4 v = load_inputs4(row + L2, 4 * g, INRF_SH_DIM, act, vec);
#pragma unroll
            for (int t = 0; t < 4; ++t) b1[S::F / 4 + t] = v[t];
        } else {
#pragma unroll
            for (int c = 0; c < S::F / 32; ++c) {
                const f32x4 lo = load_inputs4(row, 32 * c + 8 * g, L2, act, vec);
                const f32x4 hi = load_inputs4(row, 32 * c + 8 * g + 4, L2, act, vec);
                Vec v;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    v[t] = M::cvt(lo[t]);
                    v[4 + t] = M::cvt(hi[t]);
                }
                b1[c] = v;
            }
            const f32x4 lo = load_inputs4(row + L2, 8 * g, g < 2 ? INRF_SH_DIM : 0, act, vec);
            const f32x4 hi = load_inputs4(row + L2, 8 * g + 4, g < 2 ? INRF_SH_DIM : 0, act, vec);
            Vec v;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v[t] = M::cvt(lo[t]);
                v[4 + t] = M::cvt(hi[t]);
            }
            b1[S::S1 - 1] = v;
        }
        const f32x4 o = mlp_block<P, S::F>(W, b1);
        if (g == 0 && act)
            reinterpret_cast<float4*>(rgba)[ray] =
                make_float4(sigmoidf(o[0]), sigmoidf(o[1]), sigmoidf(o[2]), sigmoidf(o[3]));
    }
}

// The network on 16-bit encodings and view directions: enc [n][2L] of the
// precision's 16-bit type (P), dir [n][3] FP32.  Lane (g, r) loads exactly
// its B operands of ray r (feature slots 32c + 8g .. +7 of the row, one
// 16-byte load per chunk when `vec` says rows are 16-byte aligned) and
// computes the SH values of the unit direction itself, as the shading
// kernel does, so the input is 4L + 12 bytes per ray instead of
// 4 (2L + 16).
// Inputs of ray `ray` for lane group g: the chunks of its 16-bit encoding
// row this lane supplies, and the view direction.
// Feature slots 32c + 8g .. +7 of the row (c < F / 32) of an encoding of 2L
// 16-bit values, zeros past the row and for inactive rays.  VEC: rows are
// 16-byte aligned and 2L is a multiple of 8, so a chunk lies wholly inside
// the row or wholly past it and is one 16-byte load; otherwise value by
// value.
template <class P, int F, bool VEC>
__device__ __forceinline__ void load_enc(const P* __restrict__ enc, int64_t ray, bool act, int L2, int g,
                                         typename Mfma<P>::vec* e) {
    typedef typename Mfma<P>::vec Vec;
    const P* row = enc + (act ? ray : 0) * L2;
#pragma unroll
    for (int c = 0; c < F / 32; ++c) {
        const int k0 = 32 * c + 8 * g;
        Vec v = {};
        if constexpr (VEC) {
            if (act && k0 < L2) v = *reinterpret_cast<const Vec*>(row + k0);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (act && k0 + i < L2) v[i] = row[k0 + i];
        }
        e[c] = v;
    }
}

// Row stride (elements) of the per-wave SH tile of k_mlp_enc: 16 values and
// padding, rows 16-byte aligned.
constexpr int kShRow = INRF_SH_DIM + 8;

#ifndef KMLP_BLOCKS
#define KMLP_BLOCKS 4
#endif
constexpr int kMlpBlocks = KMLP_BLOCKS;  // blocks of 16 rays per wave step of k_mlp_enc (1, 2 or 4)

// The network on 16-bit encodings and view directions: enc [n][2L] of the
// precision's 16-bit type (P), dir [n][3] FP32.  A wave step takes
// 16 * kMlpBlocks rays.  The lane that owns a ray (lane l of block l / 16)
// normalises its direction, computes its 16 SH values once and writes them
// to a row of the wave's LDS tile; for each block, lane (g, r) then loads
// its B operands of ray r directly (feature slots 32c + 8g .. +7 of the
// encoding row) and reads SH values 8g .. 8g + 7 of the ray from the tile.
// The input is 4L + 12 bytes per ray instead of 4 (2L + 16).
template <class P, int LPG, bool VEC>
__global__ __launch_bounds__(kThreads) INRF_MFMA_VGPR void k_mlp_enc(ModelC m, const P* __restrict__ enc,
                                                                     const float* __restrict__ dir, int64_t n,
                                                                     float* __restrict__ rgba) {
    typedef Mfma<P> M;
    typedef typename M::vec Vec;
    typedef ShadeShape<P, LPG> S;
    static_assert(S::V == 8, "16-bit operands only");
    constexpr int NB = kMlpBlocks, RAYS = 16 * NB;
    extern __shared__ float4 lds_v[];
    Vec* W = reinterpret_cast<Vec*>(lds_v);
    stage_weights<P>(m.weights, m.n_levels, S::F, W);
    P* shtile = reinterpret_cast<P*>(reinterpret_cast<char*>(lds_v) + weight_bytes(S::F, S::V)) +
                (threadIdx.x / 64) * RAYS * kShRow;
    __syncthreads();
    const int L2 = 2 * m.n_levels;
    const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
    // the lane's weight fragments, loaded once: no weight reads from LDS in the loop
    WReg<Vec, weight_frags<P, S::F>()> wr;
#pragma unroll
    for (int f = 0; f < weight_frags<P, S::F>(); ++f) wr.w[f] = W[f * 64 + lane];
    const int64_t stride = int64_t(gridDim.x) * (kThreads / 64);
    for (int64_t step = int64_t(blockIdx.x) * (kThreads / 64) + threadIdx.x / 64; step * RAYS < n; step += stride) {
        const int64_t base = step * RAYS;
        Vec e[NB][S::F / 32];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int64_t ray = base + 16 * k + r;
            load_enc<P, S::F, VEC>(enc, ray, ray < n, L2, g, e[k]);
        }
        if (lane < RAYS) {  // the lane's own ray: its SH row
            const int64_t ray = base + lane;
            const bool act = ray < n;
            const float dx = act ? dir[3 * ray] : 0.f, dy = act ? dir[3 * ray + 1] : 0.f,
                        dz = act ? dir[3 * ray + 2] : 1.f;
            const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
            float sh[16];
            sh16(dx * inv, dy * inv, dz * inv, sh);
            Vec lo, hi;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                lo[i] = M::cvt(sh[i]);
                hi[i] = M::cvt(sh[8 + i]);
            }
            Vec* row = reinterpret_cast<Vec*>(shtile + lane * kShRow);
            row[0] = lo;
            row[1] = hi;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            Vec b1[S::S1];
#pragma unroll
            for (int c = 0; c < S::F / 32; ++c) b1[c] = e[k][c];
            Vec v = reinterpret_cast<const Vec*>(shtile + (16 * k + r) * kShRow)[g & 1];
            if (g >= 2) {
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = M::cvt(0.f);
            }
            b1[S::S1 - 1] = v;
            const f32x4 o = mlp_block_w<P, S::F, 0>(wr, b1);
            // output c = g of ray r: lane (g, r) takes element g of lane r's
            // tile result, so each lane applies one sigmoid and the block's
            // 64 outputs go out as one contiguous store
            const int64_t ray = base + 16 * k + r;
            const float t0 = __shfl(o[0], r), t1 = __shfl(o[1], r), t2 = __shfl(o[2], r), t3 = __shfl(o[3], r);
            const float z = g == 0 ? t0 : (g == 1 ? t1 : (g == 2 ? t2 : t3));
            if (ray < n) rgba[4 * ray + g] = __builtin_amdgcn_rcpf(1.f + __expf(-z));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the SH tile is rewritten by the next step
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace dev
}  // namespace inrf

#include "backward_device.hpp"
#include "scene_device.hpp"
#include "nolf_device.hpp"

namespace inrf {

// ------------------------------------------------------------ host side ---
namespace {

using namespace dev;

constexpr int64_t kWsHeader = 256;
constexpr int kMaxChunks = 2;  // hit counters at the start of the header: the frame's, then one kept at zero

constexpr int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// Workspace of a trace of up to n rays: counter | records | per-tile
// records | per-tile (count, base) | per-tile offsets | per-run offsets |
// screen bins (quadrant counters, the global list, the spill area).  A
// camera of W x H = n pixels has at most ceil(W/16) ceil(H/16) <= n/8 + 2
// tiles.
//
// The quadrant lists of a camera frame share the records' space: the trace
// reads them before k_compact writes the first record.  The spill area holds
// n entries (at most INT32_MAX).
struct WsLayout {
    int64_t recs, tmp, blk, offsets, runs;
    int64_t qcnt, qfcnt, qtotal, entries;  // screen bins of a camera frame (bin_device.hpp)
    int64_t qbase, qscnt, qsfcnt, qtop, spill;
    int64_t n_quads, n_spill, end;
    // Quadrants of a W x H = n pixel frame: at most (W + 7)(H + 7) / 64,
    // below n/64 + isqrt(n) + 16 for every aspect ratio up to about 1:70; a
    // frame with more walks the BVH.
    static constexpr int64_t isqrt(int64_t n) {  // floor(sqrt(n)), bit by bit
        int64_t r = 0;
        for (int64_t b = int64_t(1) << 31; b > 0; b >>= 1)
            if (r + b <= n / (r + b)) r += b;
        return r;
    }
    // extra: 2 more tiles per additional camera of a batch.
    constexpr explicit WsLayout(int64_t n, int64_t extra = 0)
        : recs(0), tmp(0), blk(0), offsets(0), runs(0), qcnt(0), qfcnt(0), qtotal(0), entries(0), qbase(0), qscnt(0),
          qsfcnt(0), qtop(0), spill(0), n_quads(0), n_spill(0), end(0) {
        const int64_t nb = n / 8 + 2 + extra, nr = nb / kScanRun + 1 + kMaxChunks;
        n_quads = n / 64 + isqrt(n) + 16;
        recs = kWsHeader;
        entries = recs;
        tmp = align256(recs + std::max(n * int64_t(sizeof(HitRec)), n_quads * kBinCap * int64_t(sizeof(int2))));
        blk = align256(tmp + n * int64_t(sizeof(HitRec)));
        offsets = align256(blk + nb * int64_t(sizeof(int2)));
        runs = align256(offsets + nb * int64_t(sizeof(int32_t)));
        qcnt = align256(runs + nr * int64_t(sizeof(int32_t)));
        qfcnt = align256(qcnt + n_quads * int64_t(sizeof(int32_t)));
        qtotal = align256(qfcnt + n_quads * int64_t(sizeof(int32_t)));
        qbase = align256(qtotal + (2 + kBinGlobal) * int64_t(sizeof(int32_t)));
        qscnt = align256(qbase + n_quads * int64_t(sizeof(int32_t)));
        qsfcnt = align256(qscnt + n_quads * int64_t(sizeof(int32_t)));
        qtop = align256(qsfcnt + n_quads * int64_t(sizeof(int32_t)));
        spill = align256(qtop + int64_t(sizeof(unsigned long long)));
        n_spill = std::min<int64_t>(n, INT32_MAX);
        end = align256(spill + n_spill * int64_t(sizeof(int2)));
    }
};

// Scratch memory of inrf_render_static, for callers that cannot allocate: a
// file-scope device array that each GPU the library runs on holds until the
// process ends, sized for the workspace of INRF_STATIC_MAX_PIXELS pixels.
// Host code never passes `scratch` itself (its name is a host-side stand-in,
// not a device address): static_scratch() looks up the array's address on
// the current device once and keeps it.
constexpr int64_t kStaticScratchBytes = WsLayout(INRF_STATIC_MAX_PIXELS).end;
static_assert(kStaticScratchBytes <= (int64_t(80) << 20), "static scratch stays modest");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void check_hip(hipError_t e, const char* what);

void* static_scratch() {
    static std::mutex mu;
    static std::vector<std::pair<int, void*>> addr;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& e : addr)
        if (e.first == dev) return e.second;
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (p == nullptr) fail(INRF_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    addr.push_back({dev, p});
    return p;
}

template <class T>
T* ws_at(void* ws, int64_t off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(INRF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int num_cus(int dev) {
    int n = 0;
    check_hip(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    return n > 0 ? n : 1;
}

ModelC make_model(const inrf_model* m, bool need_table, bool need_bvh) {
    require(m != nullptr, "model is NULL");
    require(m->n_levels >= 1 && m->n_levels <= INRF_MAX_LEVELS, "n_levels must be in [1, 32]");
    require(m->table_dtype == INRF_F32 || m->table_dtype == INRF_F16, "table_dtype must be INRF_F32 or INRF_F16");
    ModelC c;
    std::memset(&c, 0, sizeof(c));
    c.n_levels = m->n_levels;
    c.table_dtype = m->table_dtype;
    c.phi = m->phi;
    c.table = m->table;
    c.weights = m->weights;
    c.nodes = reinterpret_cast<const BvhNode*>(m->bvh_nodes);
    c.tris = reinterpret_cast<const BvhTri*>(m->bvh_tris);
    c.n_tris = m->n_tris;
    c.stack_depth = 1;
    if (need_table) require(m->phi && m->table, "phi and table must be set");
    if (need_bvh) {
        require(m->n_tris >= 0, "n_tris must be >= 0");
        require(m->n_tris == 0 || (m->bvh_nodes && m->bvh_tris), "bvh images must be set");
        require(m->n_tris == 0 || (m->bvh_stack >= 1 && m->bvh_stack <= kBvhMaxStack),
                "bvh_stack must be the image's stack bound (1..64)");
        require(m->n_tris == 0 || m->bvh_n_nodes >= 1, "bvh_n_nodes must be the image's node count");
        c.stack_depth = std::max(1, m->bvh_stack);
        c.n_nodes = m->n_tris == 0 ? 0 : m->bvh_n_nodes;
    }
    for (int l = 0; l < m->n_levels; ++l) {
        const inrf_level_desc& d = m->levels[l];
        require(d.res >= 1 && d.res <= 4096, "level resolution must be in [1, 4096]");
        require(d.mbar >= 2 && d.mbar <= 1024, "mbar must be in [2, 1024]");
        require(d.rbar >= 2 && d.rbar <= 1024, "rbar must be in [2, 1024]");
        require(int64_t(d.rbar) * d.rbar * d.rbar < (int64_t(1) << 31), "rbar^3 must fit 31 bits");
        require(d.phi_offset >= 0 && d.slot_offset >= 0, "negative level offsets");
        LevelC& L = c.lv[l];
        L.res = d.res;
        L.mbar = d.mbar;
        L.rbar = d.rbar;
        L.magic_mbar = uint32_t(((uint64_t(1) << 32) + uint64_t(d.mbar) - 1) / uint64_t(d.mbar));
        L.magic_rbar = uint32_t(((uint64_t(1) << 32) + uint64_t(d.rbar) - 1) / uint64_t(d.rbar));
        L.row_m = brick_row(d.mbar);
        L.plane_m = brick_plane(d.mbar);
        L.row_r = brick_row(d.rbar);
        L.plane_r = brick_plane(d.rbar);
        // table entries of the level are addressed with 32-bit byte offsets
        const int64_t entries = brick_entries(d.mbar);
        L.last_m = uint32_t(entries - 1);
        const int64_t elem = m->table_dtype == INRF_F32 ? 8 : 4;
        require(entries * elem <= (int64_t(1) << 32), "a level's table must be below 4 GiB (mbar too large for FP32)");
        L.phi_off = d.phi_offset;
        L.slot_off = d.slot_offset;
    }
    return c;
}

void launch_check(const char* what) { check_hip(hipGetLastError(), what); }

// Launch set-up of a persistent kernel, done once per (device, kernel, LDS
// size) and kept until the process ends: the dynamic-LDS attribute (for
// more than the default 64 KB window) and the resident workgroup count
// (occupancy per CU times the CUs), so a frame does no host-side queries.
struct GridEntry {
    int dev;
    const void* kernel;
    size_t lds;
    unsigned grid;
};

template <class K>
unsigned resident_grid(K kernel, size_t lds) {
    static std::mutex mu;
    static std::vector<GridEntry> cache;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    const void* k = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    for (const GridEntry& e : cache)
        if (e.dev == dev && e.kernel == k && e.lds == lds) return e.grid;
    if (lds > 65536)
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)), "hipFuncSetAttribute");
    int per_cu = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, lds),
              "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    const unsigned grid = unsigned(std::max(1, per_cu) * num_cus(dev));
    cache.push_back({dev, k, lds, grid});
    return grid;
}

template <class TableT, class P, int LPG>
void launch_shade_t(const ModelC& c, const void* recs, const CamC& cam, const int32_t* first, const int32_t* counter,
                    float* rgba, hipStream_t s) {
    const size_t lds = ShadeShape<P, LPG>::lds_bytes;
    auto kern = k_shade<TableT, P, LPG>;
    hipLaunchKernelGGL(kern, dim3(resident_grid(kern, lds)), dim3(kThreads), lds, s, c, recs, cam, first, counter,
                       rgba);
}

template <class P, int LPG>
void launch_mlp_t(const ModelC& c, const float* in, int64_t n, float* rgba, hipStream_t s) {
    const size_t lds = size_t(weight_bytes(ShadeShape<P, LPG>::F, ShadeShape<P, LPG>::V));
    auto kern = k_mlp<P, LPG>;
    const int64_t blocks = (n + kThreads / 4 - 1) / (kThreads / 4);  // 16 rays per wave step
    const unsigned grid = unsigned(std::min<int64_t>(blocks, resident_grid(kern, lds)));
    // rows start 16-byte aligned when the input array does and d_in = 2L + 16 is a multiple of 4
    const bool vec = (reinterpret_cast<uintptr_t>(in) & 15) == 0 && (c.n_levels % 2) == 0;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, c, in, n, rgba, vec);
}

template <class P, int LPG>
void launch_mlp_enc_t(const ModelC& c, const void* enc, const float* dir, int64_t n, float* rgba, hipStream_t s) {
    const size_t lds = size_t(weight_bytes(ShadeShape<P, LPG>::F, ShadeShape<P, LPG>::V)) +
                       (kThreads / 64) * 16 * kMlpBlocks * kShRow * sizeof(P);
    // rows start 16-byte aligned when the array does and 2L 16-bit values are a multiple of 16 bytes
    const bool vec = (reinterpret_cast<uintptr_t>(enc) & 15) == 0 && (c.n_levels % 4) == 0;
    auto kern = vec ? k_mlp_enc<P, LPG, true> : k_mlp_enc<P, LPG, false>;
    const int64_t per_wg = (kThreads / 64) * 16 * kMlpBlocks;  // rays per workgroup step
    const int64_t blocks = (n + per_wg - 1) / per_wg;
    const unsigned grid = unsigned(std::min<int64_t>(blocks, resident_grid(kern, lds)));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, c, reinterpret_cast<const P*>(enc), dir, n, rgba);
}

// Levels per lane group (ceil(L / 4)) selects the instantiation.
// The gradient kernel keeps the whole weight gradient in registers, which
// fits for up to 16 levels.
#define INRF_LPG_SWITCH_BACKWARD(L, CALL)                             \
    switch ((L + 3) / 4) {                                            \
        case 1: CALL(1); break;                                       \
        case 2: CALL(2); break;                                       \
        case 3: CALL(3); break;                                       \
        case 4: CALL(4); break;                                       \
        default: fail(INRF_E_UNSUPPORTED, "the gradient supports at most 16 levels"); \
    }

#define INRF_LPG_SWITCH(L, CALL)                              \
    switch ((L + 3) / 4) {                                    \
        case 1: CALL(1); break;                               \
        case 2: CALL(2); break;                               \
        case 3: CALL(3); break;                               \
        case 4: CALL(4); break;                               \
        case 5: CALL(5); break;                               \
        case 6: CALL(6); break;                               \
        case 7: CALL(7); break;                               \
        case 8: CALL(8); break;                               \
        default: fail(INRF_E_UNSUPPORTED, "level count");     \
    }

// HitRec records, or the CamHit records of camera *cam's frame.
template <class TableT>
void launch_shade(const ModelC& c, int32_t precision, const void* recs, const int32_t* first,
                  const int32_t* counter, float* rgba, hipStream_t s, const CamC* cam = nullptr) {
    CamC none{};
    const CamC& k = cam ? *cam : none;
#define INRF_SHADE(LPG)                                                                                      \
    do {                                                                                                    \
        if (precision == INRF_PREC_FP32) launch_shade_t<TableT, float, LPG>(c, recs, k, first, counter, rgba, s); \
        else if (precision == INRF_PREC_FP16)                                                               \
            launch_shade_t<TableT, _Float16, LPG>(c, recs, k, first, counter, rgba, s);                     \
        else launch_shade_t<TableT, __bf16, LPG>(c, recs, k, first, counter, rgba, s);                      \
    } while (0)
    INRF_LPG_SWITCH(c.n_levels, INRF_SHADE)
#undef INRF_SHADE
}

// Every object of a scene in one shading launch (k_shade_scene); the
// objects share the table type, and LPG covers the largest level count.
template <class TableT, class P, int LPG>
void launch_shade_scene_t(const ShadeSet& ss, const HitRec* recs, const int32_t* seg, float* rgba, hipStream_t s) {
    const size_t lds = ShadeShape<P, LPG>::lds_bytes;
    auto kern = k_shade_scene<TableT, P, LPG>;
    hipLaunchKernelGGL(kern, dim3(resident_grid(kern, lds)), dim3(kThreads), lds, s, ss, recs, seg, rgba);
}

template <class TableT>
void launch_shade_scene(const ShadeSet& ss, int max_levels, int32_t precision, const HitRec* recs, const int32_t* seg,
                        float* rgba, hipStream_t s) {
#define INRF_SHADE_SCENE(LPG)                                                                        \
    do {                                                                                            \
        if (precision == INRF_PREC_FP32) launch_shade_scene_t<TableT, float, LPG>(ss, recs, seg, rgba, s); \
        else if (precision == INRF_PREC_FP16)                                                       \
            launch_shade_scene_t<TableT, _Float16, LPG>(ss, recs, seg, rgba, s);                    \
        else launch_shade_scene_t<TableT, __bf16, LPG>(ss, recs, seg, rgba, s);                     \
    } while (0)
    switch ((max_levels + 3) / 4) {
        case 1: INRF_SHADE_SCENE(1); break;
        case 2: INRF_SHADE_SCENE(2); break;
        case 3: INRF_SHADE_SCENE(3); break;
        default: fail(INRF_E_UNSUPPORTED, "level count");
    }
#undef INRF_SHADE_SCENE
}

void check_precision(int32_t p) {
    require(p == INRF_PREC_FP32 || p == INRF_PREC_FP16 || p == INRF_PREC_BF16, "unknown precision");
}

void record(void* const* events, int i, hipStream_t s) {
    if (events && events[i]) check_hip(hipEventRecord(reinterpret_cast<hipEvent_t>(events[i]), s), "hipEventRecord");
}

// Screen bins of one camera frame in the workspace (bin_device.hpp).
// Returns false (the frame then walks the BVH) when the camera basis is too
// close to singular for the projection to be conservative.
bool make_bins(const CamC& cam, void* ws, const WsLayout& L, BinsC& b) {
    std::memset(&b, 0, sizeof(b));
    const double r[3] = {cam.r[0], cam.r[1], cam.r[2]}, u[3] = {cam.u[0], cam.u[1], cam.u[2]},
                 f[3] = {cam.f[0], cam.f[1], cam.f[2]};
    // inverse of the matrix with columns r, u, f: rows (u x f, f x r, r x u) / det
    const double uf[3] = {u[1] * f[2] - u[2] * f[1], u[2] * f[0] - u[0] * f[2], u[0] * f[1] - u[1] * f[0]};
    const double fr[3] = {f[1] * r[2] - f[2] * r[1], f[2] * r[0] - f[0] * r[2], f[0] * r[1] - f[1] * r[0]};
    const double ru[3] = {r[1] * u[2] - r[2] * u[1], r[2] * u[0] - r[0] * u[2], r[0] * u[1] - r[1] * u[0]};
    const double det = r[0] * uf[0] + r[1] * uf[1] + r[2] * uf[2];
    const auto norm = [](const double* v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
    const double scale = norm(r) * norm(u) * norm(f);
    if (!(std::fabs(det) > 1e-3 * scale) || !std::isfinite(det)) return false;
    for (int k = 0; k < 3; ++k) {
        b.a[k] = float(uf[k] / det);
        b.a[3 + k] = float(fr[k] / det);
        b.a[6 + k] = float(ru[k] / det);
        b.o[k] = cam.o[k];
        if (!std::isfinite(b.a[k]) || !std::isfinite(b.a[3 + k]) || !std::isfinite(b.a[6 + k]) ||
            !std::isfinite(b.o[k]))
            return false;
    }
    b.sjx = float(double(cam.W) / (2.0 * double(cam.tan_x)));
    b.sjb = float(0.5 * double(cam.W) - 0.5);
    b.siy = float(-double(cam.H) / (2.0 * double(cam.tan_y)));
    b.sib = float(0.5 * double(cam.H) - 0.5);
    b.W = cam.W;
    b.H = cam.H;
    b.QX = (cam.W + kQuad - 1) / kQuad;
    b.QY = (cam.H + kQuad - 1) / kQuad;
    if (int64_t(b.QX) * b.QY > L.n_quads) return false;
    b.cnt = ws_at<int32_t>(ws, L.qcnt);
    b.fcnt = ws_at<int32_t>(ws, L.qfcnt);
    b.total = ws_at<int32_t>(ws, L.qtotal);
    b.entries = ws_at<int2>(ws, L.entries);
    b.base = ws_at<int32_t>(ws, L.qbase);
    b.scnt = ws_at<int32_t>(ws, L.qscnt);
    b.sfcnt = ws_at<int32_t>(ws, L.qsfcnt);
    b.top = ws_at<unsigned long long>(ws, L.qtop);
    b.spill = ws_at<int2>(ws, L.spill);
    b.spill_cap = int32_t(L.n_spill);
    // distance bound per unit of lambda: t >= lambda / |a_f| for unit rays
    const double af = std::sqrt(double(b.a[6]) * b.a[6] + double(b.a[7]) * b.a[7] + double(b.a[8]) * b.a[8]);
    b.tscale = float((1.0 - 1e-4) / af);
    return true;
}

// Sorts the proxy's triangles into the frame's quadrant lists: clear, fill,
// spill lists for the quadrants that overflowed, their fill.
void bin_frame(const ModelC& c, const BinsC& b, hipStream_t s) {
    const int nq = b.QX * b.QY;
    const unsigned qgrid = unsigned((nq + 255) / 256), tgrid = unsigned((c.n_tris + 255) / 256);
    hipLaunchKernelGGL(k_bin_clear, dim3(qgrid), dim3(256), 0, s, b);
    launch_check("k_bin_clear");
    if (c.n_tris == 0) return;
    hipLaunchKernelGGL(k_bin, dim3(tgrid), dim3(256), 0, s, b, c.tris, c.n_tris);
    launch_check("k_bin");
    hipLaunchKernelGGL(k_spill_alloc, dim3(qgrid), dim3(256), 0, s, b);
    launch_check("k_spill_alloc");
    hipLaunchKernelGGL(k_bin_spill, dim3(tgrid), dim3(256), 0, s, b, c.tris, c.n_tris);
    launch_check("k_bin_spill");
}

// Clears the hit counter, then traces n rays (camera rays when cam is set),
// writing depth / triangle / zero colour of misses and appending hit records.
// Launches k_trace, one workgroup per tile (cameras) or 256-ray block
// (batch); returns the number of workgroups.
template <int NCAM>
int launch_trace(const ModelC& c, const CamSet<NCAM>* cams, const TraceArgs& a, int64_t n, hipStream_t s,
                 const BinsC* bins) {
    BinsC none_b;
    std::memset(&none_b, 0, sizeof(none_b));
    if (cams) {
        const CamC& last = cams->c[cams->n - 1];
        const int n_blk = last.tile0 + last.tiles_x * ((last.H + kTile - 1) / kTile);
        if constexpr (NCAM == 1) {
            if (bins) {
                hipLaunchKernelGGL((k_trace<true, 1, true>), dim3(n_blk), dim3(kThreads), 0, s, c, *cams, a, *bins);
                launch_check("k_trace");
                return n_blk;
            }
        }
        hipLaunchKernelGGL((k_trace<true, NCAM>), dim3(n_blk), dim3(kThreads), 0, s, c, *cams, a, none_b);
        launch_check("k_trace");
        return n_blk;
    }
    CamSet<1> none;
    std::memset(&none, 0, sizeof(none));
    const int n_blk = int((n + kThreads - 1) / kThreads);
    const size_t stack_bytes = size_t(c.stack_depth) * kThreads * sizeof(int);
    hipLaunchKernelGGL((k_trace<false, 1>), dim3(n_blk), dim3(kThreads), stack_bytes, s, c, none, a, none_b);
    launch_check("k_trace");
    return n_blk;
}

// Traces n rays (camera rays when cam is set), writing depth / triangle /
// zero colour of misses, then packs the hit records into one list in
// workgroup order and writes its length to the counter.
template <int NCAM>
void trace_to_hits(const ModelC& c, const CamSet<NCAM>* cams, const float* ray_o, const float* ray_d, int64_t n,
                   float* rgba, float* depth, int32_t* tri, void* ws, hipStream_t s, const BinsC* bins = nullptr) {
    const WsLayout L(n, cams ? 2 * int64_t(cams->n - 1) : 0);
    int32_t* counter = ws_at<int32_t>(ws, 0);
    HitRec* recs = ws_at<HitRec>(ws, L.recs);
    int2* blk = ws_at<int2>(ws, L.blk);
    int32_t* offsets = ws_at<int32_t>(ws, L.offsets);
    int32_t* runs = ws_at<int32_t>(ws, L.runs);
    TraceArgs a{ray_o, ray_d, n, rgba, depth, tri, ws_at<HitRec>(ws, L.tmp), blk};
    const int n_blk = launch_trace(c, cams, a, n, s, bins);
    const int n_runs = (n_blk + kScanRun - 1) / kScanRun;
    hipLaunchKernelGGL(k_scan_local, dim3(n_runs), dim3(kScanThreads), 0, s, reinterpret_cast<const int32_t*>(blk), 2, n_blk, offsets, runs, INT32_MAX);
    launch_check("k_scan_local");
    hipLaunchKernelGGL(k_scan_runs, dim3(1), dim3(kScanThreads), 0, s, runs, n_runs, counter, counter + 1,
                       kMaxChunks - 1);
    launch_check("k_scan_runs");
    const dim3 cgrid(unsigned((n_blk + kThreads / 64 - 1) / (kThreads / 64)));
    if (cams && NCAM == 1)
        hipLaunchKernelGGL(k_compact_runs<CamHit>, cgrid, dim3(kThreads), 0, s, blk, offsets, runs,
                           static_cast<const CamHit*>(a.tmp), ws_at<CamHit>(ws, L.recs), n_blk);
    else
        hipLaunchKernelGGL(k_compact_runs<HitRec>, cgrid, dim3(kThreads), 0, s, blk, offsets, runs,
                           static_cast<const HitRec*>(a.tmp), recs, n_blk);
    launch_check("k_compact");
}

template <int NCAM>
void run_path(const inrf_model* m, int32_t precision, const CamSet<NCAM>* cams, const float* ray_o,
              const float* ray_d, int64_t n, float* rgba, float* depth, int32_t* tri, void* ws, int64_t ws_bytes,
              void* stream, void* const* events = nullptr) {
    check_precision(precision);
    const ModelC c = make_model(m, true, true);
    require(m->weights != nullptr, "weights must be set");
    if (n == 0) return;
    require(rgba != nullptr, "rgba is NULL");
    require(ws != nullptr, "workspace is NULL");
    require((reinterpret_cast<uintptr_t>(ws) & 15) == 0 && (reinterpret_cast<uintptr_t>(rgba) & 15) == 0,
            "rgba and workspace must be 16-byte aligned");
    const WsLayout L(n, cams ? 2 * int64_t(cams->n - 1) : 0);
    if (ws_bytes < L.end)
        fail(INRF_E_SIZE, "workspace of " + std::to_string(ws_bytes) + " bytes < " + std::to_string(L.end) +
                              " needed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // a single camera's frame is traced through screen bins of the proxy
    BinsC bins_v;
    const BinsC* bins = nullptr;
    if constexpr (NCAM == 1) {
        if (cams && make_bins(cams->c[0], ws, L, bins_v)) bins = &bins_v;
    }
    record(events, 0, s);
    if (bins) bin_frame(c, *bins, s);
    const int32_t* counter = ws_at<int32_t>(ws, 0);
    const HitRec* recs = ws_at<HitRec>(ws, L.recs);
    trace_to_hits(c, cams, ray_o, ray_d, n, rgba, depth, tri, ws, s, bins);
    record(events, 1, s);
    // a single camera's records are CamHit records
    const CamC* rec_cam = (cams && NCAM == 1) ? &cams->c[0] : nullptr;
    if (c.table_dtype == INRF_F32) launch_shade<float>(c, precision, recs, nullptr, counter, rgba, s, rec_cam);
    else launch_shade<__half>(c, precision, recs, nullptr, counter, rgba, s, rec_cam);
    launch_check("k_shade");
    record(events, 2, s);
}

// ---- gradient (k_backward)

// Workgroups of the backward launch (one weight-gradient partial each): as
// many as the device keeps resident.
template <class TableT, int LPG>
unsigned backward_grid_t() {
    const size_t lds = BackShape<LPG>::lds_bytes;
    auto kern = k_backward<TableT, LPG>;
    return resident_grid(kern, lds);
}

unsigned backward_grid(const ModelC& c) {
    unsigned g = 0;
#define INRF_BGRID(LPG) \
    g = c.table_dtype == INRF_F32 ? backward_grid_t<float, LPG>() : backward_grid_t<__half, LPG>()
    INRF_LPG_SWITCH_BACKWARD(c.n_levels, INRF_BGRID)
#undef INRF_BGRID
    return g;
}

int64_t backward_ws_bytes(const ModelC& c, int64_t n) {
    return WsLayout(n).end + int64_t(backward_grid(c)) * weight_count(c.n_levels) * int64_t(sizeof(float));
}

template <class TableT, int LPG>
void launch_backward_t(const ModelC& c, unsigned grid, const HitRec* recs, const int32_t* counter,
                       const float* d_rgba, float* d_table, float* partial, float* rgba, hipStream_t s) {
    const size_t lds = BackShape<LPG>::lds_bytes;
    hipLaunchKernelGGL((k_backward<TableT, LPG>), dim3(grid), dim3(kThreads), lds, s, c, recs, counter, d_rgba,
                       d_table, partial, rgba);
}

void run_backward(const inrf_model* m, const float* ray_o, const float* ray_d, int64_t n, const float* d_rgba,
                  float* d_table, float* d_weights, float* rgba, void* ws, int64_t ws_bytes, void* stream) {
    const ModelC c = make_model(m, true, true);
    require(m->weights != nullptr, "weights must be set");
    require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31)");
    if (n == 0) return;
    require(ray_o && ray_d && d_rgba, "ray and gradient buffers must be set");
    require(ws != nullptr, "workspace is NULL");
    require((reinterpret_cast<uintptr_t>(ws) & 255) == 0, "workspace must be 256-byte aligned");
    require((reinterpret_cast<uintptr_t>(d_rgba) & 15) == 0 && (reinterpret_cast<uintptr_t>(rgba) & 15) == 0,
            "d_rgba and rgba must be 16-byte aligned");
    require((reinterpret_cast<uintptr_t>(d_table) & 7) == 0, "d_table must be 8-byte aligned");
    const unsigned grid = backward_grid(c);
    const int64_t need = backward_ws_bytes(c, n);
    if (ws_bytes < need)
        fail(INRF_E_SIZE,
             "workspace of " + std::to_string(ws_bytes) + " bytes < " + std::to_string(need) + " needed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int32_t* counter = ws_at<int32_t>(ws, 0);
    const HitRec* recs = ws_at<HitRec>(ws, WsLayout(n).recs);
    float* partial = ws_at<float>(ws, WsLayout(n).end);
    trace_to_hits<1>(c, nullptr, ray_o, ray_d, n, rgba, nullptr, nullptr, ws, s);
#define INRF_BACK(LPG)                                                                                   \
    do {                                                                                                \
        if (c.table_dtype == INRF_F32)                                                                  \
            launch_backward_t<float, LPG>(c, grid, recs, counter, d_rgba, d_table, partial, rgba, s);  \
        else launch_backward_t<__half, LPG>(c, grid, recs, counter, d_rgba, d_table, partial, rgba, s); \
    } while (0)
    INRF_LPG_SWITCH_BACKWARD(c.n_levels, INRF_BACK)
#undef INRF_BACK
    launch_check("k_backward");
    if (d_weights) {
        const int nw = weight_count(c.n_levels);
        hipLaunchKernelGGL(k_reduce_partials, dim3((nw + 255) / 256), dim3(256), 0, s, partial, int(grid), nw,
                           d_weights);
        launch_check("k_reduce_partials");
    }
}

CamC make_camera(const inrf_camera* cam) {
    require(cam != nullptr, "camera is NULL");
    require(cam->width >= 1 && cam->height >= 1, "image size must be positive");
    require(int64_t(cam->width) * cam->height <= (int64_t(1) << 31) - 1, "image too large");
    CamC c;
    for (int k = 0; k < 3; ++k) {
        c.o[k] = cam->origin[k];
        c.r[k] = cam->right[k];
        c.u[k] = cam->up[k];
        c.f[k] = cam->forward[k];
    }
    require(std::isfinite(cam->tan_half_fov_y) && cam->tan_half_fov_y > 0.f, "tan_half_fov_y must be > 0");
    c.tan_y = cam->tan_half_fov_y;
    c.tan_x = cam->tan_half_fov_y * float(cam->width) / float(cam->height);
    c.W = cam->width;
    c.H = cam->height;
    c.tiles_x = (cam->width + kTile - 1) / kTile;
    c.tile0 = 0;
    c.pix0 = 0;
    return c;
}

// ---- scenes (k_trace_scene)

// Workspace of a scene render of up to n rays and K objects: counter |
// records | per-tile records | [K][tiles] (count, first) | offsets | runs |
// K + 1 run starts.
struct SceneWs {
    int64_t recs, tmp, blk, offsets, runs, seg, end;
    // extra: 2 more tiles per additional camera of a batch
    SceneWs(int64_t n, int k, int64_t extra = 0) {
        const int64_t nb = int64_t(std::max(k, 1)) * (n / 8 + 2 + extra), nr = nb / kScanRun + 1;
        recs = kWsHeader;
        tmp = align256(recs + n * int64_t(sizeof(HitRec)));
        blk = align256(tmp + n * int64_t(sizeof(HitRec)));
        offsets = align256(blk + nb * int64_t(sizeof(int2)));
        runs = align256(offsets + nb * int64_t(sizeof(int32_t)));
        seg = align256(runs + nr * int64_t(sizeof(int32_t)));
        end = align256(seg + (k + 1) * int64_t(sizeof(int32_t)));
    }
};

void make_object(const inrf_instance& in, ObjC& o) {
    require(in.model != nullptr, "instance model is NULL");
    const float s = in.scale;
    require(std::isfinite(s) && s > 0.f, "instance scale must be finite and > 0");
    const float* R = in.rotation;
    for (int i = 0; i < 9; ++i) require(std::isfinite(R[i]), "non-finite rotation");
    for (int i = 0; i < 3; ++i) require(std::isfinite(in.translation[i]), "non-finite translation");
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dot = 0;
            for (int k = 0; k < 3; ++k) dot += double(R[3 * i + k]) * R[3 * j + k];
            require(std::fabs(dot - (i == j ? 1.0 : 0.0)) < 1e-4, "rotation must be orthonormal");
        }
    const double det = double(R[0]) * (double(R[4]) * R[8] - double(R[5]) * R[7]) -
                       double(R[1]) * (double(R[3]) * R[8] - double(R[5]) * R[6]) +
                       double(R[2]) * (double(R[3]) * R[7] - double(R[4]) * R[6]);
    require(det > 0.0, "rotation must have determinant +1");
    // world -> object: x_o = R^T (x_w - t) / s
    for (int i = 0; i < 3; ++i) {
        double c = 0;
        for (int j = 0; j < 3; ++j) {
            o.m[3 * i + j] = float(double(R[3 * j + i]) / s);
            c -= double(R[3 * j + i]) * in.translation[j];
        }
        o.c[i] = float(c / s);
    }
    // world bounds of the unit cube, widened by a relative 1e-6 for rounding
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int corner = 0; corner < 8; ++corner) {
        const double x[3] = {double(corner & 1), double((corner >> 1) & 1), double((corner >> 2) & 1)};
        for (int i = 0; i < 3; ++i) {
            double w = in.translation[i];
            for (int j = 0; j < 3; ++j) w += double(s) * R[3 * i + j] * x[j];
            lo[i] = std::min(lo[i], w);
            hi[i] = std::max(hi[i], w);
        }
    }
    for (int i = 0; i < 3; ++i) {
        const double pad = 1e-6 * (std::fabs(lo[i]) + std::fabs(hi[i]) + s);
        o.lo[i] = float(lo[i] - pad);
        o.hi[i] = float(hi[i] + pad);
    }
}

template <int NCAM>
void run_scene(const inrf_instance* objects, int32_t n_objs, int32_t precision, const CamSet<NCAM>& cams,
               float* rgba, float* depth, int32_t* tri, int32_t* obj, void* ws, int64_t ws_bytes, void* stream) {
    check_precision(precision);
    require(n_objs >= 0 && n_objs <= kMaxObjects, "n_objects must be in [0, INRF_MAX_OBJECTS]");
    require(n_objs == 0 || objects != nullptr, "objects is NULL");
    const CamC& last = cams.c[cams.n - 1];
    const int64_t n = last.pix0 + int64_t(last.W) * last.H;
    require(rgba != nullptr && ws != nullptr, "rgba and workspace must be set");
    require((reinterpret_cast<uintptr_t>(ws) & 255) == 0 && (reinterpret_cast<uintptr_t>(rgba) & 15) == 0,
            "workspace must be 256-byte and rgba 16-byte aligned");
    const SceneWs L(n, n_objs, 2 * int64_t(cams.n - 1));
    if (ws_bytes < L.end)
        fail(INRF_E_SIZE, "workspace of " + std::to_string(ws_bytes) + " bytes < " + std::to_string(L.end) + " needed");
    SceneC sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.n_objs = n_objs;
    std::vector<ModelC> models(static_cast<size_t>(n_objs));
    for (int k = 0; k < n_objs; ++k) {
        models[size_t(k)] = make_model(objects[k].model, true, true);
        require(objects[k].model->weights != nullptr, "instance weights must be set");
        make_object(objects[k], sc.o[k]);
        sc.o[k].nodes = models[size_t(k)].nodes;
        sc.o[k].tris = models[size_t(k)].tris;
        sc.o[k].n_tris = int32_t(models[size_t(k)].n_tris);
        sc.o[k].stack_depth = models[size_t(k)].stack_depth;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t* counter = ws_at<int32_t>(ws, 0);
    HitRec* recs = ws_at<HitRec>(ws, L.recs);
    int2* blk = ws_at<int2>(ws, L.blk);
    int32_t* offsets = ws_at<int32_t>(ws, L.offsets);
    int32_t* runs = ws_at<int32_t>(ws, L.runs);
    int32_t* seg = ws_at<int32_t>(ws, L.seg);
    const int n_tiles = last.tile0 + last.tiles_x * ((last.H + kTile - 1) / kTile);
    const SceneArgs a{rgba, depth, tri, obj, ws_at<HitRec>(ws, L.tmp), blk};
    hipLaunchKernelGGL(k_trace_scene<NCAM>, dim3(n_tiles), dim3(kThreads), 0, s, sc, cams, a, n_tiles);
    launch_check("k_trace_scene");
    if (n_objs == 0) return;
    const int n_blk = n_objs * n_tiles;
    const int n_runs = (n_blk + kScanRun - 1) / kScanRun;
    hipLaunchKernelGGL(k_scan_local, dim3(n_runs), dim3(kScanThreads), 0, s, reinterpret_cast<const int32_t*>(blk), 2, n_blk, offsets, runs, INT32_MAX);
    launch_check("k_scan_local");
    hipLaunchKernelGGL(k_scan_runs, dim3(1), dim3(kScanThreads), 0, s, runs, n_runs, counter, counter + 1,
                       kMaxChunks - 1);
    launch_check("k_scan_runs");
    hipLaunchKernelGGL(k_compact<HitRec>, dim3(n_tiles), dim3(kThreads), 0, s, blk, offsets, runs,
                       static_cast<const HitRec*>(a.tmp), recs, n_objs, n_tiles);
    launch_check("k_compact");
    hipLaunchKernelGGL(k_segments, dim3(1), dim3(64), 0, s, offsets, runs, n_tiles, n_objs, counter, seg);
    launch_check("k_segments");
    // one shading launch for all objects when they share the table type and
    // have at most 12 levels (the kernel argument's level tables), else one
    // launch per object over its run of records
    bool together = true;
    int max_levels = 1;
    for (int k = 0; k < n_objs; ++k) {
        together = together && models[size_t(k)].n_levels <= kSceneShadeLevels &&
                   models[size_t(k)].table_dtype == models[0].table_dtype;
        max_levels = std::max(max_levels, int(models[size_t(k)].n_levels));
    }
    if (together) {
        ShadeSet ss;
        std::memset(&ss, 0, sizeof(ss));
        ss.n = n_objs;
        for (int k = 0; k < n_objs; ++k) {
            const ModelC& c = models[size_t(k)];
            ss.m[k].n_levels = c.n_levels;
            ss.m[k].phi = c.phi;
            ss.m[k].table = c.table;
            ss.m[k].weights = c.weights;
            for (int l = 0; l < c.n_levels; ++l) ss.m[k].lv[l] = c.lv[l];
        }
        if (models[0].table_dtype == INRF_F32) launch_shade_scene<float>(ss, max_levels, precision, recs, seg, rgba, s);
        else launch_shade_scene<__half>(ss, max_levels, precision, recs, seg, rgba, s);
        launch_check("k_shade_scene");
        return;
    }
    for (int k = 0; k < n_objs; ++k) {
        const ModelC& c = models[size_t(k)];
        if (c.table_dtype == INRF_F32) launch_shade<float>(c, precision, recs, seg + k, seg + k + 1, rgba, s);
        else launch_shade<__half>(c, precision, recs, seg + k, seg + k + 1, rgba, s);
        launch_check("k_shade");
    }
}

// ---- the i-NOLF form (k_march)

bool pow2(int32_t v) { return v >= 1 && (v & (v - 1)) == 0; }

CubesC make_cubes(const inrf_cubes* q) {
    require(q != nullptr, "cubes is NULL");
    require(pow2(q->base_res) && q->base_res <= 1024, "base_res must be a power of two in [1, 1024]");
    require(pow2(q->cube_res) && q->cube_res <= 64, "cube_res must be a power of two in [1, 64]");
    require(q->index && q->density && q->diffuse, "cube index, density and diffuse must be set");
    require((reinterpret_cast<uintptr_t>(q->diffuse) & 7) == 0 && (reinterpret_cast<uintptr_t>(q->density) & 1) == 0 &&
                (reinterpret_cast<uintptr_t>(q->index) & 3) == 0,
            "cube arrays must be aligned (diffuse to 8 bytes)");
    require(q->n_cubes >= 1, "n_cubes must be >= 1");
    require(std::isfinite(q->step) && q->step >= 1e-6f && q->step <= 1.f, "step must be in [1e-6, 1]");
    require(q->t_stop > 0.f && q->t_stop < 1.f, "t_stop must be in (0, 1)");
    require(std::isfinite(q->w_min) && q->w_min > 0.f && q->w_min <= 1.f, "w_min must be in (0, 1]");
    CubesC C;
    std::memset(&C, 0, sizeof(C));
    C.index = q->index;
    C.dens = reinterpret_cast<const __half*>(q->density);
    C.diff = reinterpret_cast<const __half*>(q->diffuse);
    C.n_cubes = q->n_cubes;
    C.b = q->base_res;
    C.r = q->cube_res;
    C.r1 = q->cube_res + 1;
    C.fb = float(q->base_res);
    C.fr = float(q->cube_res);
    C.step = q->step;
    C.t_stop = q->t_stop;
    C.w_min = q->w_min;
    C.j_max = int32_t(std::ceil(1.7320509 / double(q->step))) + 2;  // the cube's diagonal holds fewer samples
    return C;
}

template <class TableT, class P, int LPG>
void launch_shade_nolf_t(const ModelC& c, const HitRec* recs, const int32_t* counter, float* rgba, hipStream_t s) {
    const size_t lds = ShadeShape<P, LPG, 1>::lds_bytes;
    auto kern = k_shade<TableT, P, LPG, true>;
    hipLaunchKernelGGL(kern, dim3(resident_grid(kern, lds)), dim3(kThreads), lds, s, c, static_cast<const void*>(recs),
                       CamC{}, nullptr, counter, rgba);
}

template <class TableT>
void launch_shade_nolf(const ModelC& c, int32_t precision, const HitRec* recs, const int32_t* counter, float* rgba,
                       hipStream_t s) {
#define INRF_SHADE_NOLF(LPG)                                                                                 \
    do {                                                                                                    \
        if (precision == INRF_PREC_FP32) launch_shade_nolf_t<TableT, float, LPG>(c, recs, counter, rgba, s); \
        else if (precision == INRF_PREC_FP16)                                                               \
            launch_shade_nolf_t<TableT, _Float16, LPG>(c, recs, counter, rgba, s);                          \
        else launch_shade_nolf_t<TableT, __bf16, LPG>(c, recs, counter, rgba, s);                           \
    } while (0)
    switch ((c.n_levels + 3) / 4) {
        case 1: INRF_SHADE_NOLF(1); break;
        case 2: INRF_SHADE_NOLF(2); break;
        default: fail(INRF_E_UNSUPPORTED, "the i-NOLF form supports at most 8 levels");
    }
#undef INRF_SHADE_NOLF
}

void run_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision, const inrf_camera* camera, float* rgba,
              float* depth, float* alpha_c, void* ws, int64_t ws_bytes, void* stream) {
    check_precision(precision);
    const ModelC c = make_model(m, true, false);
    require(m->weights != nullptr, "weights must be set");
    if (c.n_levels > 8) fail(INRF_E_UNSUPPORTED, "the i-NOLF form supports at most 8 levels");
    const CubesC C = make_cubes(cubes);
    const CamC cam = make_camera(camera);
    const int64_t n = int64_t(cam.W) * cam.H;
    require(rgba != nullptr && ws != nullptr, "rgba and workspace must be set");
    require((reinterpret_cast<uintptr_t>(ws) & 255) == 0 && (reinterpret_cast<uintptr_t>(rgba) & 15) == 0,
            "workspace must be 256-byte and rgba 16-byte aligned");
    const WsLayout L(n);
    if (ws_bytes < L.end)
        fail(INRF_E_SIZE, "workspace of " + std::to_string(ws_bytes) + " bytes < " + std::to_string(L.end) + " needed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t* counter = ws_at<int32_t>(ws, 0);
    HitRec* recs = ws_at<HitRec>(ws, L.recs);
    int2* blk = ws_at<int2>(ws, L.blk);
    int32_t* offsets = ws_at<int32_t>(ws, L.offsets);
    int32_t* runs = ws_at<int32_t>(ws, L.runs);
    const int n_blk = cam.tiles_x * ((cam.H + kTile - 1) / kTile);
    // macro-cell flags go to the record area, unused until k_compact, when
    // it has room and the base grid divides into macro cells
    const int bm = C.b / kMacro;
    uint8_t* macro = nullptr;
    if (C.b % kMacro == 0 && int64_t(bm) * bm * bm <= n * int64_t(sizeof(HitRec))) {
        macro = ws_at<uint8_t>(ws, L.recs);
        hipLaunchKernelGGL(k_cube_macro, dim3(unsigned((bm * bm * bm + 255) / 256)), dim3(256), 0, s, C.index, C.b,
                           macro);
        launch_check("k_cube_macro");
    }
    const MarchArgs a{rgba, depth, alpha_c, ws_at<HitRec>(ws, L.tmp), blk, macro};
    hipLaunchKernelGGL(k_march, dim3(n_blk), dim3(kThreads), 0, s, C, cam, a);
    launch_check("k_march");
    const int n_runs = (n_blk + kScanRun - 1) / kScanRun;
    hipLaunchKernelGGL(k_scan_local, dim3(n_runs), dim3(kScanThreads), 0, s, reinterpret_cast<const int32_t*>(blk), 2, n_blk, offsets, runs, INT32_MAX);
    launch_check("k_scan_local");
    hipLaunchKernelGGL(k_scan_runs, dim3(1), dim3(kScanThreads), 0, s, runs, n_runs, counter, counter + 1,
                       kMaxChunks - 1);
    launch_check("k_scan_runs");
    hipLaunchKernelGGL(k_compact<HitRec>, dim3(n_blk), dim3(kThreads), 0, s, blk, offsets, runs,
                       static_cast<const HitRec*>(a.tmp), recs, 1, n_blk);
    launch_check("k_compact");
    if (c.table_dtype == INRF_F32) launch_shade_nolf<float>(c, precision, recs, counter, rgba, s);
    else launch_shade_nolf<__half>(c, precision, recs, counter, rgba, s);
    launch_check("k_shade");
}

void run_shade_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision, const float* x, const float* d,
                    const float* alpha_c, int64_t n, float* rgba, void* ws, int64_t ws_bytes, void* stream) {
    check_precision(precision);
    const ModelC c = make_model(m, true, false);
    require(m->weights != nullptr, "weights must be set");
    if (c.n_levels > 8) fail(INRF_E_UNSUPPORTED, "the i-NOLF form supports at most 8 levels");
    const CubesC C = make_cubes(cubes);
    require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31 - 1]");
    if (n == 0) return;
    require(x && d && alpha_c && rgba && ws, "x, d, alpha_c, rgba and workspace must be set");
    require((reinterpret_cast<uintptr_t>(ws) & 255) == 0 && (reinterpret_cast<uintptr_t>(rgba) & 15) == 0,
            "workspace must be 256-byte and rgba 16-byte aligned");
    const WsLayout L(n);
    if (ws_bytes < L.end)
        fail(INRF_E_SIZE, "workspace of " + std::to_string(ws_bytes) + " bytes < " + std::to_string(L.end) + " needed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t* counter = ws_at<int32_t>(ws, 0);
    HitRec* recs = ws_at<HitRec>(ws, L.recs);
    hipLaunchKernelGGL(k_nolf_points, dim3(unsigned((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, C, x, d,
                       alpha_c, n, rgba, recs, counter);
    launch_check("k_nolf_points");
    if (c.table_dtype == INRF_F32) launch_shade_nolf<float>(c, precision, recs, counter, rgba, s);
    else launch_shade_nolf<__half>(c, precision, recs, counter, rgba, s);
    launch_check("k_shade");
}

void run_camera_rays(const inrf_camera* camera, float* ray_o, float* ray_d, void* stream) {
    const CamC cam = make_camera(camera);
    require(ray_d != nullptr, "ray_d must be set");
    const int64_t n = int64_t(cam.W) * cam.H;
    hipLaunchKernelGGL(k_camera_rays, dim3(unsigned((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       reinterpret_cast<hipStream_t>(stream), cam, ray_o, ray_d);
    launch_check("k_camera_rays");
}

}  // namespace
}  // namespace inrf

using namespace inrf;

extern "C" {

int64_t inrf_workspace_size(int64_t n_rays) {
    if (n_rays < 0) return -1;
    return WsLayout(n_rays).end;
}

inrf_status inrf_render_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision, const inrf_camera* cam,
                             float* rgba, float* depth, float* alpha_c, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_render_nolf",
                   [&] { run_nolf(m, cubes, precision, cam, rgba, depth, alpha_c, ws, ws_bytes, stream); });
}

inrf_status inrf_shade_nolf(const inrf_model* m, const inrf_cubes* cubes, int32_t precision, const float* x,
                            const float* d, const float* alpha_c, int64_t n, float* rgba, void* ws, int64_t ws_bytes,
                            void* stream) {
    return guarded("inrf_shade_nolf",
                   [&] { run_shade_nolf(m, cubes, precision, x, d, alpha_c, n, rgba, ws, ws_bytes, stream); });
}

inrf_status inrf_camera_rays(const inrf_camera* cam, float* ray_o, float* ray_d, void* stream) {
    return guarded("inrf_camera_rays", [&] { run_camera_rays(cam, ray_o, ray_d, stream); });
}

inrf_status inrf_render(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba, float* depth,
                        int32_t* tri, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_render", [&] {
        const dev::CamSet<1> cs{1, 0, {make_camera(cam)}};
        run_path(m, precision, &cs, nullptr, nullptr, int64_t(cs.c[0].W) * cs.c[0].H, rgba, depth, tri, ws, ws_bytes,
                 stream);
    });
}

inrf_status inrf_render_static(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba,
                               float* depth, int32_t* tri, void* stream) {
    return guarded("inrf_render_static", [&] {
        const dev::CamSet<1> cs{1, 0, {make_camera(cam)}};
        const int64_t n = int64_t(cs.c[0].W) * cs.c[0].H;
        if (n > INRF_STATIC_MAX_PIXELS)
            fail(INRF_E_SIZE, "inrf_render_static renders at most " + std::to_string(INRF_STATIC_MAX_PIXELS) +
                                  " pixels, got " + std::to_string(n));
        run_path(m, precision, &cs, nullptr, nullptr, n, rgba, depth, tri, static_scratch(), kStaticScratchBytes,
                 stream);
    });
}

inrf_status inrf_render_profiled(const inrf_model* m, int32_t precision, const inrf_camera* cam, float* rgba,
                                 float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream,
                                 void* const* events) {
    return guarded("inrf_render_profiled", [&] {
        const dev::CamSet<1> cs{1, 0, {make_camera(cam)}};
        run_path(m, precision, &cs, nullptr, nullptr, int64_t(cs.c[0].W) * cs.c[0].H, rgba, depth, tri, ws, ws_bytes,
                 stream, events);
    });
}

int64_t inrf_batch_workspace_size(int32_t n_cameras, int64_t n_pixels) {
    if (n_cameras < 1 || n_cameras > INRF_MAX_CAMERAS || n_pixels < 0) return -1;
    return WsLayout(n_pixels, 2 * int64_t(n_cameras - 1)).end;
}

inrf_status inrf_render_batch(const inrf_model* m, int32_t precision, const inrf_camera* cams, int32_t n_cameras,
                              float* rgba, float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_render_batch", [&] {
        require(n_cameras >= 1 && n_cameras <= INRF_MAX_CAMERAS, "n_cameras must be in [1, INRF_MAX_CAMERAS]");
        require(cams != nullptr, "cameras is NULL");
        dev::CamSet<dev::kMaxCameras> cs;
        std::memset(&cs, 0, sizeof(cs));
        cs.n = n_cameras;
        int64_t pix = 0, tiles = 0;
        for (int j = 0; j < n_cameras; ++j) {
            cs.c[j] = make_camera(&cams[j]);
            cs.c[j].tile0 = int32_t(tiles);
            cs.c[j].pix0 = pix;
            pix += int64_t(cs.c[j].W) * cs.c[j].H;
            tiles += int64_t(cs.c[j].tiles_x) * ((cs.c[j].H + dev::kTile - 1) / dev::kTile);
            require(pix <= (int64_t(1) << 31) - 1, "batch too large (2^31 pixels)");
        }
        run_path(m, precision, &cs, nullptr, nullptr, pix, rgba, depth, tri, ws, ws_bytes, stream);
    });
}

inrf_status inrf_forward(const inrf_model* m, int32_t precision, const float* ray_o, const float* ray_d, int64_t n,
                         float* rgba, float* depth, int32_t* tri, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_forward", [&] {
        require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31)");
        require(n == 0 || (ray_o && ray_d), "ray buffers are NULL");
        run_path<1>(m, precision, nullptr, ray_o, ray_d, n, rgba, depth, tri, ws, ws_bytes, stream);
    });
}

int64_t inrf_backward_workspace_size(const inrf_model* m, int64_t n_rays) {
    int64_t out = -1;
    const inrf_status st = guarded("inrf_backward_workspace_size", [&] {
        require(n_rays >= 0, "n_rays must be >= 0");
        out = backward_ws_bytes(make_model(m, false, false), n_rays);
    });
    return st == INRF_OK ? out : -1;
}

inrf_status inrf_backward(const inrf_model* m, const float* ray_o, const float* ray_d, int64_t n, const float* d_rgba,
                          float* d_table, float* d_weights, float* rgba, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_backward", [&] {
        run_backward(m, ray_o, ray_d, n, d_rgba, d_table, d_weights, rgba, ws, ws_bytes, stream);
    });
}

int64_t inrf_scene_workspace_size(int32_t n_objects, int64_t n_rays) {
    if (n_objects < 0 || n_objects > INRF_MAX_OBJECTS || n_rays < 0) return -1;
    return SceneWs(n_rays, n_objects).end;
}

inrf_status inrf_render_scene(const inrf_instance* objects, int32_t n_objects, int32_t precision,
                              const inrf_camera* cam, float* rgba, float* depth, int32_t* tri, int32_t* object,
                              void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_render_scene", [&] {
        const dev::CamSet<1> cs{1, 0, {make_camera(cam)}};
        run_scene<1>(objects, n_objects, precision, cs, rgba, depth, tri, object, ws, ws_bytes, stream);
    });
}

int64_t inrf_scene_batch_workspace_size(int32_t n_objects, int32_t n_cameras, int64_t n_pixels) {
    if (n_objects < 0 || n_objects > INRF_MAX_OBJECTS || n_cameras < 1 || n_cameras > INRF_MAX_CAMERAS ||
        n_pixels < 0)
        return -1;
    return SceneWs(n_pixels, n_objects, 2 * int64_t(n_cameras - 1)).end;
}

inrf_status inrf_render_scene_batch(const inrf_instance* objects, int32_t n_objects, int32_t precision,
                                    const inrf_camera* cams, int32_t n_cameras, float* rgba, float* depth,
                                    int32_t* tri, int32_t* object, void* ws, int64_t ws_bytes, void* stream) {
    return guarded("inrf_render_scene_batch", [&] {
        require(n_cameras >= 1 && n_cameras <= INRF_MAX_CAMERAS, "n_cameras must be in [1, INRF_MAX_CAMERAS]");
        require(cams != nullptr, "cameras is NULL");
        dev::CamSet<dev::kMaxCameras> cs;
        std::memset(&cs, 0, sizeof(cs));
        cs.n = n_cameras;
        int64_t pix = 0, tiles = 0;
        for (int j = 0; j < n_cameras; ++j) {
            cs.c[j] = make_camera(&cams[j]);
            cs.c[j].tile0 = int32_t(tiles);
            cs.c[j].pix0 = pix;
            pix += int64_t(cs.c[j].W) * cs.c[j].H;
            tiles += int64_t(cs.c[j].tiles_x) * ((cs.c[j].H + dev::kTile - 1) / dev::kTile);
            require(pix <= (int64_t(1) << 31) - 1, "batch too large (2^31 pixels)");
        }
        require(int64_t(std::max(n_objects, 1)) * tiles <= (int64_t(1) << 31) - 1, "too many tiles x objects");
        run_scene<dev::kMaxCameras>(objects, n_objects, precision, cs, rgba, depth, tri, object, ws, ws_bytes, stream);
    });
}

inrf_status inrf_trace(const inrf_model* m, const float* ray_o, const float* ray_d, int64_t n, int32_t* tri,
                       float* t, void* stream) {
    return guarded("inrf_trace", [&] {
        const dev::ModelC c = make_model(m, false, true);
        require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31)");
        require(n == 0 || (ray_o && ray_d && tri && t), "NULL buffer");
        if (n == 0) return;
        const dev::TraceArgs a{ray_o, ray_d, n, nullptr, t, tri, nullptr, nullptr};  // no records
        launch_trace<1>(c, nullptr, a, n, reinterpret_cast<hipStream_t>(stream), nullptr);
    });
}

inrf_status inrf_encode(const inrf_model* m, const float* x, int64_t n, float* enc, int32_t* slots, void* stream) {
    return guarded("inrf_encode", [&] {
        const dev::ModelC c = make_model(m, true, false);
        require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31)");
        require(n == 0 || (x && enc), "NULL buffer");
        if (n == 0) return;
        const dim3 grid(unsigned((n + dev::kThreads - 1) / dev::kThreads)), block(dev::kThreads);
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        if (c.table_dtype == INRF_F32) hipLaunchKernelGGL(dev::k_encode<float>, grid, block, 0, s, c, x, n, enc, slots);
        else hipLaunchKernelGGL(dev::k_encode<__half>, grid, block, 0, s, c, x, n, enc, slots);
        launch_check("k_encode");
    });
}

inrf_status inrf_mlp_encoded(const inrf_model* m, int32_t precision, const void* enc, const float* dir, int64_t n,
                             float* rgba, void* stream) {
    return guarded("inrf_mlp_encoded", [&] {
        const dev::ModelC c = make_model(m, false, false);
        require(m->weights != nullptr, "weights must be set");
        require(precision == INRF_PREC_FP16 || precision == INRF_PREC_BF16,
                "inrf_mlp_encoded takes 16-bit encodings: precision must be INRF_PREC_FP16 or INRF_PREC_BF16");
        require(n >= 0 && n <= (int64_t(1) << 40), "n must be in [0, 2^40]");
        if (n == 0) return;
        require(enc && dir && rgba, "NULL buffer");
        require((reinterpret_cast<uintptr_t>(rgba) & 15) == 0 && (reinterpret_cast<uintptr_t>(enc) & 1) == 0 &&
                    (reinterpret_cast<uintptr_t>(dir) & 3) == 0,
                "rgba must be 16-byte, enc 2-byte and dir 4-byte aligned");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
#define INRF_MLPE(LPG)                                                                   \
    do {                                                                                \
        if (precision == INRF_PREC_FP16) launch_mlp_enc_t<_Float16, LPG>(c, enc, dir, n, rgba, s); \
        else launch_mlp_enc_t<__bf16, LPG>(c, enc, dir, n, rgba, s);                    \
    } while (0)
        INRF_LPG_SWITCH(c.n_levels, INRF_MLPE)
#undef INRF_MLPE
        launch_check("k_mlp_enc");
    });
}

inrf_status inrf_mlp(const inrf_model* m, int32_t precision, const float* in, int64_t n, float* rgba, void* stream) {
    return guarded("inrf_mlp", [&] {
        check_precision(precision);
        require(m != nullptr && m->weights != nullptr, "model weights must be set");
        require(m->n_levels >= 1 && m->n_levels <= INRF_MAX_LEVELS, "n_levels must be in [1, 32]");
        require(n >= 0 && n <= (int64_t(1) << 31) - 1, "n must be in [0, 2^31)");
        require(n == 0 || (in && rgba), "NULL buffer");
        require((reinterpret_cast<uintptr_t>(rgba) & 15) == 0, "rgba must be 16-byte aligned");
        if (n == 0) return;
        dev::ModelC c;
        std::memset(&c, 0, sizeof(c));
        c.n_levels = m->n_levels;
        c.weights = m->weights;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
#define INRF_MLP(LPG)                                                             \
    do {                                                                         \
        if (precision == INRF_PREC_FP32) launch_mlp_t<float, LPG>(c, in, n, rgba, s);        \
        else if (precision == INRF_PREC_FP16) launch_mlp_t<_Float16, LPG>(c, in, n, rgba, s); \
        else launch_mlp_t<__bf16, LPG>(c, in, n, rgba, s);                       \
    } while (0)
        INRF_LPG_SWITCH(c.n_levels, INRF_MLP)
#undef INRF_MLP
        launch_check("k_mlp");
    });
}

}  // extern "C"
