// Device-side building blocks shared by the kernels of libinrf: model view,
// exact grid cell, perfect-spatial-hash lookup with trilinear blend, real
// spherical harmonics.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "brick_layout.hpp"
#include "bvh_layout.hpp"
#include "inrf.h"

namespace inrf {
namespace dev {

struct LevelC {
    int32_t res, mbar, rbar, pad;
    uint32_t magic_mbar, magic_rbar;  // ceil(2^32 / m): p mod m = p - m * umulhi(p, magic)
    uint32_t row_m, plane_m, row_r, plane_r;  // brick_row / brick_plane of the two cubes
    uint32_t last_m, pad2;                    // brick_entries(mbar) - 1
    int64_t phi_off, slot_off;
};

struct ModelC {
    int32_t n_levels, table_dtype;
    const uint32_t* phi;
    const void* table;
    const float* weights;
    const BvhNode* nodes;
    const BvhTri* tris;
    int64_t n_tris;
    int32_t stack_depth;  // traversal stack entries per lane (the image's bound, >= 1)
    int32_t n_nodes;      // nodes of the image
    LevelC lv[INRF_MAX_LEVELS];
};

// a mod m for 0 <= a < 2^14 and 1 <= m <= 2^10 with magic = ceil(2^32 / m):
// magic * m - 2^32 = e < m, so a * magic / 2^32 exceeds a / m by less than
// a * e / (m 2^32) < 1 / m, which never crosses the next integer -- the
// quotient umulhi(a, magic) is exact.
__device__ __forceinline__ int mod_small(int a, int m, uint32_t magic) {
    return a - m * int(__umulhi(uint32_t(a), magic));
}

// (a >= m ? a - m : a) for 0 <= a < 2m, as an unsigned minimum.
__device__ __forceinline__ int wrap_once(int a, int m) { return int(min(uint32_t(a), uint32_t(a - m))); }

// Cell of x (already in [0,1]) on a grid of N cells: p = floor of the exact
// product N*x, clamped to N-1, and w = N*x - p rounded once (Sec. 4.1: scale
// by the resolution, take the floor).  fl(N*x) can round up onto an integer
// while the exact product lies below it; the FMA residual detects that.
__device__ __forceinline__ void cell_of(float x, int N, int& p, float& w) {
    const float fn = float(N);
    const float y = fn * x;
    const float e = __builtin_fmaf(fn, x, -y);  // exact: N*x - fl(N*x)
    float fl = floorf(y);
    if (fl == y && e < 0.f) fl -= 1.f;
    fl = fminf(fl, fn - 1.f);
    p = int(fl);
    w = __builtin_fmaf(fn, x, -fl);
}

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.f), 1.f); }

template <class T>
struct TableRead;
// Feature pair of entry i of a level's table starting at `base` (the entry
// offset in bytes fits 32 bits: the host bounds every level's table below
// 4 GiB), so the load takes a wave-uniform base and a 32-bit lane offset.
template <>
struct TableRead<float> {
    typedef float2 elem;
    __device__ static float2 get(const char* base, uint32_t i) {
        return *reinterpret_cast<const float2*>(base + (i << 3));
    }
};
template <>
struct TableRead<__half> {
    typedef __half2 elem;
    __device__ static float2 get(const char* base, uint32_t i) {
        return __half22float2(*reinterpret_cast<const __half2*>(base + (i << 2)));
    }
};

// Perfect-spatial-hash encoding (Sec. 4.1, Eq. 1):
//   slot(v) = (v mod mbar + Phi[v mod rbar]) mod mbar, component-wise,
// for the eight corners v = p + c of x's cell, blended trilinearly with
// corner c = cx + 2cy + 4cz weighted prod_i (c_i ? w_i : 1 - w_i), summed in
// ascending c.
//
// The lookup of one level is two dependent memory round trips (offsets,
// then features).  LevelQuery splits it so that a caller can issue the
// offset loads of several levels before waiting on any of them.
struct LevelQuery {
    float wx, wy, wz;
    int hx, hy, hz;  // (p mod mbar) per axis
    uint32_t o[8];   // packed offsets of the eight corners
};

// Cell, hash bases and the eight offset loads of one level.
// The model M is any descriptor with the offset and feature tables `phi`
// and `table` (the full ModelC, or the shading view of one scene object).
template <class M>
__device__ __forceinline__ void level_issue(const M& m, const LevelC& L, float x, float y, float z, LevelQuery& q) {
    int px, py, pz;
    cell_of(x, L.res, px, q.wx);
    cell_of(y, L.res, py, q.wy);
    cell_of(z, L.res, pz, q.wz);
    const int qx = mod_small(px, L.rbar, L.magic_rbar), qy = mod_small(py, L.rbar, L.magic_rbar),
              qz = mod_small(pz, L.rbar, L.magic_rbar);
    q.hx = mod_small(px, L.mbar, L.magic_mbar);
    q.hy = mod_small(py, L.mbar, L.magic_mbar);
    q.hz = mod_small(pz, L.mbar, L.magic_mbar);
    const int qx1 = (qx + 1 == L.rbar) ? 0 : qx + 1, qy1 = (qy + 1 == L.rbar) ? 0 : qy + 1,
              qz1 = (qz + 1 == L.rbar) ? 0 : qz + 1;
    const uint32_t X[2] = {brick_x(qx), brick_x(qx1)};
    const uint32_t Y[2] = {brick_y(qy, L.row_r), brick_y(qy1, L.row_r)};
    const uint32_t Z[2] = {brick_z(qz, L.plane_r), brick_z(qz1, L.plane_r)};
    const char* phi = reinterpret_cast<const char*>(m.phi + L.phi_off);
#pragma unroll
    for (int c = 0; c < 8; ++c)
        q.o[c] = *reinterpret_cast<const uint32_t*>(phi + ((X[c & 1] + Y[(c >> 1) & 1] + Z[c >> 2]) << 2));
}

// Slot of corner c once its offset has arrived, as cube coordinates.
// (p + c) mod mbar is at most mbar and a valid offset is below mbar, so one
// wrap reduces each component.
__device__ __forceinline__ void level_slot3(const LevelC& L, const LevelQuery& q, int c, uint32_t& sx, uint32_t& sy,
                                            uint32_t& sz) {
    sx = uint32_t(wrap_once(q.hx + ((c & 1) ? 1 : 0) + int(q.o[c] & 1023u), L.mbar));
    sy = uint32_t(wrap_once(q.hy + ((c & 2) ? 1 : 0) + int((q.o[c] >> 10) & 1023u), L.mbar));
    sz = uint32_t(wrap_once(q.hz + ((c & 4) ? 1 : 0) + int((q.o[c] >> 20) & 1023u), L.mbar));
}

// Storage index (in the level's table) of corner c's slot; the clamp keeps
// even a corrupt offset table inside the level.
__device__ __forceinline__ uint32_t level_store(const LevelC& L, const LevelQuery& q, int c) {
    uint32_t sx, sy, sz;
    level_slot3(L, q, c, sx, sy, sz);
    return min(brick_x(sx) + brick_y(sy, L.row_m) + brick_z(sz, L.plane_m), L.last_m);
}

// Feature loads of the eight corners.
template <class T, class M>
__device__ __forceinline__ void level_fetch(const M& m, const LevelC& L, const LevelQuery& q, float2* f,
                                            int32_t* __restrict__ slots_out) {
    const char* base = reinterpret_cast<const char*>(
        reinterpret_cast<const typename TableRead<T>::elem*>(m.table) + L.slot_off);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint32_t sx, sy, sz;
        level_slot3(L, q, c, sx, sy, sz);
        f[c] = TableRead<T>::get(base, min(brick_x(sx) + brick_y(sy, L.row_m) + brick_z(sz, L.plane_m), L.last_m));
        if (slots_out) slots_out[c] = int(__umul24(__umul24(sz, L.mbar) + sy, L.mbar) + sx);
    }
}

__device__ __forceinline__ float2 level_blend(const LevelQuery& q, const float2* f) {
    const float ux = 1.f - q.wx, uy = 1.f - q.wy, uz = 1.f - q.wz;
    float2 e = make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float wc = ((c & 1) ? q.wx : ux) * ((c & 2) ? q.wy : uy) * ((c & 4) ? q.wz : uz);
        e.x += wc * f[c].x;
        e.y += wc * f[c].y;
    }
    return e;
}

// One level, optionally writing the eight level-local linear slots
// (s_z * mbar + s_y) * mbar + s_x to slots_out[0..7] (global memory).
template <class T, class M>
__device__ __forceinline__ float2 encode_level(const M& m, const LevelC& L, float x, float y, float z,
                                               int32_t* __restrict__ slots_out) {
    LevelQuery q;
    level_issue(m, L, x, y, z, q);
    float2 f[8];
    level_fetch<T>(m, L, q, f, slots_out);
    return level_blend(q, f);
}

// Two levels with their offset loads in flight together (x in [0,1]^3; a
// lane with nothing to do passes a valid dummy point and drops the result).
template <class T, class M>
__device__ __forceinline__ void encode_level_pair(const M& m, const LevelC& La, const LevelC& Lb, float x, float y,
                                                  float z, float2& ea, float2& eb) {
    LevelQuery qa, qb;
    level_issue(m, La, x, y, z, qa);
    level_issue(m, Lb, x, y, z, qb);
    float2 fa[8], fb[8];
    level_fetch<T>(m, La, qa, fa, nullptr);
    level_fetch<T>(m, Lb, qb, fb, nullptr);
    ea = level_blend(qa, fa);
    eb = level_blend(qb, fb);
}

// Real spherical harmonics of bands 0..3 of a unit vector, index l*l + l + m,
// orthonormal, Condon-Shortley phase (closed-form polynomials).
__device__ __forceinline__ void sh16(float x, float y, float z, float* o) {
    const float xx = x * x, yy = y * y, zz = z * z;
    o[0] = 0.28209479177387814f;
    o[1] = -0.48860251190291992f * y;
    o[2] = 0.48860251190291992f * z;
    o[3] = -0.48860251190291992f * x;
    o[4] = 1.0925484305920792f * x * y;
    o[5] = -1.0925484305920792f * y * z;
    o[6] = 0.31539156525252005f * (3.f * zz - 1.f);
    o[7] = -1.0925484305920792f * x * z;
    o[8] = 0.54627421529603959f * (xx - yy);
    o[9] = -0.59004358992664352f * y * (3.f * xx - yy);
    o[10] = 2.8906114426405538f * x * y * z;
    o[11] = -0.45704579946446572f * y * (5.f * zz - 1.f);
    o[12] = 0.3731763325901154f * z * (5.f * zz - 3.f);
    o[13] = -0.45704579946446572f * x * (5.f * zz - 1.f);
    o[14] = 1.4453057213202769f * z * (xx - yy);
    o[15] = -0.59004358992664352f * x * (xx - 3.f * yy);
}

}  // namespace dev
}  // namespace inrf
