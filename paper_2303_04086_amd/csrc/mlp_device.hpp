// The specular network F_s of Sec. 4.2 (Eq. 3) on CDNA4 matrix cores:
// d_in -> 64 -> 64 -> 4, no biases, ReLU hidden, sigmoid outputs.
//
// Lane layout (both precisions).  A wave evaluates 16 rays at a time; lane
// l = 16g + r supplies B[k][r] for the k of its lane group g, i.e. a quarter
// of ray r's first-layer inputs.  The caller places the F feature slots (2 per
// level, zero-padded) of the block's rays in an LDS tile, one row per ray, and
// each lane reads its slice with 16-byte loads; the 16 SH values are computed
// by the lanes themselves.  The order in which values enter the reduction is a
// permutation of the natural input order [E_0..E_{L-1}, SH_0..SH_15]; the
// first layer's weights are stored in LDS in that permuted order ("fragment
// order"):
//   FP32 (v_mfma_f32_16x16x4f32, one value per lane per instruction): step
//     s = 4j + i carries feature slot 16j + 4g + i; the last four steps carry
//     SH value 4g + i.
//   FP16/BF16 (v_mfma_f32_16x16x32, eight values per lane): chunk c carries
//     feature slots 32c + 8g + i; the last chunk carries SH value 8g + i
//     (g < 2; zeros for g >= 2).
//
// The result of a 16x16 instruction, D[4g'+i][r] held by lane (g', r) as
// element i of tile mt, is hidden unit 16mt + 4g' + i of ray r.  The next layer
// takes its B operand from those registers unchanged by ordering its
// reduction index the same way; its weights are stored in that order too.
// Accumulation is FP32 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "device_common.hpp"
#include "inrf.h"

namespace inrf {
namespace dev {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kHidden = INRF_HIDDEN;

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + __expf(-z)); }

// ------------------------------------------------------- precision traits --
template <class P>
struct Mfma;

template <>
struct Mfma<float> {
    static constexpr int V = 1;  // values per lane per instruction
    typedef float vec;
    __device__ static float cvt(float v) { return v; }
    __device__ static f32x4 op(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<_Float16> {
    static constexpr int V = 8;
    typedef f16x8 vec;
    __device__ static _Float16 cvt(float v) { return (_Float16)v; }
    __device__ static f32x4 op(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<__bf16> {
    static constexpr int V = 8;
    typedef bf16x8 vec;
    __device__ static __bf16 cvt(float v) { return (__bf16)v; }
    __device__ static f32x4 op(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

// Feature slots of a tile row for up to lmax levels, rounded so that every
// lane's 16-byte reads stay inside the row.
__host__ __device__ constexpr int feature_slots(int lmax, int V) {
    return V == 1 ? ((2 * lmax + 15) / 16) * 16 : ((2 * lmax + 31) / 32) * 32;
}
// Number of first-layer instructions per output tile; X extra inputs (0 or
// 1) follow the SH values: FP32 takes one more step for them, FP16/BF16
// have room in the SH step.
__host__ __device__ constexpr int l1_steps(int F, int V, int X = 0) {
    return V == 1 ? F / 4 + 4 + X : F / 32 + 1;
}
// Steps of layers 2 and 3 (K = 64).
__host__ __device__ constexpr int hid_steps(int V) { return V == 1 ? 16 : 2; }
// LDS image, in units of one lane's operand (P::vec), 64 lanes per fragment:
//   W1 fragments (mt, s), W2 fragments (ot, s), W3 fragments (s).
__host__ __device__ constexpr int weight_vecs(int F, int V, int X = 0) {
    return 64 * (4 * l1_steps(F, V, X) + 4 * hid_steps(V) + hid_steps(V));
}
__host__ __device__ constexpr int weight_bytes(int F, int V, int X = 0) {
    return weight_vecs(F, V, X) * (V == 1 ? 4 : 16);
}

// Natural input index carried by element i of lane group g at first-layer
// step s, or -1 for padding (n_levels real levels, F feature slots, X extra
// inputs after the SH values).
__device__ __forceinline__ int l1_index(int V, int F, int n_levels, int s, int g, int i, int X = 0) {
    if (V == 1) {
        if (s < F / 4) {
            const int slot = 16 * (s / 4) + 4 * g + (s % 4);
            return slot < 2 * n_levels ? slot : -1;
        }
        if (s < F / 4 + 4) return 2 * n_levels + 4 * g + (s - F / 4);
        return g < X ? 2 * n_levels + INRF_SH_DIM + g : -1;
    }
    if (s < F / 32) {
        const int slot = 32 * s + 8 * g + i;
        return slot < 2 * n_levels ? slot : -1;
    }
    const int k = 8 * g + i;
    return k < INRF_SH_DIM + X ? 2 * n_levels + k : -1;
}

// Hidden unit fed by element i of lane group g at hidden-layer step s.
__device__ __forceinline__ int hidden_index(int V, int s, int g, int i) {
    if (V == 1) return 16 * (s / 4) + 4 * g + (s % 4);  // s = (tile mt, element)
    return i < 4 ? 32 * s + 4 * g + i : 32 * s + 16 + 4 * g + (i - 4);
}

template <class P, int X = 0>
__device__ inline void stage_weights(const float* __restrict__ w, int n_levels, int F,
                                     typename Mfma<P>::vec* __restrict__ lds) {
    typedef Mfma<P> M;
    constexpr int V = M::V;
    const int d_in = 2 * n_levels + INRF_SH_DIM + X;
    const float* W1 = w;
    const float* W2 = w + kHidden * d_in;
    const float* W3 = W2 + kHidden * kHidden;
    const int S1 = l1_steps(F, V, X), SH = hid_steps(V);
    const int n1 = 64 * 4 * S1, n2 = 64 * 4 * SH, n3 = 64 * SH;
    for (int e = threadIdx.x; e < n1 + n2 + n3; e += blockDim.x) {
        const int lane = e % 64, g = lane / 16, r = lane % 16;
        typename M::vec v;
        if (e < n1) {
            const int f = e / 64, mt = f / S1, s = f % S1;
            for (int i = 0; i < V; ++i) {
                const int k = l1_index(V, F, n_levels, s, g, i, X);
                const float x = k >= 0 ? W1[(16 * mt + r) * d_in + k] : 0.f;
                if constexpr (V == 1) v = M::cvt(x);
                else v[i] = M::cvt(x);
            }
        } else if (e < n1 + n2) {
            const int f = (e - n1) / 64, ot = f / SH, s = f % SH;
            for (int i = 0; i < V; ++i) {
                const float x = W2[(16 * ot + r) * kHidden + hidden_index(V, s, g, i)];
                if constexpr (V == 1) v = M::cvt(x);
                else v[i] = M::cvt(x);
            }
        } else {
            const int s = (e - n1 - n2) / 64;
            for (int i = 0; i < V; ++i) {
                const float x = r < INRF_OUT ? W3[r * kHidden + hidden_index(V, s, g, i)] : 0.f;
                if constexpr (V == 1) v = M::cvt(x);
                else v[i] = M::cvt(x);
            }
        }
        lds[e] = v;
    }
}

// The first layer's B operands of this lane: feature slots from row r of the
// block's LDS tile (element type of the precision for FP16/BF16, FP32
// otherwise), the SH values of direction d (ray r of the block) and, with
// X = 1, the extra input `extra` of that ray.
template <class P, int F, int X = 0>
__device__ __forceinline__ void load_inputs(const void* tile_row, float dx, float dy, float dz,
                                            typename Mfma<P>::vec* b, float extra = 0.f) {
    typedef Mfma<P> M;
    constexpr int V = M::V, S1 = l1_steps(F, V, X);
    const int g = __lane_id() >> 4;
    float sh[16];
    sh16(dx, dy, dz, sh);
    if constexpr (V == 1) {
        const float* row = reinterpret_cast<const float*>(tile_row);
#pragma unroll
        for (int j = 0; j < F / 16; ++j) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(row + 16 * j + 4 * g);
            b[4 * j + 0] = v[0];
            b[4 * j + 1] = v[1];
            b[4 * j + 2] = v[2];
            b[4 * j + 3] = v[3];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            b[F / 4 + i] = g == 0 ? sh[i] : (g == 1 ? sh[4 + i] : (g == 2 ? sh[8 + i] : sh[12 + i]));
        if constexpr (X == 1) b[F / 4 + 4] = g == 0 ? extra : 0.f;
    } else {
        typedef typename M::vec Vec;
        const Vec* row = reinterpret_cast<const Vec*>(tile_row);
#pragma unroll
        for (int c = 0; c < F / 32; ++c) b[c] = row[4 * c + g];
        Vec v;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            v[i] = M::cvt(g == 0 ? sh[i] : (g == 1 ? sh[8 + i] : (X == 1 && g == 2 && i == 0 ? extra : 0.f)));
        b[S1 - 1] = v;
    }
}

// The first layer's B operands of this lane from row r of the block's tile
// holding the ray's F feature slots followed by its 16 SH values (both in the
// tile's element type: the precision's 16-bit type, or FP32), and, with X = 1,
// the extra input `extra` of that ray.  The SH values are computed once per
// ray by the lane that owns the ray, rather than by every lane group.
template <class P, int F, int X = 0>
__device__ __forceinline__ void load_inputs_row(const void* tile_row, typename Mfma<P>::vec* b, float extra = 0.f) {
    typedef Mfma<P> M;
    constexpr int V = M::V, S1 = l1_steps(F, V, X);
    const int g = __lane_id() >> 4;
    if constexpr (V == 1) {
        const float* row = reinterpret_cast<const float*>(tile_row);
#pragma unroll
        for (int j = 0; j < F / 16 + 1; ++j) {  // the last read is SH values 4g .. 4g + 3
            const f32x4 v = *reinterpret_cast<const f32x4*>(row + 16 * j + 4 * g);
            b[4 * j + 0] = v[0];
            b[4 * j + 1] = v[1];
            b[4 * j + 2] = v[2];
            b[4 * j + 3] = v[3];
        }
        if constexpr (X == 1) b[F / 4 + 4] = g == 0 ? extra : 0.f;
    } else {
        typedef typename M::vec Vec;
        const Vec* row = reinterpret_cast<const Vec*>(tile_row);
#pragma unroll
        for (int c = 0; c < F / 32; ++c) b[c] = row[4 * c + g];
        Vec v = row[F / 8 + (g & 1)];  // SH values 8g .. 8g + 7 for g < 2
        if (g >= 2) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = M::cvt(X == 1 && g == 2 && i == 0 ? extra : 0.f);
        }
        b[S1 - 1] = v;
    }
}

// This lane's A operand of weight fragment f, from the LDS image (WLds) or
// from registers the lane loaded it into once (WReg).
template <class Vec>
struct WLds {
    const Vec* __restrict__ W;
    int lane;
    __device__ Vec operator()(int f) const { return W[f * 64 + lane]; }
};
template <class Vec, int N>
struct WReg {
    Vec w[N];
    __device__ Vec operator()(int f) const { return w[f]; }
};

// ReLU of hidden values and their conversion to the next layer's B operand.
// For 16-bit operands the values are converted first and the ReLU is a
// packed integer max with 0 on the 16-bit patterns: a negative value (sign
// bit set, -0 included) becomes +0, any other is kept, which is exactly the
// conversion of max(x, 0) in half the instructions and without the operand
// canonicalisation a float max needs.  FP32 does the same on 32-bit patterns.
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

template <class P>
__device__ __forceinline__ typename Mfma<P>::vec relu_pack(const f32x4& lo, const f32x4& hi) {
    typedef Mfma<P> M;
    typedef float f32x8 __attribute__((ext_vector_type(8)));
    const f32x8 x = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    const typename M::vec v = __builtin_convertvector(x, typename M::vec);
    const i16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
    return __builtin_bit_cast(typename M::vec, __builtin_elementwise_max(__builtin_bit_cast(i16x8, v), z));
}

// The network for NB blocks of 16 rays each, given each block's first-layer
// B operands b1[blk][step]; the blocks' instructions are interleaved step by
// step, so one block's matrix instructions run while another's results are
// converted.  o[blk] is D of the output tile: for lanes l < 16, element i is
// pre-sigmoid output i of ray l of that block.
template <class P, int F, int X, int NB, class WA>
__device__ __forceinline__ void mlp_blocks_w(const WA& wa, const typename Mfma<P>::vec (*b1)[l1_steps(F, Mfma<P>::V, X)],
                                             f32x4* o) {
    typedef Mfma<P> M;
    typedef typename M::vec Vec;
    constexpr int V = M::V, S1 = l1_steps(F, V, X), SH = hid_steps(V);
    f32x4 h1[NB][4];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h1[k][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S1; ++s) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const Vec w = wa(mt * S1 + s);
#pragma unroll
            for (int k = 0; k < NB; ++k) h1[k][mt] = M::op(w, b1[k][s], h1[k][mt]);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep weight loads next to their use
    }
    constexpr int F2 = 4 * S1, F3 = F2 + 4 * SH;  // first fragments of W2 and W3
    Vec b2[NB][SH];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int s = 0; s < SH; ++s) {
            if constexpr (V == 1) b2[k][s] = relu_bits(h1[k][s / 4][s % 4]);
            else b2[k][s] = relu_pack<P>(h1[k][2 * s], h1[k][2 * s + 1]);
        }
    f32x4 h2[NB][4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
#pragma unroll
        for (int k = 0; k < NB; ++k) h2[k][ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < SH; ++s) {
            const Vec w = wa(F2 + ot * SH + s);
#pragma unroll
            for (int k = 0; k < NB; ++k) h2[k][ot] = M::op(w, b2[k][s], h2[k][ot]);
            if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    Vec b3[NB][SH];
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
        for (int s = 0; s < SH; ++s) {
            if constexpr (V == 1) b3[k][s] = relu_bits(h2[k][s / 4][s % 4]);
            else b3[k][s] = relu_pack<P>(h2[k][2 * s], h2[k][2 * s + 1]);
        }
#pragma unroll
    for (int k = 0; k < NB; ++k) o[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < SH; ++s) {
        const Vec w = wa(F3 + s);
#pragma unroll
        for (int k = 0; k < NB; ++k) o[k] = M::op(w, b3[k][s], o[k]);
        if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

// One block of 16 rays (NB = 1).
template <class P, int F, int X, class WA>
__device__ __forceinline__ f32x4 mlp_block_w(const WA& wa, const typename Mfma<P>::vec* b1) {
    f32x4 o;
    mlp_blocks_w<P, F, X, 1>(wa, reinterpret_cast<const typename Mfma<P>::vec(*)[l1_steps(F, Mfma<P>::V, X)]>(b1), &o);
    return o;
}

template <class P, int F, int X = 0>
__device__ __forceinline__ f32x4 mlp_block(const typename Mfma<P>::vec* __restrict__ W,
                                           const typename Mfma<P>::vec* b1);

template <class P, int F, int X>
__device__ __forceinline__ f32x4 mlp_block(const typename Mfma<P>::vec* __restrict__ W,
                                           const typename Mfma<P>::vec* b1) {
    return mlp_block_w<P, F, X>(WLds<typename Mfma<P>::vec>{W, int(__lane_id())}, b1);
}

// Fragments of the whole weight image (first layer, then W2, then W3).
template <class P, int F, int X = 0>
__host__ __device__ constexpr int weight_frags() {
    return 4 * l1_steps(F, Mfma<P>::V, X) + 5 * hid_steps(Mfma<P>::V);
}

}  // namespace dev
}  // namespace inrf
