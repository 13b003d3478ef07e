// The specular network F_s of Sec. 4.2 (Eq. 3) on CDNA4 matrix cores:
// d_in -> 64 -> 64 -> 4, no biases, ReLU hidden, sigmoid outputs.
//
// Two lane layouts are used.
//
// FP32 (v_mfma_f32_4x4x1f32, 16 blocks of 4x4x1).  Rays are the B columns:
// lane l supplies B[0][l%4] of block l/4, i.e. its own ray's input k, and
// holds D[i][l%4] of block l/4 = hidden unit 4t+i of its own ray for tile t.
// A (the weights) is the same in every block: lane l supplies W[4t + l%4][k].
// So every layer stays "one ray per lane": the first layer is accumulated
// input by input as the encoding is produced, and later layers take their B
// operand straight from the previous layer's accumulators.
//
// FP16/BF16 (v_mfma_f32_16x16x32_{f16,bf16}).  Sixteen rays form the B
// columns; lane (g = l/16, r = l%16) supplies B[8g..8g+7][r].  The first
// layer reads its inputs from a small LDS tile; D[4g'+i][r] of tile mt is
// hidden unit 16mt + 4g' + i, which is reused as the next layer's B operand
// without data movement by ordering the reduction index accordingly: chunk kc
// of the next layer's K takes D tiles 2kc and 2kc+1 of each lane.  The weights
// in LDS are stored in that same order ("fragment order").
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include "inrf.h"

namespace inrf {
namespace dev {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kHidden = INRF_HIDDEN;

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + __expf(-z)); }

// ---------------------------------------------------------------- FP32 ----
// LDS image (floats):
//   W1 as [k][4][16]: W1[4t+j][k] at (k*4 + j)*16 + t (lane j=l%4 reads the
//      16 tiles of input k as four 16-byte vectors);
//   W2 as [16][4][kW2Stride]: W2[4q+j][k] at (q*4 + j)*kW2Stride + k (lane j
//      reads row 4q+j of output tile q; the stride keeps the four rows in
//      different banks);
//   W3 as [64][4]: W3[j][k] at k*4 + j.
constexpr int kW2Stride = 68;
__host__ __device__ constexpr int f32_lds_floats(int d_in) { return d_in * 64 + 64 * kW2Stride + 64 * 4; }

__device__ inline void f32_stage_weights(const float* __restrict__ w, int d_in, float* lds) {
    const float* W1 = w;
    const float* W2 = w + kHidden * d_in;
    const float* W3 = W2 + kHidden * kHidden;
    float* L1 = lds;
    float* L2 = lds + d_in * 64;
    float* L3 = L2 + 64 * kW2Stride;
    for (int e = threadIdx.x; e < d_in * 64; e += blockDim.x) {
        const int k = e / 64, j = (e / 16) % 4, t = e % 16;
        L1[e] = W1[(4 * t + j) * d_in + k];
    }
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int row = e / 64, k = e % 64;  // row = 4q + j
        L2[row * kW2Stride + k] = W2[row * kHidden + k];
    }
    for (int e = threadIdx.x; e < 64 * 4; e += blockDim.x) {
        const int k = e / 4, j = e % 4;
        L3[e] = W3[j * kHidden + k];
    }
}

struct F32Acc {
    f32x4 h[16];  // hidden unit 4t+i of this lane's ray in h[t][i]
};

__device__ __forceinline__ void f32_zero(F32Acc& a) {
#pragma unroll
    for (int t = 0; t < 16; ++t) a.h[t] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Adds input value b (index k of this lane's ray) into the first layer.
__device__ __forceinline__ void f32_layer1_input(F32Acc& a, const float* __restrict__ L1, int k, float b) {
    const int j = __lane_id() & 3;
    const f32x4* row = reinterpret_cast<const f32x4*>(L1 + (k * 4 + j) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4 w = row[q];
        a.h[4 * q + 0] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, b, a.h[4 * q + 0], 0, 0, 0);
        a.h[4 * q + 1] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, b, a.h[4 * q + 1], 0, 0, 0);
        a.h[4 * q + 2] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, b, a.h[4 * q + 2], 0, 0, 0);
        a.h[4 * q + 3] = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, b, a.h[4 * q + 3], 0, 0, 0);
    }
}

// Layers 2 and 3 after the first layer has seen every input; returns the
// four pre-sigmoid outputs of this lane's ray.  Layer 2 runs one output tile
// (four hidden units) at a time and feeds it straight into layer 3.
__device__ __forceinline__ f32x4 f32_tail(const F32Acc& a1, const float* __restrict__ L2, const float* __restrict__ L3) {
    const int j = __lane_id() & 3;
    float h[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) h[k] = fmaxf(a1.h[k / 4][k % 4], 0.f);
    f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma nounroll
    for (int q = 0; q < 16; ++q) {
        const f32x4* row = reinterpret_cast<const f32x4*>(L2 + (q * 4 + j) * kW2Stride);
        f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const f32x4 w = row[v];
            c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(w.x, h[4 * v + 0], c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(w.y, h[4 * v + 1], c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_4x4x1f32(w.z, h[4 * v + 2], c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_4x4x1f32(w.w, h[4 * v + 3], c1, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float b = fmaxf(c0[i] + c1[i], 0.f);
            o = __builtin_amdgcn_mfma_f32_4x4x1f32(L3[(4 * q + i) * 4 + j], b, o, 0, 0, 0);
        }
    }
    return o;
}

// ---------------------------------------------------------- FP16 / BF16 ----
template <class T>
struct LP;
template <>
struct LP<_Float16> {
    typedef f16x8 vec;
    __device__ static _Float16 cvt(float v) { return (_Float16)v; }
    __device__ static f32x4 mfma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct LP<__bf16> {
    typedef bf16x8 vec;
    __device__ static __bf16 cvt(float v) { return (__bf16)v; }
    __device__ static f32x4 mfma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

// Number of 32-wide K chunks of the first layer.
__host__ __device__ constexpr int lp_chunks(int d_in) { return (d_in + 31) / 32; }
// LDS image in 16-byte vectors (one per lane per fragment):
//   W1: fragment (mt, kc), lane l: W1[16mt + l%16][32kc + 8(l/16) + i]
//   W2: fragment (ot, kc), lane l: W2[16ot + l%16][hk(kc, l/16, i)]
//   W3: fragment kc,       lane l: l%16 < 4 ? W3[l%16][hk(kc, l/16, i)] : 0
// with hk(kc, g, i) = 32kc + 4g + i for i < 4 and 32kc + 16 + 4g + i - 4 else.
__host__ __device__ constexpr int lp_lds_vecs(int d_in) { return 4 * lp_chunks(d_in) * 64 + 8 * 64 + 2 * 64; }

__device__ __forceinline__ int lp_hk(int kc, int g, int i) { return i < 4 ? 32 * kc + 4 * g + i : 32 * kc + 16 + 4 * g + (i - 4); }

template <class T>
__device__ inline void lp_stage_weights(const float* __restrict__ w, int d_in, typename LP<T>::vec* lds) {
    typedef typename LP<T>::vec V;
    const float* W1 = w;
    const float* W2 = w + kHidden * d_in;
    const float* W3 = W2 + kHidden * kHidden;
    const int C = lp_chunks(d_in);
    for (int e = threadIdx.x; e < 4 * C * 64; e += blockDim.x) {
        const int lane = e % 64, f = e / 64, mt = f / C, kc = f % C;
        V v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * kc + 8 * (lane / 16) + i;
            v[i] = LP<T>::cvt(k < d_in ? W1[(16 * mt + lane % 16) * d_in + k] : 0.f);
        }
        lds[e] = v;
    }
    V* L2 = lds + 4 * C * 64;
    for (int e = threadIdx.x; e < 8 * 64; e += blockDim.x) {
        const int lane = e % 64, f = e / 64, ot = f / 2, kc = f % 2;
        V v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = LP<T>::cvt(W2[(16 * ot + lane % 16) * kHidden + lp_hk(kc, lane / 16, i)]);
        L2[e] = v;
    }
    V* L3 = L2 + 8 * 64;
    for (int e = threadIdx.x; e < 2 * 64; e += blockDim.x) {
        const int lane = e % 64, kc = e / 64, row = lane % 16;
        V v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = LP<T>::cvt(row < 4 ? W3[row * kHidden + lp_hk(kc, lane / 16, i)] : 0.f);
        L3[e] = v;
    }
}

// One block of 16 rays.  x16 points at this block's input rows in LDS
// (row r at x16 + r*stride, in element type T, zero-padded to 32*C); the
// result is the pre-sigmoid output o[i] = output i of ray l%16 for lanes
// l < 16 (other lanes hold padding rows).
template <class T, int C>
__device__ __forceinline__ f32x4 lp_block(const typename LP<T>::vec* __restrict__ W, const T* x16, int stride) {
    typedef typename LP<T>::vec V;
    const int lane = __lane_id(), g = lane / 16, r = lane % 16;
    f32x4 h1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h1[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < C; ++kc) {
        const V b = *reinterpret_cast<const V*>(x16 + r * stride + 32 * kc + 8 * g);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h1[mt] = LP<T>::mfma(W[(mt * C + kc) * 64 + lane], b, h1[mt]);
    }
    const V* W2 = W + 4 * C * 64;
    const V* W3 = W2 + 8 * 64;
    V b2[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b2[kc][i] = LP<T>::cvt(fmaxf(h1[2 * kc][i], 0.f));
            b2[kc][4 + i] = LP<T>::cvt(fmaxf(h1[2 * kc + 1][i], 0.f));
        }
    f32x4 h2[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        h2[ot] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) h2[ot] = LP<T>::mfma(W2[(ot * 2 + kc) * 64 + lane], b2[kc], h2[ot]);
    }
    V b3[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b3[kc][i] = LP<T>::cvt(fmaxf(h2[2 * kc][i], 0.f));
            b3[kc][4 + i] = LP<T>::cvt(fmaxf(h2[2 * kc + 1][i], 0.f));
        }
    f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) o = LP<T>::mfma(W3[kc * 64 + lane], b3[kc], o);
    return o;
}

}  // namespace dev
}  // namespace inrf
