// Gradient of a loss with respect to the network weights and the hash-table
// features (the training signal of Sec. 4.2, Eq. 8), for rays whose closest
// hits k_trace has packed into hit records.  Included by render.hip after the
// shading kernel, whose hit records, tile layout and level gather it reuses.
//
// Per hit ray, given dL/dRGBA:
//   forward again (activations are recomputed, not stored):
//     in = [E; SH], z1 = W1 in, h1 = relu(z1), z2 = W2 h1, h2 = relu(z2),
//     y = sigmoid(W3 h2)
//   adjoint:
//     dz3 = dL/dy * y (1 - y)
//     dz2 = (W3^T dz3) * [z2 > 0]
//     dz1 = (W2^T dz2) * [z1 > 0]
//     dE  = (W1^T dz1) restricted to the feature inputs
//     dW3 += dz3 h2^T,  dW2 += dz2 h1^T,  dW1 += dz1 in^T
//     dH_l[slot(p + c)] += w_c(x) dE_l   for the eight corners of each level
//
// Everything runs on v_mfma_f32_16x16x4f32 in the lane layout of the forward
// network (a wave takes 16 rays at a time; lane (g, r) holds hidden units
// 16t + 4g + i of ray r).  The products with W3^T, W2^T and W1^T keep that
// layout: their A operands are the transposed weights, staged in LDS in the
// order the B operands arrive.  The weight gradients reduce over rays, which
// the matrix instruction can only do along its K index, so the activations
// and adjoints of a block go through the wave's LDS tiles in [ray][unit]
// order; K then walks four rays per instruction.  Each wave keeps its weight
// gradients in accumulator registers for its whole share of the hits; at
// the end the waves of a workgroup add theirs in a fixed order and the
// workgroup writes one partial, which k_reduce_partials sums in a fixed
// order (the weight gradient is deterministic).  Table gradients are FP32
// atomic adds, so their rounding depends on the order in which they land.
#pragma once

#include "mlp_device.hpp"

namespace inrf {
namespace dev {

template <int LPG>
struct BackShape {
    static constexpr int LMAX = 4 * LPG;
    static constexpr int F = feature_slots(LMAX, 1);      // feature columns (multiple of 16)
    static constexpr int S1 = l1_steps(F, 1);
    static constexpr int NI = F + INRF_SH_DIM;            // input tile columns: F features, then SH
    static constexpr int NIT = NI / 16;                   // input column tiles of dW1
    static constexpr int FT = F / 16;                     // feature tiles of dE
    // Row strides that are 16 mod 32 floats: the four rows one instruction
    // reads (lane groups g) fall on disjoint banks.
    static constexpr int IN_STRIDE = (NI % 32 == 16) ? NI : NI + 16;
    static constexpr int H_STRIDE = kHidden + 16;
    static constexpr int fwd_floats = weight_vecs(F, 1);
    static constexpr int wb2_floats = 4 * 16 * 64;        // W2^T fragments (tile t, step s)
    static constexpr int wb1_floats = FT * 16 * 64;       // W1^T fragments (feature tile u, step s)
    static constexpr int tile_floats = 16 * IN_STRIDE + 2 * 16 * H_STRIDE;
    static constexpr size_t lds_bytes =
        size_t(fwd_floats + wb2_floats + wb1_floats + (kThreads / 64) * tile_floats) * sizeof(float);
};

// Number of weights of the network for n_levels levels: W1 [64][2L+16],
// W2 [64][64], W3 [4][64], row-major, in that order.
__host__ __device__ constexpr int weight_count(int n_levels) {
    return kHidden * (2 * n_levels + INRF_SH_DIM) + kHidden * kHidden + INRF_OUT * kHidden;
}

// A operands of the transposed products, in the order the forward network's
// B operands arrive (hidden_index): W2^T fragment (t, s) of lane (g, r) is
// W2[hidden_index(s, g)][16t + r]; W1^T fragment (u, s) is
// W1[hidden_index(s, g)][16u + r] (zero past the feature inputs).
template <int F>
__device__ inline void stage_back_weights(const float* __restrict__ w, int n_levels, float* __restrict__ wb2,
                                          float* __restrict__ wb1) {
    const int d_in = 2 * n_levels + INRF_SH_DIM;
    const float* W1 = w;
    const float* W2 = w + kHidden * d_in;
    constexpr int n2 = 4 * 16 * 64, n1 = (F / 16) * 16 * 64;
    for (int e = threadIdx.x; e < n2 + n1; e += blockDim.x) {
        const int lane = e % 64, g = lane / 16, r = lane % 16;
        if (e < n2) {
            const int f = e / 64, t = f / 16, s = f % 16;
            wb2[e] = W2[hidden_index(1, s, g, 0) * kHidden + 16 * t + r];
        } else {
            const int f = (e - n2) / 64, u = f / 16, s = f % 16, col = 16 * u + r;
            wb1[e - n2] = col < 2 * n_levels ? W1[hidden_index(1, s, g, 0) * d_in + col] : 0.f;
        }
    }
}

// Adds w_c * (de0, de1) to the table gradient of the eight corners of x's
// cell on level L (same slots as the forward lookup).
__device__ __forceinline__ void level_scatter(const ModelC& m, const LevelC& L, float x, float y, float z, float de0,
                                              float de1, float* __restrict__ d_table) {
    LevelQuery q;
    level_issue(m, L, x, y, z, q);
    const float ux = 1.f - q.wx, uy = 1.f - q.wy, uz = 1.f - q.wz;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float wc = ((c & 1) ? q.wx : ux) * ((c & 2) ? q.wy : uy) * ((c & 4) ? q.wz : uz);
        float* p = d_table + 2 * (L.slot_off + level_store(L, q, c));
        unsafeAtomicAdd(p, wc * de0);
        unsafeAtomicAdd(p + 1, wc * de1);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void store4(float* p, float a, float b, float c, float d) {
    *reinterpret_cast<f32x4*>(p) = f32x4{a, b, c, d};
}

template <class TableT, int LPG>
__global__ __launch_bounds__(kThreads) void k_backward(ModelC m, const HitRec* __restrict__ recs,
                                                       const int32_t* __restrict__ counter,
                                                       const float* __restrict__ d_rgba, float* __restrict__ d_table,
                                                       float* __restrict__ partial, float* __restrict__ rgba) {
    typedef Mfma<float> M;
    typedef BackShape<LPG> S;
    extern __shared__ float4 lds_v[];
    __shared__ LevelC s_lv[INRF_MAX_LEVELS];  // per-lane level lookups in the scatter
    float* Wf = reinterpret_cast<float*>(lds_v);
    float* WB2 = Wf + S::fwd_floats;
    float* WB1 = WB2 + S::wb2_floats;
    const int wave = threadIdx.x / 64;
    float* tin = WB1 + S::wb1_floats + wave * S::tile_floats;  // [16][IN_STRIDE]: features, SH
    float* tact = tin + 16 * S::IN_STRIDE;                      // [16][H_STRIDE]: activations
    float* tdz = tact + 16 * S::H_STRIDE;                       // [16][H_STRIDE]: adjoints
    stage_weights<float>(m.weights, m.n_levels, S::F, Wf);
    stage_back_weights<S::F>(m.weights, m.n_levels, WB2, WB1);
    for (int l = threadIdx.x; l < m.n_levels; l += blockDim.x) s_lv[l] = m.lv[l];
    __syncthreads();

    const int n = *counter;
    const int L2 = 2 * m.n_levels, d_in = L2 + INRF_SH_DIM;
    const int lane = __lane_id(), g = lane >> 4, r = lane & 15;
    const float* W2f = Wf + 64 * 4 * S::S1;
    const float* W3f = W2f + 64 * 4 * 16;
    float w3t[4];  // A of W3^T dz3 for tile t: W3[g][16t + r]
#pragma unroll
    for (int t = 0; t < 4; ++t) w3t[t] = m.weights[kHidden * d_in + kHidden * kHidden + g * kHidden + 16 * t + r];

    f32x4 acc1[4][S::NIT], acc2[4][4], acc3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < S::NIT; ++b) acc1[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) acc2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    for (int64_t base = (int64_t(blockIdx.x) * (kThreads / 64) + wave) * 64; base < n;
         base += int64_t(gridDim.x) * kThreads) {
        const int64_t i = base + lane;
        HitRec h;
        if (i < n) h = recs[i];
        else h = HitRec{0.f, 0.f, 0.f, 0, 0.f, 0.f, 1.f, 0};
        float e[S::F];
#pragma unroll
        for (int k = 2 * S::LMAX; k < S::F; ++k) e[k] = 0.f;
        gather_levels<TableT, 0, S::LMAX>(m, h.x, h.y, h.z, e);
        const int nb = int(min<int64_t>(4, (int64_t(n) - base + 15) / 16));
        for (int b = 0; b < nb; ++b) {
            if (g == b) {
                float* row = tin + r * S::IN_STRIDE;
#pragma unroll
                for (int k = 0; k < S::F; k += 4) store4(row + k, e[k], e[k + 1], e[k + 2], e[k + 3]);
                float sh[16];
                sh16(h.dx, h.dy, h.dz, sh);
#pragma unroll
                for (int k = 0; k < 16; k += 4) store4(row + S::F + k, sh[k], sh[k + 1], sh[k + 2], sh[k + 3]);
            }
            wave_sync();
            const int src = 16 * b + r;
            const bool valid = base + src < n;
            const float px = __shfl(h.x, src), py = __shfl(h.y, src), pz = __shfl(h.z, src);
            const int out = __shfl(h.out, src);
            float b1[S::S1];
            load_inputs<float, S::F>(tin + r * S::IN_STRIDE, __shfl(h.dx, src), __shfl(h.dy, src),
                                     __shfl(h.dz, src), b1);

            // ---- forward, keeping z1 and z2 (lane (g, r): units 16t + 4g + i of ray r)
            f32x4 z1[4], z2[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) z1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < S::S1; ++s) {
#pragma unroll
                for (int t = 0; t < 4; ++t) z1[t] = M::op(Wf[(t * S::S1 + s) * 64 + lane], b1[s], z1[t]);
            }
            float a1[16], a2[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) a1[s] = fmaxf(z1[s / 4][s % 4], 0.f);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                z2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 16; ++s) z2[t] = M::op(W2f[(t * 16 + s) * 64 + lane], a1[s], z2[t]);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) a2[s] = fmaxf(z2[s / 4][s % 4], 0.f);
            f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 16; ++s) o = M::op(W3f[s * 64 + lane], a2[s], o);

            // ---- output adjoint (lanes g == 0 hold outputs 0..3 of ray r)
            float dz3[4] = {0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
                const float4 go = reinterpret_cast<const float4*>(d_rgba)[out];
                const float y0 = sigmoidf(o[0]), y1 = sigmoidf(o[1]), y2 = sigmoidf(o[2]), y3 = sigmoidf(o[3]);
                dz3[0] = go.x * y0 * (1.f - y0);
                dz3[1] = go.y * y1 * (1.f - y1);
                dz3[2] = go.z * y2 * (1.f - y2);
                dz3[3] = go.w * y3 * (1.f - y3);
                if (rgba) reinterpret_cast<float4*>(rgba)[out] = make_float4(y0, y1, y2, y3);
            }
            // B of W3^T dz3: lane (g, r) supplies dz3[g] of ray r, held by lane r
            const float q0 = __shfl(dz3[0], r), q1 = __shfl(dz3[1], r), q2 = __shfl(dz3[2], r),
                        q3 = __shfl(dz3[3], r);
            const float bz = g == 0 ? q0 : (g == 1 ? q1 : (g == 2 ? q2 : q3));
            f32x4 dz2[4], dz1[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const f32x4 d = M::op(w3t[t], bz, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int k = 0; k < 4; ++k) dz2[t][k] = z2[t][k] > 0.f ? d[k] : 0.f;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 16; ++s) d = M::op(WB2[(t * 16 + s) * 64 + lane], dz2[s / 4][s % 4], d);
#pragma unroll
                for (int k = 0; k < 4; ++k) dz1[t][k] = z1[t][k] > 0.f ? d[k] : 0.f;
            }

            // ---- feature adjoint and table scatter: lane (g, r) holds dE of
            //      feature slots 16u + 4g + i, i.e. levels 8u + 2g and 8u + 2g + 1
            if (d_table) {
#pragma unroll
                for (int u = 0; u < S::FT; ++u) {
                    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < 16; ++s) d = M::op(WB1[(u * 16 + s) * 64 + lane], dz1[s / 4][s % 4], d);
                    const int la = 8 * u + 2 * g;
                    if (valid && la < m.n_levels) level_scatter(m, s_lv[la], px, py, pz, d[0], d[1], d_table);
                    if (valid && la + 1 < m.n_levels) level_scatter(m, s_lv[la + 1], px, py, pz, d[2], d[3], d_table);
                }
            }

            // ---- weight gradients: K of the matrix instruction walks rays
            //      4s + g through the [ray][unit] tiles
#pragma unroll
            for (int t = 0; t < 4; ++t) store4(tact + r * S::H_STRIDE + 16 * t + 4 * g, a2[4 * t], a2[4 * t + 1],
                                               a2[4 * t + 2], a2[4 * t + 3]);
            if (g == 0) store4(tdz + r * S::H_STRIDE, dz3[0], dz3[1], dz3[2], dz3[3]);
            wave_sync();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int row = 4 * s + g;
                const float av = r < INRF_OUT ? tdz[row * S::H_STRIDE + r] : 0.f;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc3[nt] = M::op(av, tact[row * S::H_STRIDE + 16 * nt + r], acc3[nt]);
            }
            wave_sync();
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                store4(tact + r * S::H_STRIDE + 16 * t + 4 * g, a1[4 * t], a1[4 * t + 1], a1[4 * t + 2], a1[4 * t + 3]);
                store4(tdz + r * S::H_STRIDE + 16 * t + 4 * g, dz2[t][0], dz2[t][1], dz2[t][2], dz2[t][3]);
            }
            wave_sync();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int row = 4 * s + g;
                float av[4], bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    av[t] = tdz[row * S::H_STRIDE + 16 * t + r];
                    bv[t] = tact[row * S::H_STRIDE + 16 * t + r];
                }
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) acc2[mt][nt] = M::op(av[mt], bv[nt], acc2[mt][nt]);
            }
            wave_sync();
#pragma unroll
            for (int t = 0; t < 4; ++t)
                store4(tdz + r * S::H_STRIDE + 16 * t + 4 * g, dz1[t][0], dz1[t][1], dz1[t][2], dz1[t][3]);
            wave_sync();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int row = 4 * s + g;
                float av[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) av[t] = tdz[row * S::H_STRIDE + 16 * t + r];
#pragma unroll
                for (int nt = 0; nt < S::NIT; ++nt) {
                    const float bv = tin[row * S::IN_STRIDE + 16 * nt + r];
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) acc1[mt][nt] = M::op(av[mt], bv, acc1[mt][nt]);
                }
            }
            wave_sync();  // the tiles are rewritten by the next block
        }
    }

    // ---- workgroup sum of the waves' weight gradients, in wave order, into
    //      the (no longer needed) forward-weight region, natural layout
    __syncthreads();
    float* red = Wf;
    const int nw = weight_count(m.n_levels);
    float* r2 = red + kHidden * d_in;
    float* r3 = r2 + kHidden * kHidden;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int unit = 16 * mt + 4 * g + k;
#pragma unroll
                    for (int nt = 0; nt < S::NIT; ++nt) {
                        const int col = 16 * nt + r;
                        const int nat = col < S::F ? (col < L2 ? col : -1) : L2 + (col - S::F);
                        if (nat >= 0) {
                            float* p = red + unit * d_in + nat;
                            *p = (w == 0 ? 0.f : *p) + acc1[mt][nt][k];
                        }
                    }
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        float* p = r2 + unit * kHidden + 16 * nt + r;
                        *p = (w == 0 ? 0.f : *p) + acc2[mt][nt][k];
                    }
                }
            if (g == 0) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        float* p = r3 + k * kHidden + 16 * nt + r;
                        *p = (w == 0 ? 0.f : *p) + acc3[nt][k];
                    }
            }
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < nw; k += blockDim.x) partial[int64_t(blockIdx.x) * nw + k] = red[k];
}

// d_w[k] += sum over workgroups b (ascending) of partial[b][k].
__global__ void k_reduce_partials(const float* __restrict__ partial, int n_parts, int nw, float* __restrict__ d_w) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nw) return;
    float s = 0.f;
    for (int b = 0; b < n_parts; ++b) s += partial[int64_t(b) * nw + k];
    d_w[k] += s;
}

}  // namespace dev
}  // namespace inrf
