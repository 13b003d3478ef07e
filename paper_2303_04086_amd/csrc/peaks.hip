// Measurement kernels of the benchmark (include/inrf_peaks.h): a streaming
// HBM read and a matrix-core loop with the instructions the network uses.
// They give the measured ceilings the render path's kernels are compared
// with; the render path never calls them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "inrf_peaks.h"

namespace {

thread_local std::string g_err;

int32_t fail(const std::string& msg) {
    g_err = msg;
    return -1;
}

constexpr int kThreads = 256;
constexpr int kReadBlocksPerCu = 8;
constexpr int kMaxCus = 256;

int num_cus(int& cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail("hipGetDevice failed");
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return fail("hipDeviceGetAttribute(multiprocessor count) failed");
    return 0;
}

// XOR of v over the workgroup, written by thread 0.
__device__ void block_xor(uint32_t v, uint32_t* out) {
    __shared__ uint32_t s[kThreads / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v ^= uint32_t(__shfl_xor(int(v), d));
    if (__lane_id() == 0) s[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = s[0] ^ s[1] ^ s[2] ^ s[3];
}

// Four independent 16-byte loads per thread per step, grid-strided.
__global__ __launch_bounds__(kThreads) void k_read(const uint4* __restrict__ buf, int64_t n16, int reps,
                                                   uint32_t* __restrict__ sink) {
    uint32_t acc = 0;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int r = 0; r < reps; ++r) {
        int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
        for (; i + 3 * stride < n16; i += 4 * stride) {
            const uint4 a = buf[i], b = buf[i + stride], c = buf[i + 2 * stride], d = buf[i + 3 * stride];
            acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
        }
        for (; i < n16; i += stride) {
            const uint4 a = buf[i];
            acc ^= a.x ^ a.y ^ a.z ^ a.w;
        }
    }
    block_xor(acc, sink + blockIdx.x);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ f32x4 mma(float s, f32x4 c) {
    if constexpr (PREC == 0) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(s, s, c, 0, 0, 0);
    } else if constexpr (PREC == 1) {
        const f16x8 v = {(_Float16)s, (_Float16)s, (_Float16)s, (_Float16)s,
                         (_Float16)s, (_Float16)s, (_Float16)s, (_Float16)s};
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(v, v, c, 0, 0, 0);
    } else {
        const bf16x8 v = {(__bf16)s, (__bf16)s, (__bf16)s, (__bf16)s, (__bf16)s, (__bf16)s, (__bf16)s, (__bf16)s};
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(v, v, c, 0, 0, 0);
    }
}

// Four independent accumulator chains per wave; the operands come from the
// lane index, so nothing can be folded away.
template <int PREC>
__global__ __launch_bounds__(kThreads) void k_mfma(int64_t iters, float* __restrict__ sink) {
    const float s = 1e-3f * float(__lane_id() + 1);
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
    for (int64_t i = 0; i < iters; ++i) {
        c0 = mma<PREC>(s, c0);
        c1 = mma<PREC>(s, c1);
        c2 = mma<PREC>(s, c2);
        c3 = mma<PREC>(s, c3);
    }
    if (__lane_id() == 0) sink[(int64_t(blockIdx.x) * kThreads + threadIdx.x) / 64] = c0[0] + c1[1] + c2[2] + c3[3];
}

}  // namespace

extern "C" {

const char* inrf_peaks_last_error(void) { return g_err.c_str(); }

int32_t inrf_peak_read_sink_size(void) { return kReadBlocksPerCu * kMaxCus; }

int32_t inrf_peak_hbm_read(const void* buf, int64_t bytes, int32_t reps, uint32_t* sink, void* stream) {
    if (!buf || !sink) return fail("buf and sink must be set");
    if (bytes <= 0 || bytes % 16 != 0) return fail("bytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0) return fail("buf must be 16-byte aligned");
    if (reps < 1) return fail("reps must be >= 1");
    int cus = 0;
    if (num_cus(cus) != 0) return -1;
    const int blocks = kReadBlocksPerCu * (cus < kMaxCus ? cus : kMaxCus);
    hipLaunchKernelGGL(k_read, dim3(blocks), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream),
                       reinterpret_cast<const uint4*>(buf), bytes / 16, reps, sink);
    return hipGetLastError() == hipSuccess ? 0 : fail("k_read launch failed");
}

int64_t inrf_peak_mfma_waves(int32_t waves_per_simd) {
    int cus = 0;
    if (waves_per_simd < 1 || waves_per_simd > 8 || num_cus(cus) != 0) return -1;
    return int64_t(waves_per_simd) * 4 * cus;
}

int32_t inrf_peak_mfma(int32_t precision, int32_t waves_per_simd, int64_t iters, float* sink, void* stream) {
    if (!sink) return fail("sink must be set");
    if (precision < 0 || precision > 2) return fail("precision must be 0 (FP32), 1 (FP16) or 2 (BF16)");
    if (waves_per_simd < 1 || waves_per_simd > 8) return fail("waves_per_simd must be in [1, 8]");
    if (iters < 1) return fail("iters must be >= 1");
    int cus = 0;
    if (num_cus(cus) != 0) return -1;
    const dim3 grid(unsigned(waves_per_simd * cus)), block(kThreads);  // 4 waves per workgroup: one per SIMD
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (precision == 0) hipLaunchKernelGGL(k_mfma<0>, grid, block, 0, s, iters, sink);
    else if (precision == 1) hipLaunchKernelGGL(k_mfma<1>, grid, block, 0, s, iters, sink);
    else hipLaunchKernelGGL(k_mfma<2>, grid, block, 0, s, iters, sink);
    return hipGetLastError() == hipSuccess ? 0 : fail("k_mfma launch failed");
}

}  // extern "C"
