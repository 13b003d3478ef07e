// Adam (Kingma and Ba, 2015) over flat FP32 parameter arrays: the optimiser
// that trains the feature tables and network weights (Sec. 4.2).  A purely
// streaming kernel: per parameter it reads param, grad, m, v and writes
// param, m, v (and optionally an FP16 copy, and a cleared grad), so it runs
// at HBM bandwidth; four parameters per lane with 16-byte accesses.
// Lazy mode updates only parameters with a nonzero gradient (value and
// moments of the others stay as they are): a batch touches the table slots
// around its rays' hit points, a small part of the table, and the step then
// reads the gradient everywhere but param, m and v only where it is nonzero.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "host_common.hpp"
#include "inrf.h"

namespace inrf {
namespace dev {

struct AdamC {
    float lr, beta1, beta2, eps;
    float inv_bias1, inv_sqrt_bias2;  // 1 / (1 - beta1^t), 1 / sqrt(1 - beta2^t)
    int32_t zero_grad, lazy;
};

__device__ __forceinline__ float adam_one(float& p, float g, float& m, float& v, const AdamC& a) {
    m = a.beta1 * m + (1.f - a.beta1) * g;
    v = a.beta2 * v + (1.f - a.beta2) * g * g;
    p -= a.lr * (m * a.inv_bias1) / (sqrtf(v) * a.inv_sqrt_bias2 + a.eps);
    return p;
}

__global__ void k_adam(float* __restrict__ param, float* __restrict__ grad, float* __restrict__ mom,
                       float* __restrict__ vel, int64_t n, AdamC a, __half* __restrict__ p16) {
    const int64_t n4 = n / 4;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 g = reinterpret_cast<const float4*>(grad)[i];
        const bool ux = !a.lazy || g.x != 0.f, uy = !a.lazy || g.y != 0.f, uz = !a.lazy || g.z != 0.f,
                   uw = !a.lazy || g.w != 0.f;
        if (!(ux || uy || uz || uw)) continue;  // lazy: nothing to update, nothing to clear
        float4 p = reinterpret_cast<float4*>(param)[i];
        float4 m = reinterpret_cast<float4*>(mom)[i];
        float4 v = reinterpret_cast<float4*>(vel)[i];
        if (ux) adam_one(p.x, g.x, m.x, v.x, a);
        if (uy) adam_one(p.y, g.y, m.y, v.y, a);
        if (uz) adam_one(p.z, g.z, m.z, v.z, a);
        if (uw) adam_one(p.w, g.w, m.w, v.w, a);
        reinterpret_cast<float4*>(param)[i] = p;
        reinterpret_cast<float4*>(mom)[i] = m;
        reinterpret_cast<float4*>(vel)[i] = v;
        if (a.zero_grad) reinterpret_cast<float4*>(grad)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p16) {
            reinterpret_cast<__half2*>(p16)[2 * i] = __floats2half2_rn(p.x, p.y);
            reinterpret_cast<__half2*>(p16)[2 * i + 1] = __floats2half2_rn(p.z, p.w);
        }
    }
    // tail of n % 4 elements
    const int64_t k = 4 * n4 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n && (!a.lazy || grad[k] != 0.f)) {
        float p = param[k], m = mom[k], v = vel[k];
        adam_one(p, grad[k], m, v, a);
        param[k] = p;
        mom[k] = m;
        vel[k] = v;
        if (a.zero_grad) grad[k] = 0.f;
        if (p16) p16[k] = __float2half_rn(p);
    }
}

}  // namespace dev
}  // namespace inrf

using namespace inrf;

extern "C" inrf_status inrf_adam(float* param, float* grad, float* m, float* v, int64_t n,
                                 const inrf_adam_params* p, void* param_f16, void* stream) {
    return guarded("inrf_adam", [&] {
        require(p != nullptr, "params is NULL");
        require(n >= 0, "n must be >= 0");
        require(p->step >= 1, "step must be >= 1");
        require(std::isfinite(p->lr) && p->beta1 >= 0.f && p->beta1 < 1.f && p->beta2 >= 0.f && p->beta2 < 1.f &&
                    p->eps > 0.f,
                "need finite lr, beta1 and beta2 in [0,1), eps > 0");
        if (n == 0) return;
        require(param && grad && m && v, "NULL array");
        for (const void* q : {(const void*)param, (const void*)grad, (const void*)m, (const void*)v})
            require((reinterpret_cast<uintptr_t>(q) & 15) == 0, "arrays must be 16-byte aligned");
        require((reinterpret_cast<uintptr_t>(param_f16) & 7) == 0, "param_f16 must be 8-byte aligned");
        dev::AdamC a;
        a.lr = p->lr;
        a.beta1 = p->beta1;
        a.beta2 = p->beta2;
        a.eps = p->eps;
        a.inv_bias1 = float(1.0 / (1.0 - std::pow(double(p->beta1), double(p->step))));
        a.inv_sqrt_bias2 = float(1.0 / std::sqrt(1.0 - std::pow(double(p->beta2), double(p->step))));
        a.zero_grad = p->zero_grad;
        a.lazy = p->lazy;
        const int64_t n4 = n / 4;
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n4 + 255) / 256, 8192));
        hipLaunchKernelGGL(dev::k_adam, dim3(unsigned(blocks)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                           param, grad, m, v, n, a, reinterpret_cast<__half*>(param_f16));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) fail(INRF_E_DEVICE, std::string("k_adam: ") + hipGetErrorString(e));
    });
}
