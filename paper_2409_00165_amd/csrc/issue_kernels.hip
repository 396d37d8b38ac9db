// issue_kernels.hip -- throughput of the VALU instruction forms the photon
// walk is made of, on the walk's own launch shape (256-thread workgroups,
// 8 per CU, so 8 waves per SIMD): FP32 multiply-add in its three-operand
// (v_fma_f32) and accumulating (v_fmac_f32) encodings and multiply
// (v_mul_f32), the four transcendental forms of a step (log, reciprocal,
// square root, cosine) and whole Philox4x32-10 blocks (32x32->64 products
// and three-input xors).  Each thread runs kChains independent chains, so issue,
// not latency, sets the pace.  These rates are the measured ceiling the
// walk's roofline is quoted against beside the chip's nominal FP32 peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fos_device.hpp"
#include "fos_kernels.hpp"

namespace fos {

constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void issue_k(int iters, float seed, float* sink)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    if constexpr (KIND == kIssuePhilox) {
        uint32_t x = 0u;
        for (int i = 0; i < iters; ++i) {
            const uint4 b = philox4x32_10(tid, (uint32_t)i, (uint32_t)i ^ tid, x, __float_as_uint(seed), 0x5EEDu);
            x ^= b.x ^ b.y ^ b.z ^ b.w;
        }
        acc = (float)x;
    } else {
        float a[kChains];
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = seed + 0.001f * (float)(tid + j);
        const float m = 1.0f - 1e-7f * seed, c = 1e-7f * seed;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < kChains; ++j) {
                if constexpr (KIND == kIssueFma) a[j] = fmaf(a[j], m, c);
                if constexpr (KIND == kIssueFmac) a[j] = fmaf(m, c, a[j]);
                if constexpr (KIND == kIssueMul) a[j] = a[j] * m;
                if constexpr (KIND == kIssueRcp) a[j] = __builtin_amdgcn_rcpf(a[j]);
                if constexpr (KIND == kIssueSqrt) a[j] = __builtin_amdgcn_sqrtf(a[j]);
                if constexpr (KIND == kIssueLog) a[j] = __builtin_amdgcn_logf(a[j]);
                if constexpr (KIND == kIssueCos) a[j] = __builtin_amdgcn_cosf(a[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc += a[j];
    }
    sink[tid] = acc;
}

int issue_ops_per_iteration(int kind) { return kind == kIssuePhilox ? 1 : kChains; }

hipError_t launch_issue(int kind, int iters, int grid, int block, float* sink, hipStream_t st)
{
    const float seed = 1.2345f;
    switch (kind) {
    case kIssueFma: hipLaunchKernelGGL(issue_k<kIssueFma>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueRcp: hipLaunchKernelGGL(issue_k<kIssueRcp>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueSqrt: hipLaunchKernelGGL(issue_k<kIssueSqrt>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueLog: hipLaunchKernelGGL(issue_k<kIssueLog>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueCos: hipLaunchKernelGGL(issue_k<kIssueCos>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueFmac: hipLaunchKernelGGL(issue_k<kIssueFmac>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssueMul: hipLaunchKernelGGL(issue_k<kIssueMul>, dim3(grid), dim3(block), 0, st, iters, seed, sink); break;
    case kIssuePhilox:
        hipLaunchKernelGGL(issue_k<kIssuePhilox>, dim3(grid), dim3(block), 0, st, iters, seed, sink);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fos
