// tune_kernels.hip -- kernels of the launch tuner: a per-item estimate of
// the walk's length from the packed item table, and the gather of a sample
// of item records (with their photon budgets rescaled) into a table of its
// own, on which trial launches are timed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fos_device.hpp"
#include "fos_kernels.hpp"

namespace fos {

// Estimated photon-steps per photon of item i (and its photon budget): one for the entry, plus per
// layer the scatterings of its longest walks -- a diffusive walk across a
// scattering depth tau_s needs about tau_s^2 (1 - g) of them, absorption
// ends it after about tau_s / tau_a -- whichever is smaller, at least
// tau_s (a ballistic pass).  Only the ranking of items matters.
__global__ void item_cost_kernel(const float4* table, int rf, int n, float* cost, uint64_t* photons)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4* rec = table + (size_t)i * rf;
    photons[i] = (uint64_t)__float_as_uint(rec[1].x) | ((uint64_t)__float_as_uint(rec[1].y) << 32);
    const int L = __float_as_int(rec[1].z);
    float steps = 1.0f;
    for (int l = 0; l < L; ++l) {
        const float4 a = rec[kHdrF4 + kLayerF4 * l], b = rec[kHdrF4 + kLayerF4 * l + 1];
        const uint32_t fl = __float_as_uint(rec[kHdrF4 + kLayerF4 * l + 2].w);
        const float tau = a.x * a.w, ts = tau * a.y, ta = tau - ts;
        const float g = (fl & kHgMirror) ? -b.x : b.x;
        const float diffusion = fmaxf(ts * ts * (1.0f - g), ts);
        const float absorbed = ta > 0.0f ? ts / ta : diffusion;
        steps += fminf(fminf(diffusion, absorbed), 1e8f);
    }
    cost[i] = steps;
}

// out record j = table record idx[j], its photon budget set to photons[j]
// and its item word to j
__global__ void gather_records_kernel(const float4* table, int rf, const int32_t* idx, const uint64_t* photons, int m,
                                      float4* out)
{
    const int j = blockIdx.x;
    if (j >= m) return;
    const float4* src = table + (size_t)idx[j] * rf;
    float4* dst = out + (size_t)j * rf;
    for (int k = threadIdx.x; k < rf; k += blockDim.x) {
        float4 v = src[k];
        if (k == 1) {
            const uint64_t N = photons[j];
            v.x = __uint_as_float((uint32_t)N);
            v.y = __uint_as_float((uint32_t)(N >> 32));
            v.w = __int_as_float(j);
        }
        dst[k] = v;
    }
}

hipError_t launch_item_cost(const float4* table, int rf, int n, float* cost, uint64_t* photons, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(item_cost_kernel, dim3((n + 255) / 256), dim3(256), 0, st, table, rf, n, cost, photons);
    return hipGetLastError();
}

hipError_t launch_gather_records(const float4* table, int rf, const int32_t* idx, const uint64_t* photons, int m,
                                 float4* out, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_records_kernel, dim3(m), dim3(64), 0, st, table, rf, idx, photons, m, out);
    return hipGetLastError();
}

}  // namespace fos
