// mlp_kernels.hip -- the surrogate network on gfx950: a small MLP that maps a
// single-layer transport problem to its R/A/T fractions, standing in for the
// Monte Carlo walk the way the paper's pre-trained network does
// (Methodology, Photon transport), with the walk as its fallback.
//
// Network (per ensemble member): 8 standardised features -> 256 -> 256 ->
// 256 -> 256 (tanh-form GELU after each) -> 3 logits -> softmax.
//
//   gemm<TA,TB,EPI> : C = op(A) op(B), bf16 operands on v_mfma_f32_16x16x32_bf16,
//                     fp32 accumulation, 64x64x32 LDS tiles, fused epilogues
//                     (store fp32 / bias + GELU -> fp32 Z and bf16 H /
//                     multiply by GELU'(Z) -> fp32 and bf16 dZ); grid.z walks
//                     the ensemble members.
//   backward_layer  : one layer of the backward pass in one launch: the
//                     weight gradient H^T dZ cut into K ranges (the batch)
//                     whose partial tiles, with the bias gradient as column
//                     sums, go to a workspace, and the next dZ product.
//   splitk_reduce_jobs : the partials of all five layers added in a fixed
//                     order into the flat gradient, one launch.
//   features        : transport problem -> the 8 raw features.
//   input_layer     : gather and standardisation of a training batch and the
//                     8-wide input layer on the VALU (fp32), one launch.
//   softmax_ce      : softmax of the 3 logits, cross-entropy against the Monte
//                     Carlo fractions, d loss / d logits = (p - y) / B.
//   adam_loss       : Adam on fp32 master weights, refreshing bf16 copies, and
//                     the per-member loss of the batch (deterministic tree).
// Prediction (network + ensemble gate) is one fused kernel in mlp_infer.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "fos_mlp.hpp"

namespace fos {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float tanh_fast(float u)
{
    // tanh(u) = 1 - 2 / (1 + e^{2u}); saturates correctly at +-inf
    const float e = __expf(2.0f * u);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}
__device__ __forceinline__ float gelu_f(float z)
{
    return 0.5f * z * (1.0f + tanh_fast(kGeluC * fmaf(kGeluA * z, z * z, z)));
}
__device__ __forceinline__ float gelu_grad_f(float z)
{
    const float t = tanh_fast(kGeluC * fmaf(kGeluA * z, z * z, z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * kGeluC * fmaf(3.0f * kGeluA, z * z, 1.0f);
}

// ---------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------
constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

// One 64 x 64 output tile (bx, by) of member / K range bz (of nz = members x
// splits) of the product g.
template <bool TA, bool TB, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, const int bx, const int by, const int bz, const int nz)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[kBM][kBK + kPad];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kBN][kBK + kPad];
    const int net = bz / g.splits, split = bz - net * g.splits;
    const int kspan = g.K / g.splits;
    const __bf16* A = g.A + (size_t)net * g.strideA;
    const __bf16* B = g.B + (size_t)net * g.strideB;
    const int m0 = by * kBM, n0 = bx * kBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // column sums of B over the same K range (the bias gradient), by the first
    // M tile from the B tile in LDS: lane = column, wave w the rows 8w .. 8w + 7
    // of each k-step
    const bool col_sums = g.colsum && by == 0 && n0 + lane < g.ncol;
    float csv = 0.f;
    // the next k-step's tiles are loaded into registers while this one
    // multiplies (one register set, written to LDS after the barrier)
    const int kbeg = split * kspan, kend = kbeg + kspan;
    auto load_a = [&](int k0) -> bf16x8 {
        if (!TA) return *reinterpret_cast<const bf16x8*>(A + (size_t)(m0 + (tid >> 2)) * g.lda + k0 + (tid & 3) * 8);
        return *reinterpret_cast<const bf16x8*>(A + (size_t)(k0 + (tid >> 3)) * g.lda + m0 + (tid & 7) * 8);
    };
    auto load_b = [&](int k0) -> bf16x8 {
        if (TB) return *reinterpret_cast<const bf16x8*>(B + (size_t)(n0 + (tid >> 2)) * g.ldb + k0 + (tid & 3) * 8);
        return *reinterpret_cast<const bf16x8*>(B + (size_t)(k0 + (tid >> 3)) * g.ldb + n0 + (tid & 7) * 8);
    };
    bf16x8 va = load_a(kbeg), vb = load_b(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        if (!TA) {   // A(m,k) = A[m*lda + k]
            *reinterpret_cast<bf16x8*>(&As[tid >> 2][(tid & 3) * 8]) = va;
        } else {     // A(m,k) = A[k*lda + m]
            const int kk = tid >> 3, mc = (tid & 7) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) As[mc + j][kk] = va[j];
        }
        if (TB) {    // B(k,n) = B[n*ldb + k]
            *reinterpret_cast<bf16x8*>(&Bs[tid >> 2][(tid & 3) * 8]) = vb;
        } else {     // B(k,n) = B[k*ldb + n]
            const int kk = tid >> 3, nc = (tid & 7) * 8;
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[nc + j][kk] = vb[j];
        }
        __syncthreads();
        if (k0 + kBK < kend) {
            va = load_a(k0 + kBK);
            vb = load_b(k0 + kBK);
        }
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + j * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (col_sums) {
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(&Bs[lane][wave * 8]);
#pragma unroll
            for (int e = 0; e < 8; ++e) csv += (float)v[e];
        }
        __syncthreads();
    }

    if (g.colsum && by == 0) {   // the 4 waves' column sums
        __shared__ float csl[4][64];
        const int c = n0 + lane;
        csl[wave][lane] = csv;
        __syncthreads();
        if (wave == 0 && c < g.ncol) {
            const float v = (csl[0][lane] + csl[1][lane]) + (csl[2][lane] + csl[3][lane]);
            if (g.splits == 1 && !g.partials) g.csum[(size_t)net * g.strideCsum + c] = v;
            else g.ws[(size_t)nz * g.M * g.N + (size_t)bz * g.N + c] = v;
        }
    }
    float* Cf = g.Cf ? g.Cf + (size_t)net * g.strideC : nullptr;
    long ldc = g.ldc;
    if (EPI == kEpiStore && (g.splits > 1 || g.partials)) {   // partial tile of this K range
        Cf = g.ws + (size_t)bz * g.M * g.N;
        ldc = g.N;
    }
    __bf16* Cb = g.Cb ? g.Cb + (size_t)net * g.strideCb : nullptr;
    const float* bias = g.bias ? g.bias + (size_t)net * g.strideBias : nullptr;
    const float* Z = g.Z ? g.Z + (size_t)net * g.strideZ : nullptr;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int col = n0 + wn + j * 16 + (lane & 15);
                const size_t o = (size_t)row * ldc + col;
                const float v = acc[i][j][r];
                if (EPI == kEpiStore) {
                    Cf[o] = v;
                } else if (EPI == kEpiBiasGelu) {
                    const float z = v + bias[col];
                    if (Cf) Cf[o] = z;
                    Cb[o] = (__bf16)gelu_f(z);
                } else {   // kEpiGeluGrad: v is dH, Z the saved pre-activation
                    const float dz = v * gelu_grad_f(Z[o]);
                    if (Cf) Cf[o] = dz;
                    Cb[o] = (__bf16)dz;
                }
            }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    gemm_tile<TA, TB, EPI>(g, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z);
}

// A layer of the backward pass in one launch: the split-K weight gradient
// dW = H^T dZ (g1, partial tiles to its workspace) and, independent of it,
// the next dZ = (dZ W^T) * gelu'(Z) (g2).  The first blocks take g1's tiles.
__global__ __launch_bounds__(256) void backward_layer_kernel(GemmArgs g1, GemmArgs g2, int nets)
{
    const int gx1 = g1.N / kBN, gy1 = g1.M / kBM, gz1 = nets * g1.splits;
    int b = blockIdx.x;
    if (b < gx1 * gy1 * gz1) {
        gemm_tile<true, false, kEpiStore>(g1, b % gx1, (b / gx1) % gy1, b / (gx1 * gy1), gz1);
    } else {
        b -= gx1 * gy1 * gz1;
        const int gx2 = g2.N / kBN, gy2 = g2.M / kBM;
        gemm_tile<false, true, kEpiGeluGrad>(g2, b % gx2, (b / gx2) % gy2, b / (gx2 * gy2), nets);
    }
}

// The ordered split-K sums of several weight gradients in one launch
// (grid.z = job): C[net][row][col] (ldc, strideC, rows < rows_out and cols <
// cols_out, so padded products land in the flat gradient directly) = the sum
// over s = 0 .. splits-1, in that order, of the partial tiles ws[net][s], and
// likewise the column sums.
__global__ void splitk_reduce_jobs_kernel(ReduceJobs jobs, int nets)
{
    const ReduceJob& J = jobs.job[blockIdx.z];
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int net = blockIdx.y;
    const size_t MN = (size_t)J.M * J.N;
    if (e >= MN) return;
    const float* p = J.ws + (size_t)net * J.splits * MN + e;
    const int row = (int)(e / J.N), col = (int)(e % J.N);
    if (row < J.rows_out && col < J.cols_out) {
        float s = 0.0f;
        for (int k = 0; k < J.splits; ++k) s += p[(size_t)k * MN];
        J.C[(size_t)net * J.strideC + (size_t)row * J.ldc + col] = s;
    }
    if (J.csum && e < (size_t)J.ncol) {
        const float* q = J.ws + (size_t)nets * J.splits * MN + (size_t)net * J.splits * J.N + e;
        float t = 0.0f;
        for (int k = 0; k < J.splits; ++k) t += q[(size_t)k * J.N];
        J.csum[(size_t)net * J.strideCsum + e] = t;
    }
}

template <bool TA, bool TB, int EPI>
static hipError_t launch_gemm_t(const GemmArgs& g, int nets, hipStream_t st)
{
    hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI>), dim3(g.N / kBN, g.M / kBM, nets), dim3(256), 0, st, g);
    return hipGetLastError();
}

static bool gemm_shape_ok(const GemmArgs& g)
{
    return g.M > 0 && g.N > 0 && g.K > 0 && g.M % kBM == 0 && g.N % kBN == 0 && g.K % kBK == 0 &&
           g.splits >= 1 && g.splits <= kMaxSplits && g.K % (g.splits * kBK) == 0;
}

hipError_t launch_backward_layer(const GemmArgs& g1, const GemmArgs& g2, int nets, hipStream_t st)
{
    if (!gemm_shape_ok(g1) || !gemm_shape_ok(g2) || g2.splits != 1 || !g1.ws || !g2.Cb || !g2.Z ||
        (g1.colsum && (!g1.csum || g1.ncol < 1 || g1.ncol > g1.N)))
        return hipErrorInvalidValue;
    const int blocks = (g1.N / kBN) * (g1.M / kBM) * nets * g1.splits + (g2.N / kBN) * (g2.M / kBM) * nets;
    hipLaunchKernelGGL(backward_layer_kernel, dim3(blocks), dim3(256), 0, st, g1, g2, nets);
    return hipGetLastError();
}

hipError_t launch_gemm_partials(const GemmArgs& g, int nets, hipStream_t st)
{
    if (!gemm_shape_ok(g) || !g.ws || (g.colsum && (!g.csum || g.ncol < 1 || g.ncol > g.N)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_kernel<true, false, kEpiStore>), dim3(g.N / kBN, g.M / kBM, nets * g.splits), dim3(256),
                       0, st, g);
    return hipGetLastError();
}

hipError_t launch_splitk_reduce_jobs(const ReduceJobs& jobs, int nets, hipStream_t st)
{
    if (jobs.n < 1 || jobs.n > kMaxReduceJobs) return hipErrorInvalidValue;
    size_t mn = 0;
    for (int j = 0; j < jobs.n; ++j) mn = std::max(mn, (size_t)jobs.job[j].M * jobs.job[j].N);
    hipLaunchKernelGGL(splitk_reduce_jobs_kernel, dim3((unsigned)((mn + 255) / 256), nets, jobs.n), dim3(256), 0, st,
                       jobs, nets);
    return hipGetLastError();
}

int gemm_splits(int K)
{
    int s = 1;
    while (s < kMaxSplits && K % (2 * s * kBK) == 0 && K / (2 * s * kBK) >= 8) s *= 2;
    return s;
}

hipError_t launch_gemm(const GemmArgs& g, bool ta, bool tb, int epi, int nets, hipStream_t st)
{
    if (!gemm_shape_ok(g) || g.splits != 1 || g.partials || g.colsum) return hipErrorInvalidValue;
    if (!ta && !tb && epi == kEpiBiasGelu) return launch_gemm_t<false, false, kEpiBiasGelu>(g, nets, st);
    if (!ta && !tb && epi == kEpiStore) return launch_gemm_t<false, false, kEpiStore>(g, nets, st);
    if (!ta && tb && epi == kEpiGeluGrad) return launch_gemm_t<false, true, kEpiGeluGrad>(g, nets, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// features, standardisation, first layer
// ---------------------------------------------------------------------------
// Raw features of item i (single layer): log10(tau_s + 1e-6),
// log10(tau_a + 1e-6), -log10(1 - g + 1e-3), n_layer, n_lower,
// log10(k_lower + 1e-4), mu0, 0.  The anisotropy enters through log(1 - g):
// near g = 1 the transport depends on the reduced depth tau_s (1 - g), which
// the first layer then reaches as a sum of two features.
// eligible = one layer and an upper medium of index 1.
__global__ void features_kernel(int n, int L, const int32_t* n_layers, const float* mu_s, const float* mu_a,
                                const float* g, const float* n_layer, const float* thickness,
                                const float* n_upper, const float* n_lower, const float* k_lower,
                                const float* mu0, float* x, uint8_t* eligible)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t o = (size_t)i * L;
    const float t = thickness[o];
    float* xi = x + (size_t)i * kFeatures;
    xi[0] = log10f(mu_s[o] * t + 1e-6f);
    xi[1] = log10f(mu_a[o] * t + 1e-6f);
    xi[2] = -log10f(1.001f - g[o]);
    xi[3] = n_layer[o];
    xi[4] = n_lower[i];
    xi[5] = log10f(k_lower[i] + 1e-4f);
    xi[6] = mu0[i];
    xi[7] = 0.0f;
    if (eligible) eligible[i] = (n_layers[i] == 1 && n_upper[i] == 1.0f) ? 1 : 0;
}

// The standardisation of a training batch and the first layer in one
// launch: block (b, m) takes rows 16b .. 16b + 15 of member m; its first 16
// threads gather and standardise one row each (writing xs, the
// bf16 copy xb padded to 64 for the first layer's weight gradient, and ys),
// then thread t computes Z1 = X W1 + b1 (fp32, K = 8) and H1 = bf16(gelu(Z1))
// for neuron t of the 16 rows.
constexpr int kInRows = 16;
__global__ __launch_bounds__(256) void input_layer_kernel(StdArgs a, const float* params, size_t pstride, float* Z1,
                                                          __bf16* H1)
{
    __shared__ float sx[kInRows][kFeatures];
    const int m = blockIdx.y, t = threadIdx.x;
    const int r0 = blockIdx.x * kInRows;
    if (t < kInRows) {
        const int r = r0 + t;
        float* xs = a.xs + ((size_t)m * a.rows_pad + r) * kFeatures;
        if (r < a.rows) {
            int64_t src = a.base + r;
            if (a.perm_mul)
                src = (int64_t)(((uint64_t)a.perm_mul[m] * (uint64_t)(a.base + r) + a.perm_add[m]) % (uint64_t)a.n_src);
            const bool valid = src < a.n_src;
            __bf16* xb = a.xb ? a.xb + ((size_t)m * a.rows_pad + r) * kPadIn : nullptr;
            for (int k = 0; k < kFeatures; ++k) {
                const float v = valid ? (a.x[(size_t)src * kFeatures + k] - a.mean[k]) * a.inv_std[k] : 0.0f;
                xs[k] = v;
                sx[t][k] = v;
                if (xb) xb[k] = (__bf16)v;
            }
            if (xb)
                for (int k = kFeatures; k < kPadIn; ++k) xb[k] = (__bf16)0.0f;
            if (a.y && a.ys) {
                float* ys = a.ys + ((size_t)m * a.rows_pad + r) * 3;
                for (int c = 0; c < 3; ++c) ys[c] = valid ? a.y[(size_t)src * 3 + c] : 0.0f;
            }
        } else {
            for (int k = 0; k < kFeatures; ++k) sx[t][k] = r < a.rows_pad ? xs[k] : 0.0f;
        }
    }
    __syncthreads();
    const float* P = params + (size_t)m * pstride;
    float w[kFeatures];
#pragma unroll
    for (int k = 0; k < kFeatures; ++k) w[k] = P[kOffW1 + k * kHidden + t];
    const float b = P[kOffB1 + t];
    for (int i = 0; i < kInRows; ++i) {
        const int r = r0 + i;
        if (r >= a.rows_pad) break;
        float z = b;
#pragma unroll
        for (int k = 0; k < kFeatures; ++k) z = fmaf(sx[i][k], w[k], z);
        const size_t o = ((size_t)m * a.rows_pad + r) * kHidden + t;
        if (Z1) Z1[o] = z;
        H1[o] = (__bf16)gelu_f(z);
    }
}

// softmax over the 3 logits (columns 0..2 of a 64-wide fp32 row) + b5;
// with targets: per-row loss into loss_rows, dlogits (p - y)/B into a 64-wide
// bf16 row (zeros beyond 3)
__global__ void softmax_ce_kernel(SoftmaxArgs a)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (r >= a.rows_pad) return;
    const float* P = a.params + (size_t)m * a.pstride;
    const float* lg = a.logits + ((size_t)m * a.rows_pad + r) * kPadOut;
    float l[3];
    for (int c = 0; c < 3; ++c) l[c] = lg[c] + P[kOffB5 + c];
    const float mx = fmaxf(l[0], fmaxf(l[1], l[2]));
    float e[3], s = 0.f;
    for (int c = 0; c < 3; ++c) { e[c] = __expf(l[c] - mx); s += e[c]; }
    const float is = 1.0f / s;
    float p[3];
    for (int c = 0; c < 3; ++c) p[c] = e[c] * is;
    float* po = a.probs + ((size_t)m * a.rows_pad + r) * 3;
    for (int c = 0; c < 3; ++c) po[c] = p[c];
    if (a.ys) {
        const float* y = a.ys + ((size_t)m * a.rows_pad + r) * 3;
        const bool valid = r < a.rows;
        const float ls = logf(s) + mx;
        float loss = 0.f;
        for (int c = 0; c < 3; ++c) loss -= y[c] * (l[c] - ls);
        a.loss_rows[(size_t)m * a.rows_pad + r] = valid ? loss : 0.f;
        __bf16* d = a.dlog + ((size_t)m * a.rows_pad + r) * kPadOut;
        for (int c = 0; c < 3; ++c) d[c] = (__bf16)(valid ? (p[c] - y[c]) * a.inv_batch : 0.f);
        for (int c = 3; c < kPadOut; ++c) d[c] = (__bf16)0.0f;
    }
}

// The Adam step of a training step and, in the extra last block of each
// member, its batch loss (loss_sum_kernel's fixed tree) in one launch.
__global__ __launch_bounds__(256) void adam_loss_kernel(AdamArgs a, const float* __restrict__ loss_rows, int rows,
                                                        float* dst, float scale)
{
    const int m = blockIdx.y, t = threadIdx.x;
    if (dst && blockIdx.x == gridDim.x - 1) {
        __shared__ float part[256];
        const float* l = loss_rows + (size_t)m * rows;
        float s = 0.f;
        for (int r = t; r < rows; r += 256) s += l[r];
        part[t] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) part[t] += part[t + o];
            __syncthreads();
        }
        if (t == 0) dst[m] += scale * part[0];
        return;
    }
    const size_t j = (size_t)blockIdx.x * blockDim.x + t;
    if (j >= (size_t)kParams) return;
    const size_t o = (size_t)m * kParams + j;
    const float g = a.grads[o];
    const float mm = a.b1 * a.m[o] + (1.0f - a.b1) * g;
    const float vv = a.b2 * a.v[o] + (1.0f - a.b2) * g * g;
    a.m[o] = mm;
    a.v[o] = vv;
    const float mh = mm * a.c1, vh = vv * a.c2;
    const float w = a.w[o] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.w[o] = w;
    if (j >= kOffW2 && j < kOffB2) a.wb[(size_t)m * kBfParams + kBfW2 + (j - kOffW2)] = (__bf16)w;
    else if (j >= kOffW3 && j < kOffB3) a.wb[(size_t)m * kBfParams + kBfW3 + (j - kOffW3)] = (__bf16)w;
    else if (j >= kOffW4 && j < kOffB4) a.wb[(size_t)m * kBfParams + kBfW4 + (j - kOffW4)] = (__bf16)w;
    else if (j >= kOffW5 && j < kOffB5) {
        const int k = (int)((j - kOffW5) / 3), c = (int)((j - kOffW5) % 3);
        a.wb[(size_t)m * kBfParams + kBfW5p + (size_t)k * kPadOut + c] = (__bf16)w;
        a.wb[(size_t)m * kBfParams + kBfW5t + (size_t)k * kPadK5 + c] = (__bf16)w;
    }
}

// bf16 copies from the fp32 master weights (after loading a model)
__global__ void refresh_bf16_kernel(const float* w, __bf16* wb)
{
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (j >= (size_t)kBfParams) return;
    const float* P = w + (size_t)m * kParams;
    float v = 0.0f;
    if (j < kBfW3) v = P[kOffW2 + (j - kBfW2)];
    else if (j < kBfW4) v = P[kOffW3 + (j - kBfW3)];
    else if (j < kBfW5p) v = P[kOffW4 + (j - kBfW4)];
    else if (j < kBfW5t) {
        const size_t k = (j - kBfW5p) / kPadOut, c = (j - kBfW5p) % kPadOut;
        v = c < 3 ? P[kOffW5 + k * 3 + c] : 0.0f;
    } else {
        const size_t k = (j - kBfW5t) / kPadK5, c = (j - kBfW5t) % kPadK5;
        v = c < 3 ? P[kOffW5 + k * 3 + c] : 0.0f;
    }
    wb[(size_t)m * kBfParams + j] = (__bf16)v;
}

// dst[m] (+)= scale * sum of member m's `rows` per-row losses, one block of 256
// per member: strided partial sums, then a fixed tree (deterministic)
__global__ __launch_bounds__(256) void loss_sum_kernel(const float* __restrict__ loss_rows, int rows, float* dst,
                                                       float scale, int add)
{
    __shared__ float part[256];
    const int m = blockIdx.x, t = threadIdx.x;
    const float* l = loss_rows + (size_t)m * rows;
    float s = 0.f;
    for (int r = t; r < rows; r += 256) s += l[r];
    part[t] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) part[t] += part[t + o];
        __syncthreads();
    }
    if (t == 0) dst[m] = (add ? dst[m] : 0.f) + scale * part[0];
}

// member mean, spread = max_c (max_m p - min_m p), domain test of the raw
// features against the training box, and the fallback decision
// per-feature mean, 1/std and min/max of n raw rows (one block, 8 x 128 threads)
__global__ void feature_stats_kernel(const float* x, int64_t n, float* stats)
{
    __shared__ double s1[kFeatures][128], s2[kFeatures][128];
    __shared__ float mn[kFeatures][128], mx[kFeatures][128];
    const int k = threadIdx.y, t = threadIdx.x;
    double a = 0.0, b = 0.0;
    float lo = 3e38f, hi = -3e38f;
    for (int64_t i = t; i < n; i += 128) {
        const float v = x[(size_t)i * kFeatures + k];
        a += v; b += (double)v * v;
        lo = fminf(lo, v); hi = fmaxf(hi, v);
    }
    s1[k][t] = a; s2[k][t] = b; mn[k][t] = lo; mx[k][t] = hi;
    __syncthreads();
    if (t == 0) {
        double A = 0.0, Bq = 0.0;
        float L = 3e38f, H = -3e38f;
        for (int j = 0; j < 128; ++j) { A += s1[k][j]; Bq += s2[k][j]; L = fminf(L, mn[k][j]); H = fmaxf(H, mx[k][j]); }
        const double mean = A / (double)n;
        double var = Bq / (double)n - mean * mean;
        if (var < 0) var = 0;
        const double sd = sqrt(var);
        stats[k] = (float)mean;
        stats[kFeatures + k] = sd > 1e-6 ? (float)(1.0 / sd) : 1.0f;
        stats[2 * kFeatures + k] = L;
        stats[3 * kFeatures + k] = H;
    }
}

// ---------------------------------------------------------------------------
// sweep: fallback selection and compaction (count / scan / write), gather of
// the fallback sub-problem, scatter of its Monte Carlo fractions, spectral
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool fallback_of(const SweepSelectArgs& a, int64_t i)
{
    return !(a.in_domain[i] != 0) || !(a.spread[i] <= a.spread_max);
}

__global__ void select_count_kernel(SweepSelectArgs a)
{
    __shared__ unsigned int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * kSelectPerBlock;
    unsigned int c = 0;
    for (int j = 0; j < 8; ++j) {
        const int64_t i = b0 + (int64_t)threadIdx.x * 8 + j;
        if (i < a.n) {
            const bool f = fallback_of(a, i);
            a.used_mc[i] = f ? 1 : 0;
            c += f ? 1u : 0u;
        }
    }
    atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) a.block_count[blockIdx.x] = cnt;
}

__global__ __launch_bounds__(1024) void select_scan_kernel(unsigned long long* count, unsigned long long* offset,
                                                           int blocks, unsigned long long* total)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int per = (blocks + 1023) / 1024;
    const int b = t * per, e = b + per < blocks ? b + per : blocks;
    unsigned long long s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = t > 0 ? part[t - 1] : 0ull;
    for (int i = b; i < e; ++i) { offset[i] = run; run += count[i]; }
    if (t == 1023) *total = part[1023];
}

__global__ void select_write_kernel(SweepSelectArgs a)
{
    __shared__ unsigned int pre[256];
    const int64_t b0 = (int64_t)blockIdx.x * kSelectPerBlock;
    const int t = threadIdx.x;
    unsigned int c = 0;
    for (int j = 0; j < 8; ++j) {
        const int64_t i = b0 + (int64_t)t * 8 + j;
        if (i < a.n && a.used_mc[i]) ++c;
    }
    pre[t] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned int v = t >= off ? pre[t - off] : 0u;
        __syncthreads();
        pre[t] += v;
        __syncthreads();
    }
    unsigned long long o = a.block_offset[blockIdx.x] + (t > 0 ? pre[t - 1] : 0u);
    for (int j = 0; j < 8; ++j) {
        const int64_t i = b0 + (int64_t)t * 8 + j;
        if (i < a.n && a.used_mc[i]) a.idx[o++] = i;
    }
}

__global__ void gather_items_kernel(GatherArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const int64_t i = a.idx[k];
    a.o_n_layers[k] = a.n_layers[i];
    for (int l = 0; l < a.L; ++l) {
        const size_t s = (size_t)i * a.L + l, d = (size_t)k * a.L + l;
        a.o_mu_s[d] = a.mu_s[s]; a.o_mu_a[d] = a.mu_a[s]; a.o_g[d] = a.g[s];
        a.o_n_layer[d] = a.n_layer[s]; a.o_thickness[d] = a.thickness[s];
    }
    a.o_n_upper[k] = a.n_upper[i]; a.o_n_lower[k] = a.n_lower[i]; a.o_k_lower[k] = a.k_lower[i];
    a.o_mu0[k] = a.mu0[i];
    a.o_photons[k] = a.photons;
}

// R = (specular + diffuse)/N, A, T of fallback item k into row idx[k]
__global__ void scatter_mc_kernel(int64_t m, const int64_t* idx, const unsigned long long* t, float* rat)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const unsigned long long* tk = t + (size_t)k * 6;
    const double N = (double)(tk[0] + tk[1] + tk[2] + tk[3] + tk[4]);
    const int64_t i = idx[k];
    rat[i * 3 + 0] = (float)((double)(tk[0] + tk[1]) / N);
    rat[i * 3 + 1] = (float)((double)tk[2] / N);
    rat[i * 3 + 2] = (float)((double)tk[3] / N);
}

// out[d] = (sum_l w_r[l] R[d][l], sum_l w_e[l] A[d][l]) -- one wave per design
__global__ void spectral_reduce_kernel(int designs, int lambdas, const float* rat, const float* w_r, const float* w_e,
                                       float* out)
{
    const int d = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (d >= designs) return;
    float r = 0.f, e = 0.f;
    for (int l = lane; l < lambdas; l += 64) {
        const float* p = rat + ((size_t)d * lambdas + l) * 3;
        r = fmaf(w_r[l], p[0], r);
        e = fmaf(w_e[l], p[1], e);
    }
    for (int off = 32; off > 0; off >>= 1) {
        r += __shfl_xor(r, off);
        e += __shfl_xor(e, off);
    }
    if (lane == 0) { out[2 * (size_t)d] = r; out[2 * (size_t)d + 1] = e; }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_select_count(const SweepSelectArgs& a, hipStream_t st)
{
    const int64_t blocks = (a.n + kSelectPerBlock - 1) / kSelectPerBlock;
    hipLaunchKernelGGL(select_count_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_select_scan(const SweepSelectArgs& a, unsigned long long* total, hipStream_t st)
{
    const int blocks = (int)((a.n + kSelectPerBlock - 1) / kSelectPerBlock);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(1024), 0, st, a.block_count, a.block_offset, blocks, total);
    return hipGetLastError();
}

hipError_t launch_select_write(const SweepSelectArgs& a, hipStream_t st)
{
    const int64_t blocks = (a.n + kSelectPerBlock - 1) / kSelectPerBlock;
    hipLaunchKernelGGL(select_write_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gather_items(const GatherArgs& a, hipStream_t st)
{
    if (a.m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_items_kernel, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_scatter_mc(int64_t m, const int64_t* idx, const unsigned long long* tallies, float* rat,
                             hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_mc_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, idx, tallies, rat);
    return hipGetLastError();
}

hipError_t launch_spectral_reduce(int designs, int lambdas, const float* rat, const float* w_r, const float* w_e,
                                  float* out, hipStream_t st)
{
    if (designs <= 0) return hipSuccess;
    hipLaunchKernelGGL(spectral_reduce_kernel, dim3((designs + 3) / 4), dim3(256), 0, st, designs, lambdas, rat, w_r,
                       w_e, out);
    return hipGetLastError();
}
hipError_t launch_features(int n, int L, const int32_t* n_layers, const float* mu_s, const float* mu_a,
                           const float* g, const float* n_layer, const float* thickness, const float* n_upper,
                           const float* n_lower, const float* k_lower, const float* mu0, float* x,
                           uint8_t* eligible, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, L, n_layers, mu_s, mu_a, g,
                       n_layer, thickness, n_upper, n_lower, k_lower, mu0, x, eligible);
    return hipGetLastError();
}

hipError_t launch_softmax_ce(const SoftmaxArgs& a, int nets, hipStream_t st)
{
    hipLaunchKernelGGL(softmax_ce_kernel, dim3((a.rows_pad + 255) / 256, nets), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_input_layer(const StdArgs& a, const float* params, size_t pstride, float* Z1, __bf16* H1, int nets,
                              hipStream_t st)
{
    hipLaunchKernelGGL(input_layer_kernel, dim3((a.rows_pad + kInRows - 1) / kInRows, nets), dim3(kHidden), 0, st, a,
                       params, pstride, Z1, H1);
    return hipGetLastError();
}

hipError_t launch_adam_loss(const AdamArgs& a, const float* loss_rows, int rows, float* dst, float scale, int nets,
                            hipStream_t st)
{
    const unsigned blocks = (unsigned)((kParams + 255) / 256) + (dst ? 1u : 0u);
    hipLaunchKernelGGL(adam_loss_kernel, dim3(blocks, nets), dim3(256), 0, st, a, loss_rows, rows, dst, scale);
    return hipGetLastError();
}

hipError_t launch_refresh_bf16(const float* w, __bf16* wb, int nets, hipStream_t st)
{
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)((kBfParams + 255) / 256), nets), dim3(256), 0, st, w, wb);
    return hipGetLastError();
}

hipError_t launch_loss_sum(const float* loss_rows, int rows, float* dst, float scale, bool add, int nets,
                           hipStream_t st)
{
    hipLaunchKernelGGL(loss_sum_kernel, dim3(nets), dim3(256), 0, st, loss_rows, rows, dst, scale, add ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_feature_stats(const float* x, int64_t n, float* stats, hipStream_t st)
{
    hipLaunchKernelGGL(feature_stats_kernel, dim3(1), dim3(128, kFeatures), 0, st, x, n, stats);
    return hipGetLastError();
}

}  // namespace fos
