// mlp_infer.hip -- fused ensemble inference of the surrogate network with its
// validity gate: one workgroup carries a tile of rows through all five layers
// of all four members without leaving the CU, then writes the ensemble mean,
// the spread and the domain flag.
//
// Per member the rows see: standardise -> 8 -> 256 (GELU) -> 256 (GELU) ->
// 256 (GELU) -> 256 (GELU) -> 3 -> softmax, the same network the training
// kernels (mlp_kernels.hip) fit.  Every product runs on
// v_mfma_f32_16x16x32_bf16 with fp32 accumulation:
//   * the 8-wide input layer keeps fp32-like accuracy by splitting inputs and
//     weights into bf16 high and low parts: one K=32 product holds
//     W_hi x_hi + W_hi x_lo + W_lo x_hi (the dropped W_lo x_lo term is below
//     2^-16 relative);
//   * hidden layers multiply bf16 weights by the bf16 activations kept in LDS;
//   * the output layer pads its 3 neurons to one 16-wide tile.
// The products are computed transposed (neurons x rows): the weights are the
// A operand, streamed from L2 in a pre-swizzled fragment order (one coalesced
// 1 KB load per 16 x 32 fragment), and the activations are the B operand read
// from LDS.  A lane's accumulator then holds 4 consecutive neurons of one
// row: the biases enter as the first product's accumulator, and the GELU
// epilogue writes two such quads (one per 16-neuron tile) as one 16-byte
// chunk back to LDS (layout below).
//
// Work split inside a workgroup (4 waves, TILE = kInferTile rows): wave w
// owns neurons 64w .. 64w+63 of every hidden layer for all rows (TILE/4
// accumulator tiles) and TILE/64 row tiles of the output layer; the lanes that
// end with a row's logits keep that row's ensemble sum / min / max in
// registers across the members.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fos_mlp.hpp"

namespace fos {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kHRow = kHidden;               // bf16 per LDS activation row (512 B, 16-byte chunks swizzled)
constexpr int kXRow = 32 + 8;                // bf16 per LDS input-fragment row

// gelu(z) = 0.5 z (1 + tanh(u)), u = sqrt(2/pi)(z + 0.044715 z^3), evaluated
// as z * sigmoid(2u) = z / (1 + 2^(z (k1 + k2 z^2))); saturates to 0 and z
// at the two ends without NaN.
constexpr float kG1 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
constexpr float kG2 = kG1 * 0.044715f;

__device__ __forceinline__ float gelu_sig(float z)
{
    const float t = z * fmaf(kG2, z * z, kG1);
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

__device__ __forceinline__ floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// The 4 biases of the neurons a lane's accumulator quad holds in tile j: the
// first product of a layer starts from them instead of from zero, so the
// epilogue has no bias add.
__device__ __forceinline__ void bias_quads(floatx4 (&b)[4], const float* __restrict__ bias, int w, int q)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n0 = 16 * (4 * w + j) + 4 * q;
        b[j] = {bias[n0], bias[n0 + 1], bias[n0 + 2], bias[n0 + 3]};
    }
}

// Activations in LDS.  Hidden neuron n = 32b + 16t + 4q + e (b = 32-column
// block, t = which of the block's two 16-neuron tiles, q = lane quarter,
// e = 0..3) sits in column 32b + 8q + 4t + e, so the two 4-neuron quads a
// lane holds for the tiles of one block are 16 contiguous bytes (the next
// layer's weights are packed with the same K order).  Row r keeps its
// 16-byte chunks in XOR order: logical chunk c is stored at c ^ (r & 15).
// With the LDS serving 16 consecutive lanes per pass, the 16-byte reads of
// the B operand (16 rows, one chunk) and the 16-byte writes of the epilogue
// (16 rows, one chunk) both hit 16 distinct bank groups.
__device__ __forceinline__ int h_chunk(int row, int chunk) { return (chunk ^ (row & 15)) * 8; }

// logical neuron index of physical activation column p
__host__ __device__ __forceinline__ int h_neuron(int p)
{
    return (p & ~31) + (((p >> 2) & 1) << 4) + (((p >> 3) & 3) << 2) + (p & 3);
}

// GELU of a wave's 64 neurons x TILE rows (biases already in the
// accumulators), written to H as 16-byte chunks (tiles 2m and 2m + 1 of a
// wave form block 2w + m)
template <int TILE>
__device__ __forceinline__ void epilogue(floatx4 (&acc)[4][TILE / 16], __bf16* H, int w, int q, int c16)
{
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int chunk = 4 * (2 * w + m) + q;
#pragma unroll
        for (int i = 0; i < TILE / 16; ++i) {
            bf16x8 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = (__bf16)gelu_sig(acc[2 * m][i][e]);
                v[4 + e] = (__bf16)gelu_sig(acc[2 * m + 1][i][e]);
            }
            const int r = 16 * i + c16;
            *reinterpret_cast<bf16x8*>(H + r * kHRow + h_chunk(r, chunk)) = v;
        }
    }
}

}  // namespace

// Fragment-ordered bf16 weights of every member from the fp32 masters.
//   layer 1 : [16 neuron tiles][64 lanes][8]; lane l of tile t holds neuron
//             16t + l%16 and, by quarter q = l/16: q0 W_hi[0..7], q1 W_hi[0..7],
//             q2 W_lo[0..7], q3 zero (matching x_hi, x_lo, x_hi, 0 in B).
//   hidden  : [16 neuron tiles][8 k-steps][64 lanes][8]: neuron 16t + l%16,
//             inputs 32s + 8q .. 32s + 8q + 7.
//   output  : [8 k-steps][64 lanes][8]: neuron l%16 (zero beyond 3).
__global__ void pack_infer_kernel(const float* __restrict__ params, __bf16* __restrict__ pk)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (e >= kPkParams) return;
    const float* P = params + (size_t)m * kParams;
    float v = 0.0f;
    if (e < kPkOffL2) {
        const int t = (int)(e / 512), l = (int)(e / 8) % 64, j = (int)(e % 8), q = l / 16;
        const int n = 16 * t + l % 16;
        const float w = P[kOffW1 + j * kHidden + n];
        const float hi = (float)(__bf16)w;
        v = q == 3 ? 0.0f : (q == 2 ? w - hi : w);
    } else if (e < kPkOffOut) {
        const size_t r = (e - kPkOffL2) % kPkHid;
        const int layer = (int)((e - kPkOffL2) / kPkHid);
        const int t = (int)(r / 4096), s = (int)(r / 512) % 8, l = (int)(r / 8) % 64, j = (int)(r % 8);
        const int n = 16 * t + l % 16, k = h_neuron(32 * s + 8 * (l / 16) + j);
        const size_t off = layer == 0 ? kOffW2 : layer == 1 ? kOffW3 : kOffW4;
        v = P[off + (size_t)k * kHidden + n];
    } else {
        const size_t r = e - kPkOffOut;
        const int s = (int)(r / 512), l = (int)(r / 8) % 64, j = (int)(r % 8);
        const int n = l % 16, k = h_neuron(32 * s + 8 * (l / 16) + j);
        v = n < 3 ? P[kOffW5 + k * 3 + n] : 0.0f;
    }
    pk[(size_t)m * kPkParams + e] = (__bf16)v;
}

template <int TILE>
__global__ __launch_bounds__(256, TILE == 128 ? 2 : 3) void mlp_infer_kernel(InferArgs a)
{
    constexpr int kTile = TILE;                    // rows per workgroup
    constexpr int OT = TILE / 64;                  // output-layer row tiles per wave
    __shared__ __attribute__((aligned(16))) __bf16 H[kTile * kHRow];
    __shared__ __attribute__((aligned(16))) __bf16 X[kTile * kXRow];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, c16 = lane & 15;
    const int64_t row0 = (int64_t)blockIdx.x * kTile;

    // standardised inputs split into bf16 high / low parts: X[r] = x_hi, x_lo, x_hi, 0
    if (tid < kTile) {
        const int64_t row = row0 + tid;
        bf16x8 hi8, lo8;
#pragma unroll
        for (int k = 0; k < kFeatures; ++k) {
            float v = 0.0f;
            if (row < a.n) v = (a.x[row * kFeatures + k] - a.stats[k]) * a.stats[kFeatures + k];
            const __bf16 h = (__bf16)v;
            hi8[k] = h;
            lo8[k] = (__bf16)(v - (float)h);
        }
        __bf16* xr = X + tid * kXRow;
        *reinterpret_cast<bf16x8*>(xr) = hi8;
        *reinterpret_cast<bf16x8*>(xr + 8) = lo8;
        *reinterpret_cast<bf16x8*>(xr + 16) = hi8;
        bf16x8 z8;
#pragma unroll
        for (int k = 0; k < 8; ++k) z8[k] = (__bf16)0.0f;
        *reinterpret_cast<bf16x8*>(xr + 24) = z8;
    }

    float sum[OT][3], mn[OT][3], mx[OT][3];
#pragma unroll
    for (int i = 0; i < OT; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) { sum[i][c] = 0.0f; mn[i][c] = 1e30f; mx[i][c] = -1e30f; }

    const floatx4 zero4 = {0.f, 0.f, 0.f, 0.f};
    for (int m = 0; m < kNets; ++m) {
        const __bf16* P = a.pk + (size_t)m * kPkParams;
        const float* F = a.params + (size_t)m * kParams;
        floatx4 acc[4][kTile / 16];

        // layer 1: one K=32 product per tile
        __syncthreads();   // X written / previous member's output layer done with H
        {
            bf16x8 wf[4];
            floatx4 b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                wf[j] = *reinterpret_cast<const bf16x8*>(P + kPkOffL1 + ((size_t)(4 * w + j) * 64 + lane) * 8);
            bias_quads(b, F + kOffB1, w, q);
#pragma unroll
            for (int i = 0; i < kTile / 16; ++i) {
                const bf16x8 xf = *reinterpret_cast<const bf16x8*>(X + (16 * i + c16) * kXRow + 8 * q);
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j][i] = mfma(wf[j], xf, b[j]);
            }
        }
        epilogue<TILE>(acc, H, w, q, c16);

        // hidden layers 2..4, in place in H.  The weight fragments of k-step
        // s + 1 are in flight while k-step s multiplies (two register sets
        // used in turn, so every wait is for loads issued a step earlier).
#pragma unroll 1
        for (int layer = 0; layer < 3; ++layer) {
            const __bf16* W = P + kPkOffL2 + (size_t)layer * kPkHid + ((size_t)(4 * w) * 8 * 64 + lane) * 8;
            const size_t boff = layer == 0 ? kOffB2 : layer == 1 ? kOffB3 : kOffB4;
            auto load = [&](bf16x8 (&f)[4], int s) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    f[j] = *reinterpret_cast<const bf16x8*>(W + ((size_t)(j * 8 + s) * 64) * 8);
            };
            auto step = [&](const bf16x8 (&f)[4], int s) {
#pragma unroll
                for (int i = 0; i < kTile / 16; ++i) {
                    const int r = 16 * i + c16;
                    const bf16x8 hf = *reinterpret_cast<const bf16x8*>(H + r * kHRow + h_chunk(r, 4 * s + q));
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[j][i] = mfma(f[j], hf, acc[j][i]);
                }
            };
            bf16x8 wa[4], wb[4];
            floatx4 b[4];
            load(wa, 0);
            load(wb, 1);
            bias_quads(b, F + boff, w, q);
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();   // H of the previous layer complete
#pragma unroll
            for (int i = 0; i < kTile / 16; ++i) {
                const int r = 16 * i + c16;
                const bf16x8 hf = *reinterpret_cast<const bf16x8*>(H + r * kHRow + h_chunk(r, q));
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j][i] = mfma(wa[j], hf, b[j]);
            }
            // the scheduling barriers keep each prefetch ahead of the products
            // it overlaps (left alone, the scheduler sinks the loads past them)
#pragma unroll 1
            for (int t = 0; t < 3; ++t) {
                load(wa, 2 * t + 2);
                __builtin_amdgcn_sched_barrier(0);
                step(wb, 2 * t + 1);
                __builtin_amdgcn_sched_barrier(0);
                load(wb, 2 * t + 3);
                __builtin_amdgcn_sched_barrier(0);
                step(wa, 2 * t + 2);
                __builtin_amdgcn_sched_barrier(0);
            }
            step(wb, 7);
            __syncthreads();   // every wave done reading this layer's input
            epilogue<TILE>(acc, H, w, q, c16);
        }

        // output layer: wave w takes the OT row tiles OT w .. OT w + OT - 1
        __syncthreads();
        floatx4 o[OT];
#pragma unroll
        for (int i = 0; i < OT; ++i) o[i] = zero4;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bf16x8 wf = *reinterpret_cast<const bf16x8*>(P + kPkOffOut + ((size_t)s * 64 + lane) * 8);
#pragma unroll
            for (int i = 0; i < OT; ++i) {
                const int r = 16 * (OT * w + i) + c16;
                const bf16x8 hf = *reinterpret_cast<const bf16x8*>(H + r * kHRow + h_chunk(r, 4 * s + q));
                o[i] = mfma(wf, hf, o[i]);
            }
        }
        if (q == 0) {   // lanes 0..15 hold logits 0..3 of rows 16 (OT w + i) + lane
#pragma unroll
            for (int i = 0; i < OT; ++i) {
                float l[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) l[c] = o[i][c] + F[kOffB5 + c];
                const float lm = fmaxf(l[0], fmaxf(l[1], l[2]));
                float e[3], se = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) { e[c] = __expf(l[c] - lm); se += e[c]; }
                const float is = 1.0f / se;
                const int64_t row = row0 + 16 * (OT * w + i) + c16;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // the rounded probability is what the members output holds;
                    // no contraction, so the mean is the same sum of the same
                    // values whichever register tile the row sits in
#pragma clang fp contract(off)
                    const float p = e[c] * is;
                    sum[i][c] = sum[i][c] + p;
                    mn[i][c] = fminf(mn[i][c], p);
                    mx[i][c] = fmaxf(mx[i][c], p);
                    if (a.members && row < a.n) a.members[((size_t)m * a.n + row) * 3 + c] = p;
                }
            }
        }
    }

    if (q == 0) {
#pragma unroll
        for (int i = 0; i < OT; ++i) {
            const int64_t row = row0 + 16 * (OT * w + i) + c16;
            if (row >= a.n) continue;
            float spread = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) spread = fmaxf(spread, mx[i][c] - mn[i][c]);
            const float* xr = a.x + row * kFeatures;
            bool in = a.eligible ? a.eligible[row] != 0 : true;
#pragma unroll
            for (int k = 0; k < kFeatures; ++k)
                in = in && xr[k] >= a.stats[2 * kFeatures + k] && xr[k] <= a.stats[3 * kFeatures + k];
            if (a.rat)
#pragma unroll
                for (int c = 0; c < 3; ++c) a.rat[row * 3 + c] = sum[i][c] / (float)kNets;
            if (a.spread) a.spread[row] = spread;
            if (a.in_domain) a.in_domain[row] = in ? 1 : 0;
        }
    }
}

hipError_t launch_pack_infer(const float* params, __bf16* pk, int nets, hipStream_t st)
{
    hipLaunchKernelGGL(pack_infer_kernel, dim3((unsigned)((kPkParams + 255) / 256), nets), dim3(256), 0, st, params,
                       pk);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const InferArgs& a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = (a.n + kInferTile - 1) / kInferTile;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_infer_kernel<kInferTile>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace fos
