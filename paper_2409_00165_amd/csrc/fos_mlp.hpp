// fos_mlp.hpp -- layout of the surrogate network's parameters and the
// argument blocks of its kernels (mlp_kernels.hip), shared with the host
// runtime (surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fos {

constexpr int kFeatures = 8;     // network inputs
constexpr int kHidden = 256;     // width of the 4 hidden layers
constexpr int kNets = 4;         // ensemble members
constexpr int kPadIn = 64;       // bf16 copy of the inputs, padded for the W1 gradient GEMM
constexpr int kPadOut = 64;      // logits / logit-gradient rows padded to one GEMM tile
constexpr int kPadK5 = 32;       // W5 padded on the class axis for the dH4 GEMM

// flat fp32 parameters of one member: W1 [8][256], b1, W2 [256][256], b2,
// W3, b3, W4, b4, W5 [256][3], b5 (W[k_in][n_out], row-major)
constexpr size_t kOffW1 = 0;
constexpr size_t kOffB1 = kOffW1 + (size_t)kFeatures * kHidden;
constexpr size_t kOffW2 = kOffB1 + kHidden;
constexpr size_t kOffB2 = kOffW2 + (size_t)kHidden * kHidden;
constexpr size_t kOffW3 = kOffB2 + kHidden;
constexpr size_t kOffB3 = kOffW3 + (size_t)kHidden * kHidden;
constexpr size_t kOffW4 = kOffB3 + kHidden;
constexpr size_t kOffB4 = kOffW4 + (size_t)kHidden * kHidden;
constexpr size_t kOffW5 = kOffB4 + kHidden;
constexpr size_t kOffB5 = kOffW5 + (size_t)kHidden * 3;
constexpr size_t kParams = kOffB5 + 3;   // 200,451

// bf16 copies of one member: W2, W3, W4 [256][256], W5p [256][64] (W5 with
// zero columns 3..63), W5t [256][32] (W5 with zero columns 3..31)
constexpr size_t kBfW2 = 0;
constexpr size_t kBfW3 = kBfW2 + (size_t)kHidden * kHidden;
constexpr size_t kBfW4 = kBfW3 + (size_t)kHidden * kHidden;
constexpr size_t kBfW5p = kBfW4 + (size_t)kHidden * kHidden;
constexpr size_t kBfW5t = kBfW5p + (size_t)kHidden * kPadOut;
constexpr size_t kBfParams = kBfW5t + (size_t)kHidden * kPadK5;

// fragment-ordered bf16 weights of one member for the fused inference kernel
// (mlp_infer.hip): layer 1 (hi/lo split), hidden layers 2..4, output layer
constexpr size_t kPkHid = (size_t)16 * 8 * 64 * 8;    // 16 neuron tiles x 8 k-steps x 64 lanes x 8
constexpr size_t kPkOffL1 = 0;
constexpr size_t kPkOffL2 = kPkOffL1 + (size_t)16 * 64 * 8;
constexpr size_t kPkOffOut = kPkOffL2 + 3 * kPkHid;
constexpr size_t kPkParams = kPkOffOut + (size_t)8 * 64 * 8;
#ifndef FOS_INFER_TILE
#define FOS_INFER_TILE 128
#endif
constexpr int kInferTile = FOS_INFER_TILE;             // rows per inference workgroup (64 or 128)
static_assert(kInferTile == 64 || kInferTile == 128, "inference tile must be 64 or 128 rows");

struct InferArgs {
    int64_t n;
    const float* x;              // raw features [n][8]
    const uint8_t* eligible;     // [n] or null (all eligible)
    const float* stats;          // mean[8], 1/std[8], box min[8], box max[8]
    const float* params;         // fp32 masters [nets][kParams] (biases)
    const __bf16* pk;            // [nets][kPkParams]
    float* rat;                  // [n][3] ensemble mean, or null
    float* spread;               // [n] or null
    uint8_t* in_domain;          // [n] or null
    float* members;              // [nets][n][3] or null
};

enum Epilogue : int { kEpiStore = 0, kEpiBiasGelu = 1, kEpiGeluGrad = 2 };

struct GemmArgs {
    int M, N, K;
    const __bf16* A; long lda; long strideA;
    const __bf16* B; long ldb; long strideB;
    float* Cf; long ldc; long strideC;     // fp32 output (may be null for BiasGelu/GeluGrad)
    __bf16* Cb; long strideCb;             // bf16 output, leading dimension ldc
    const float* bias; long strideBias;    // BiasGelu
    const float* Z; long strideZ;          // GeluGrad: saved pre-activation, leading dimension ldc
    // split-K (store epilogue only): K is cut into `splits` equal ranges, each
    // workgroup writes its partial M x N tile to ws [nets][splits][M][N], and a
    // second kernel adds the partials in split order into Cf
    int splits = 1;
    float* ws = nullptr;
    bool partials = false;     // write the partial tiles (and column sums) to ws even for one K range
    // optional (TA, !TB only): the column sums of B over K for the first ncol
    // columns (a bias gradient when B is dZ), written to
    // csum[net * strideCsum + c]; they take the same K ranges and the same
    // ordered reduction as the product
    bool colsum = false; int ncol = 0;
    float* csum = nullptr; long strideCsum = 0;
};

// one ordered split-K sum of a batched training step (splitk_reduce_jobs)
struct ReduceJob {
    const float* ws;           // partial tiles [nets][splits][M][N], then column sums [nets][splits][N]
    int splits, M, N;
    float* C; long ldc; long strideC;
    int rows_out, cols_out;    // the part of the M x N product written to C
    int ncol;                  // column sums written (0 = none)
    float* csum; long strideCsum;
};
constexpr int kMaxReduceJobs = 5;
struct ReduceJobs {
    ReduceJob job[kMaxReduceJobs];
    int n;
};

struct StdArgs {
    const float* x;            // raw features [n_src][8]
    int64_t n_src, base;
    int rows, rows_pad;
    const uint64_t* perm_mul;  // per member (training gather) or null
    const uint64_t* perm_add;
    const float* mean;
    const float* inv_std;
    float* xs;                 // [nets][rows_pad][8]
    __bf16* xb;                // [nets][rows_pad][64] or null
    const float* y;            // [n_src][3] or null
    float* ys;                 // [nets][rows_pad][3] or null
};

struct SoftmaxArgs {
    int rows, rows_pad;
    const float* params; size_t pstride;
    const float* logits;       // [nets][rows_pad][64]
    float* probs;              // [nets][rows_pad][3]
    const float* ys;           // targets or null (inference)
    float* loss_rows;          // [nets][rows_pad]
    __bf16* dlog;              // [nets][rows_pad][64]
    float inv_batch;
};

struct AdamArgs {
    float* w; float* m; float* v;
    const float* grads;
    __bf16* wb;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
};

// sweep: fallback selection, compaction, gather/scatter of sub-problems
struct SweepSelectArgs {
    int64_t n;
    const float* spread; const uint8_t* in_domain;
    float spread_max;
    uint8_t* used_mc;               // fallback flag per item
    unsigned long long* block_count; // [blocks]
    unsigned long long* block_offset;
    int64_t* idx;                   // compacted item indices
};
constexpr int kSelectPerBlock = 2048;   // 256 threads x 8 items

struct GatherArgs {
    int64_t m; int L;
    const int64_t* idx;
    const int32_t* n_layers; const float *mu_s, *mu_a, *g, *n_layer, *thickness;
    const float *n_upper, *n_lower, *k_lower, *mu0;
    int32_t* o_n_layers; float *o_mu_s, *o_mu_a, *o_g, *o_n_layer, *o_thickness;
    float *o_n_upper, *o_n_lower, *o_k_lower, *o_mu0; uint64_t* o_photons;
    uint64_t photons;
};

hipError_t launch_select_count(const SweepSelectArgs& a, hipStream_t st);
hipError_t launch_select_scan(const SweepSelectArgs& a, unsigned long long* total, hipStream_t st);
hipError_t launch_select_write(const SweepSelectArgs& a, hipStream_t st);
hipError_t launch_gather_items(const GatherArgs& a, hipStream_t st);
hipError_t launch_scatter_mc(int64_t m, const int64_t* idx, const unsigned long long* tallies, float* rat,
                             hipStream_t st);
hipError_t launch_spectral_reduce(int designs, int lambdas, const float* rat, const float* w_r, const float* w_e,
                                  float* out, hipStream_t st);

hipError_t launch_pack_infer(const float* params, __bf16* pk, int nets, hipStream_t st);
hipError_t launch_mlp_infer(const InferArgs& a, hipStream_t st);
hipError_t launch_gemm(const GemmArgs& g, bool ta, bool tb, int epi, int nets, hipStream_t st);
// training step, grouped: a layer's split-K weight gradient (g1, partials
// only) with the next dZ product (g2), the partials of a weight gradient
// alone, and the ordered sums of several layers' partials in one launch
hipError_t launch_backward_layer(const GemmArgs& g1, const GemmArgs& g2, int nets, hipStream_t st);
hipError_t launch_gemm_partials(const GemmArgs& g, int nets, hipStream_t st);
hipError_t launch_splitk_reduce_jobs(const ReduceJobs& jobs, int nets, hipStream_t st);
hipError_t launch_input_layer(const StdArgs& a, const float* params, size_t pstride, float* Z1, __bf16* H1, int nets,
                              hipStream_t st);
hipError_t launch_adam_loss(const AdamArgs& a, const float* loss_rows, int rows, float* dst, float scale, int nets,
                            hipStream_t st);
// split-K ranges for a weight-gradient product over K rows: the largest power
// of two up to kMaxSplits that keeps at least 8 k-steps of 32 per range
constexpr int kMaxSplits = 16;
int gemm_splits(int K);
hipError_t launch_features(int n, int L, const int32_t* n_layers, const float* mu_s, const float* mu_a,
                           const float* g, const float* n_layer, const float* thickness, const float* n_upper,
                           const float* n_lower, const float* k_lower, const float* mu0, float* x,
                           uint8_t* eligible, hipStream_t st);
hipError_t launch_softmax_ce(const SoftmaxArgs& a, int nets, hipStream_t st);
hipError_t launch_refresh_bf16(const float* w, __bf16* wb, int nets, hipStream_t st);
hipError_t launch_feature_stats(const float* x, int64_t n, float* stats, hipStream_t st);
// dst[m] = (add ? dst[m] : 0) + scale * (sum of member m's per-row losses [nets][rows])
hipError_t launch_loss_sum(const float* loss_rows, int rows, float* dst, float scale, bool add, int nets,
                           hipStream_t st);

}  // namespace fos
