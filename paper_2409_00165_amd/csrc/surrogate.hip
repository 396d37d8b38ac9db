// surrogate.hip -- host side of the surrogate network: training loop,
// ensemble prediction with the validity gate, gradient test hook, model
// (de)serialisation.  All arithmetic runs in mlp_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "fos_ctx.hpp"

using fosrt::DeviceGuard;
using fosrt::fail;
using fosrt::grow;
using fosrt::hip_fail;

namespace {


// split-K partials of the five weight gradients of a training step, one
// region per layer: [nets][splits][M][N] tiles, then [nets][splits][N] column
// sums, M x N at most 256 x 256
constexpr int kSplitkLayers = 5;
constexpr size_t kSplitkLayerFloats = (size_t)fos::kNets * fos::kMaxSplits * (fos::kHidden + 1) * fos::kHidden;

hipError_t alloc_ws(fos_sur_state& S, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) S.ws.push_back(*p);
    return e;
}

void free_ws(fos_sur_state& S)
{
    for (void* p : S.ws) (void)hipFree(p);
    S.ws.clear();
    S.ws_rows = 0;
}

// model buffers (weights, optimiser, stats) -- allocated once
hipError_t ensure_model(fos_sur_state& S)
{
    if (S.params) return hipSuccess;
    const size_t P = (size_t)fos::kNets * fos::kParams * sizeof(float);
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.params), P)) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.m), P)) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.v), P)) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.grads), P)) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.wb), (size_t)fos::kNets * fos::kBfParams * sizeof(__bf16))) !=
        hipSuccess)
        return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.pk), (size_t)fos::kNets * fos::kPkParams * sizeof(__bf16))) !=
        hipSuccess)
        return e;
    return hipMalloc(reinterpret_cast<void**>(&S.stats), 32 * sizeof(float));
}

// training workspaces for `rows` rows per member (a multiple of 64): inputs,
// saved pre-activations and activations, logits and gradient buffers
hipError_t ensure_ws(fos_sur_state& S, int rows)
{
    if (S.ws_rows >= rows) return hipSuccess;
    free_ws(S);
    S.xs = nullptr; S.xb = nullptr; S.ys = nullptr; S.logits = S.probs = S.loss_rows = nullptr;
    S.dlog = nullptr; S.dW5pad = S.dW1pad = S.splitk = nullptr;
    for (int l = 0; l < 4; ++l) { S.Z[l] = nullptr; S.H[l] = nullptr; }
    for (int i = 0; i < 2; ++i) S.dZ[i] = nullptr;
    const size_t R = (size_t)fos::kNets * rows;
    hipError_t e = hipSuccess;
    auto A = [&](void* pp, size_t bytes) {
        if (e == hipSuccess) e = alloc_ws(S, reinterpret_cast<void**>(pp), bytes);
    };
    A(&S.xs, R * fos::kFeatures * sizeof(float));
    A(&S.xb, R * fos::kPadIn * sizeof(__bf16));
    A(&S.ys, R * 3 * sizeof(float));
    A(&S.logits, R * fos::kPadOut * sizeof(float));
    A(&S.probs, R * 3 * sizeof(float));
    A(&S.loss_rows, R * sizeof(float));
    A(&S.dlog, R * fos::kPadOut * sizeof(__bf16));
    for (int l = 0; l < 4; ++l) {
        A(&S.Z[l], R * fos::kHidden * sizeof(float));
        A(&S.H[l], R * fos::kHidden * sizeof(__bf16));
    }
    for (int i = 0; i < 2; ++i) {
        A(&S.dZ[i], R * fos::kHidden * sizeof(__bf16));
    }
    A(&S.dW5pad, (size_t)fos::kNets * fos::kHidden * fos::kPadOut * sizeof(float));
    A(&S.dW1pad, (size_t)fos::kNets * fos::kPadIn * fos::kHidden * sizeof(float));
    A(&S.splitk, kSplitkLayers * kSplitkLayerFloats * sizeof(float));
    if (e == hipSuccess) S.ws_rows = rows;
    return e;
}

fos::GemmArgs gemm(int M, int N, int K, const __bf16* A, long lda, long sA, const __bf16* B, long ldb, long sB,
                   float* Cf, long ldc, long sC, __bf16* Cb, long sCb, const float* bias, long sbias,
                   const float* Z, long sZ)
{
    fos::GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.strideA = sA;
    g.B = B; g.ldb = ldb; g.strideB = sB;
    g.Cf = Cf; g.ldc = ldc; g.strideC = sC;
    g.Cb = Cb; g.strideCb = sCb;
    g.bias = bias; g.strideBias = sbias;
    g.Z = Z; g.strideZ = sZ;
    return g;
}

// Training forward: the batch rows of `sa` gathered and standardised into
// S.xs, then the 4 hidden layers and the logits for sa.rows_pad rows per
// member; the pre-activations Z1..Z4 and activations H1..H4 are kept for the
// backward pass.  (Prediction uses the fused kernel of mlp_infer.hip instead.)
hipError_t forward(fos_sur_state& S, const fos::StdArgs& sa, hipStream_t st)
{
    const int rows_pad = sa.rows_pad;
    const long RH = (long)rows_pad * fos::kHidden;
    const long PS = (long)fos::kParams, BS = (long)fos::kBfParams;
    // gather + standardisation and the first layer in one launch
    hipError_t e = fos::launch_input_layer(sa, S.params, fos::kParams, S.Z[0], S.H[0], fos::kNets, st);
    if (e != hipSuccess) return e;
    const size_t wof[3] = {fos::kBfW2, fos::kBfW3, fos::kBfW4};
    const size_t bof[3] = {fos::kOffB2, fos::kOffB3, fos::kOffB4};
    for (int l = 0; l < 3; ++l) {
        fos::GemmArgs g = gemm(rows_pad, fos::kHidden, fos::kHidden, S.H[l], fos::kHidden, RH, S.wb + wof[l],
                               fos::kHidden, BS, S.Z[l + 1], fos::kHidden, RH, S.H[l + 1], RH, S.params + bof[l], PS,
                               nullptr, 0);
        if ((e = fos::launch_gemm(g, false, false, fos::kEpiBiasGelu, fos::kNets, st)) != hipSuccess) return e;
    }
    fos::GemmArgs g = gemm(rows_pad, fos::kPadOut, fos::kHidden, S.H[3], fos::kHidden, RH, S.wb + fos::kBfW5p,
                           fos::kPadOut, BS, S.logits, fos::kPadOut, (long)rows_pad * fos::kPadOut, nullptr, 0,
                           nullptr, 0, nullptr, 0);
    return fos::launch_gemm(g, false, false, fos::kEpiStore, fos::kNets, st);
}

// Backward pass after a training forward + softmax_ce: fills S.grads.  The
// weight gradients reduce over the batch rows, so they run split-K; each
// layer's weight-gradient partials and the next layer's dZ product share one
// launch, and one more launch adds the partials of all five layers in split
// order into the flat gradient (biases: the column sums of dZ, folded into
// the same products).
hipError_t backward(fos_sur_state& S, int rows, hipStream_t st)
{
    const int R = rows;                       // rows_pad == rows in training
    const long RH = (long)R * fos::kHidden;
    const long PS = (long)fos::kParams, BS = (long)fos::kBfParams;
    const int splits = fos::gemm_splits(R);
    fos::ReduceJobs jobs{};
    // weight-gradient partials of layer slot l into its workspace region, with
    // the bias gradient from the column sums of the same dZ operand
    auto partials = [&](fos::GemmArgs& a, int l, int ncol, float* C, long ldc, int rows_out, int cols_out,
                        float* bias_grad) {
        a.splits = splits; a.ws = S.splitk + (size_t)l * kSplitkLayerFloats; a.partials = true;
        a.colsum = true; a.ncol = ncol; a.csum = bias_grad; a.strideCsum = PS;
        fos::ReduceJob& J = jobs.job[jobs.n++];
        J.ws = a.ws; J.splits = splits; J.M = a.M; J.N = a.N;
        J.C = C; J.ldc = ldc; J.strideC = PS; J.rows_out = rows_out; J.cols_out = cols_out;
        J.ncol = ncol; J.csum = bias_grad; J.strideCsum = PS;
    };
    hipError_t e;
    // dW5 = H4^T dlog (padded to 64 columns, the first 3 kept), db5 = colsum(dlog);
    // dZ4 = (dlog W5^T) * gelu'(Z4)
    fos::GemmArgs g1 = gemm(fos::kHidden, fos::kPadOut, R, S.H[3], fos::kHidden, RH, S.dlog, fos::kPadOut,
                            (long)R * fos::kPadOut, nullptr, fos::kPadOut, 0, nullptr, 0, nullptr, 0, nullptr, 0);
    partials(g1, 0, 3, S.grads + fos::kOffW5, 3, fos::kHidden, 3, S.grads + fos::kOffB5);
    fos::GemmArgs g2 = gemm(R, fos::kHidden, fos::kPadK5, S.dlog, fos::kPadOut, (long)R * fos::kPadOut,
                            S.wb + fos::kBfW5t, fos::kPadK5, BS, nullptr, fos::kHidden, RH, S.dZ[0], RH, nullptr, 0,
                            S.Z[3], RH);
    if ((e = fos::launch_backward_layer(g1, g2, fos::kNets, st)) != hipSuccess) return e;
    // layers 4, 3, 2: dW = H_{l-1}^T dZ_l, db = colsum(dZ_l), dZ_{l-1} = (dZ_l W^T) * gelu'(Z_{l-1})
    const size_t wof[3] = {fos::kOffW4, fos::kOffW3, fos::kOffW2};
    const size_t bof[3] = {fos::kOffB4, fos::kOffB3, fos::kOffB2};
    const size_t wbf[3] = {fos::kBfW4, fos::kBfW3, fos::kBfW2};
    int cur = 0;
    for (int s = 0; s < 3; ++s) {
        const int hl = 2 - s;                 // H index of the layer input: H3, H2, H1
        g1 = gemm(fos::kHidden, fos::kHidden, R, S.H[hl], fos::kHidden, RH, S.dZ[cur], fos::kHidden, RH, nullptr,
                  fos::kHidden, 0, nullptr, 0, nullptr, 0, nullptr, 0);
        partials(g1, 1 + s, fos::kHidden, S.grads + wof[s], fos::kHidden, fos::kHidden, fos::kHidden,
                 S.grads + bof[s]);
        g2 = gemm(R, fos::kHidden, fos::kHidden, S.dZ[cur], fos::kHidden, RH, S.wb + wbf[s], fos::kHidden, BS, nullptr,
                  fos::kHidden, RH, S.dZ[cur ^ 1], RH, nullptr, 0, S.Z[hl], RH);
        if ((e = fos::launch_backward_layer(g1, g2, fos::kNets, st)) != hipSuccess) return e;
        cur ^= 1;
    }
    // layer 1: dW1 = X^T dZ1 (inputs padded to 64, the first 8 rows kept), db1 = colsum(dZ1)
    g1 = gemm(fos::kPadIn, fos::kHidden, R, S.xb, fos::kPadIn, (long)R * fos::kPadIn, S.dZ[cur], fos::kHidden, RH,
              nullptr, fos::kHidden, 0, nullptr, 0, nullptr, 0, nullptr, 0);
    partials(g1, 4, fos::kHidden, S.grads + fos::kOffW1, fos::kHidden, fos::kFeatures, fos::kHidden,
             S.grads + fos::kOffB1);
    if ((e = fos::launch_gemm_partials(g1, fos::kNets, st)) != hipSuccess) return e;
    return fos::launch_splitk_reduce_jobs(jobs, fos::kNets, st);
}

hipError_t softmax(fos_sur_state& S, int rows, int rows_pad, bool targets, hipStream_t st)
{
    fos::SoftmaxArgs a{};
    a.rows = rows; a.rows_pad = rows_pad;
    a.params = S.params; a.pstride = fos::kParams;
    a.logits = S.logits; a.probs = S.probs;
    a.ys = targets ? S.ys : nullptr;
    a.loss_rows = S.loss_rows; a.dlog = S.dlog;
    a.inv_batch = 1.0f / (float)rows;
    return fos::launch_softmax_ce(a, fos::kNets, st);
}

fos::StdArgs std_args(fos_sur_state& S, const float* x, const float* y, int64_t n, int64_t base, int rows,
                      int rows_pad, const uint64_t* perm)
{
    fos::StdArgs a{};
    a.x = x; a.n_src = n; a.base = base; a.rows = rows; a.rows_pad = rows_pad;
    a.perm_mul = perm; a.perm_add = perm ? perm + fos::kNets : nullptr;
    a.mean = S.stats; a.inv_std = S.stats + fos::kFeatures;
    a.xs = S.xs; a.xb = S.xb; a.y = y; a.ys = y ? S.ys : nullptr;
    return a;
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) { const uint64_t t = a % b; a = b; b = t; }
    return a;
}

}  // namespace

static void free_sweep(fos_sur_state& S)
{
    for (void* p : S.sweep) (void)hipFree(p);
    S.sweep.clear();
    S.sweep_cap = 0;
    for (void* p : S.sub) (void)hipFree(p);
    S.sub.clear();
    S.sub_cap = 0;
    S.sub_layers = 0;
}

void fos_sur_free(fos_sur_state& S)
{
    free_sweep(S);
    if (S.total_host) (void)hipHostFree(S.total_host);
    free_ws(S);
    for (float* p : {S.params, S.m, S.v, S.grads, S.stats})
        if (p) (void)hipFree(p);
    if (S.wb) (void)hipFree(S.wb);
    if (S.pk) (void)hipFree(S.pk);
    if (S.perm) (void)hipFree(S.perm);
    S = fos_sur_state();
}

extern "C" {

fos_status fos_sur_features(fos_ctx* c, const fos_mc_problem* p, float* x, uint8_t* eligible, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!p) return fail(c, FOS_E_INVALID_ARG, "problem is NULL");
    if (p->n_items < 0 || p->max_layers < 1 || p->max_layers > FOS_MAX_LAYERS)
        return fail(c, FOS_E_INVALID_ARG, "bad n_items or max_layers");
    if (p->n_items == 0) return FOS_OK;
    if (!x || !p->n_layers || !p->mu_s || !p->mu_a || !p->g || !p->n_layer || !p->thickness || !p->n_upper ||
        !p->n_lower || !p->k_lower || !p->mu0)
        return fail(c, FOS_E_INVALID_ARG, "a NULL array");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_features(p->n_items, p->max_layers, p->n_layers, p->mu_s, p->mu_a, p->g,
                                        p->n_layer, p->thickness, p->n_upper, p->n_lower, p->k_lower, p->mu0, x,
                                        eligible, reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "features kernel");
}

fos_status fos_sur_train(fos_ctx* c, const float* x, const float* y, int64_t n, const fos_train_opts* o,
                         void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!x || !y || !o) return fail(c, FOS_E_INVALID_ARG, "x, y and opts must be non-NULL");
    if (o->epochs < 1) return fail(c, FOS_E_INVALID_ARG, "epochs must be >= 1");
    if (o->batch < 64 || o->batch % 64 || o->batch > (1 << 20))
        return fail(c, FOS_E_INVALID_ARG, "batch must be a multiple of 64 in [64, 2^20]");
    if (n < o->batch) return fail(c, FOS_E_INVALID_ARG, "n must be >= batch");
    if (!(o->lr > 0.f) || !(o->lr_min >= 0.f) || o->lr_min > o->lr)
        return fail(c, FOS_E_INVALID_ARG, "need lr > 0 and 0 <= lr_min <= lr");
    fos_sur_state& S = c->sur;
    if (o->resume && !S.trained) return fail(c, FOS_E_NOT_PREPARED, "resume requested but no model is loaded");
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if ((e = ensure_model(S)) != hipSuccess) return hip_fail(c, e, "model buffers");
    const int B = o->batch;
    if ((e = ensure_ws(S, B)) != hipSuccess) return hip_fail(c, e, "training workspace");
    const int64_t steps_per_epoch = n / B;
    // per-epoch, per-member affine shuffles i -> (a i + b) mod n, gcd(a, n) = 1
    std::mt19937_64 rng(o->seed ^ 0x5EEDF05ull);
    std::vector<uint64_t> perm((size_t)o->epochs * 2 * fos::kNets);
    for (int ep = 0; ep < o->epochs; ++ep)
        for (int m = 0; m < fos::kNets; ++m) {
            uint64_t a;
            do { a = 1 + rng() % (uint64_t)n; } while (gcd64(a, (uint64_t)n) != 1);
            perm[(size_t)ep * 2 * fos::kNets + m] = a;
            perm[(size_t)ep * 2 * fos::kNets + fos::kNets + m] = rng() % (uint64_t)n;
        }
    if ((e = grow(S.perm, S.perm_cap, perm.size() * sizeof(uint64_t))) != hipSuccess) return hip_fail(c, e, "perm");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "train");
    if ((e = hipMemcpy(S.perm, perm.data(), perm.size() * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "perm upload");
    if (!o->resume) {
        // standardisation and validity box from the training rows
        if ((e = fos::launch_feature_stats(x, n, S.stats, st)) != hipSuccess) return hip_fail(c, e, "stats");
        // He initialisation N(0, 2/K), zero biases, zero optimiser state
        std::vector<float> w((size_t)fos::kNets * fos::kParams, 0.f);
        std::mt19937_64 r2(o->seed);
        for (int m = 0; m < fos::kNets; ++m) {
            float* P = w.data() + (size_t)m * fos::kParams;
            auto fill = [&](size_t off, int K, int N) {
                std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)K));
                for (size_t j = 0; j < (size_t)K * N; ++j) P[off + j] = nd(r2);
            };
            fill(fos::kOffW1, fos::kFeatures, fos::kHidden);
            fill(fos::kOffW2, fos::kHidden, fos::kHidden);
            fill(fos::kOffW3, fos::kHidden, fos::kHidden);
            fill(fos::kOffW4, fos::kHidden, fos::kHidden);
            fill(fos::kOffW5, fos::kHidden, 3);
        }
        if ((e = hipMemcpy(S.params, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemsetAsync(S.m, 0, w.size() * sizeof(float), st)) != hipSuccess ||
            (e = hipMemsetAsync(S.v, 0, w.size() * sizeof(float), st)) != hipSuccess ||
            (e = fos::launch_refresh_bf16(S.params, S.wb, fos::kNets, st)) != hipSuccess)
            return hip_fail(c, e, "initialisation");
        S.adam_step = 0;
    }
    if (o->loss_history &&
        (e = hipMemsetAsync(o->loss_history, 0, (size_t)o->epochs * fos::kNets * sizeof(float), st)) != hipSuccess)
        return hip_fail(c, e, "loss history");
    const int64_t total = (int64_t)o->epochs * steps_per_epoch;
    int64_t step = 0;
    for (int ep = 0; ep < o->epochs; ++ep) {
        const uint64_t* pm = S.perm + (size_t)ep * 2 * fos::kNets;
        for (int64_t s = 0; s < steps_per_epoch; ++s, ++step) {
            fos::StdArgs sa = std_args(S, x, y, n, s * B, B, B, pm);
            if ((e = forward(S, sa, st)) != hipSuccess) return hip_fail(c, e, "forward");
            if ((e = softmax(S, B, B, true, st)) != hipSuccess) return hip_fail(c, e, "softmax");
            if ((e = backward(S, B, st)) != hipSuccess) return hip_fail(c, e, "backward");
            const double frac = total > 1 ? (double)step / (double)(total - 1) : 1.0;
            const float lr = o->lr_min + 0.5f * (o->lr - o->lr_min) * (float)(1.0 + std::cos(M_PI * frac));
            S.adam_step++;
            fos::AdamArgs aa{S.params, S.m, S.v, S.grads, S.wb, lr, 0.9f, 0.999f, 1e-8f,
                             (float)(1.0 / (1.0 - std::pow(0.9, (double)S.adam_step))),
                             (float)(1.0 / (1.0 - std::pow(0.999, (double)S.adam_step)))};
            // the Adam step and the batch loss of the epoch's history in one launch
            if ((e = fos::launch_adam_loss(aa, S.loss_rows, B,
                                           o->loss_history ? o->loss_history + (size_t)ep * fos::kNets : nullptr,
                                           (float)(1.0 / ((double)B * steps_per_epoch)), fos::kNets, st)) !=
                hipSuccess)
                return hip_fail(c, e, "adam");
        }
    }
    // host copy of the stats for save()
    if ((e = hipMemcpyAsync(S.stats_host, S.stats, 32 * sizeof(float), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "train");
    S.trained = true;
    return FOS_OK;
}

fos_status fos_sur_predict(fos_ctx* c, const float* x, const uint8_t* eligible, int64_t n, float* rat,
                           float* spread, uint8_t* in_domain, float* members, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    fos_sur_state& S = c->sur;
    if (!S.trained) return fail(c, FOS_E_NOT_PREPARED, "no trained or loaded surrogate");
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return FOS_OK;
    if (!x) return fail(c, FOS_E_INVALID_ARG, "x is NULL");
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // fragment-ordered weights from the current masters, then one fused launch
    // (network of every member + gate) over all rows
    hipError_t e = fos::launch_pack_infer(S.params, S.pk, fos::kNets, st);
    if (e != hipSuccess) return hip_fail(c, e, "inference weights");
    fos::InferArgs ia{};
    ia.n = n; ia.x = x; ia.eligible = eligible; ia.stats = S.stats; ia.params = S.params; ia.pk = S.pk;
    ia.rat = rat; ia.spread = spread; ia.in_domain = in_domain; ia.members = members;
    if ((e = fos::launch_mlp_infer(ia, st)) != hipSuccess) return hip_fail(c, e, "inference");
    return FOS_OK;
}

fos_status fos_sur_grad(fos_ctx* c, const float* x, const float* y, int64_t n, float* grads, float* loss,
                        void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    fos_sur_state& S = c->sur;
    if (!S.trained) return fail(c, FOS_E_NOT_PREPARED, "no trained or loaded surrogate");
    if (n < 64 || n % 64 || n > (1 << 20)) return fail(c, FOS_E_INVALID_ARG, "n must be a multiple of 64 in [64, 2^20]");
    if (!x || !y || !grads) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = ensure_ws(S, (int)n);
    if (e != hipSuccess) return hip_fail(c, e, "workspace");
    const int R = (int)n;
    fos::StdArgs sa = std_args(S, x, y, n, 0, R, R, nullptr);
    if ((e = forward(S, sa, st)) != hipSuccess || (e = softmax(S, R, R, true, st)) != hipSuccess ||
        (e = backward(S, R, st)) != hipSuccess)
        return hip_fail(c, e, "gradient");
    if ((e = hipMemcpyAsync(grads, S.grads, (size_t)fos::kNets * fos::kParams * sizeof(float),
                            hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(c, e, "gradient copy");
    if (loss && (e = fos::launch_loss_sum(S.loss_rows, R, loss, 1.0f / (float)R, false, fos::kNets, st)) != hipSuccess)
        return hip_fail(c, e, "loss");
    return FOS_OK;
}

// per-item sweep scratch for n items (features, flags, compaction)
static hipError_t ensure_sweep(fos_sur_state& S, int64_t n)
{
    if (!S.total_host) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&S.total_host), sizeof(unsigned long long));
        if (e != hipSuccess) return e;
    }
    if (S.sweep_cap >= n) return hipSuccess;
    for (void* p : S.sweep) (void)hipFree(p);
    S.sweep.clear();
    S.sweep_cap = 0;
    hipError_t e = hipSuccess;
    auto A = [&](void* pp, size_t bytes) {
        if (e != hipSuccess) return;
        void** p = reinterpret_cast<void**>(pp);
        e = hipMalloc(p, std::max<size_t>(bytes, 256));
        if (e == hipSuccess) S.sweep.push_back(*p);
    };
    const size_t N = (size_t)n;
    const size_t blocks = (N + fos::kSelectPerBlock - 1) / fos::kSelectPerBlock;
    A(&S.sx, N * fos::kFeatures * sizeof(float));
    A(&S.selig, N);
    A(&S.sdom, N);
    A(&S.sspread, N * sizeof(float));
    A(&S.sblock, 2 * (blocks + 1) * sizeof(unsigned long long));
    A(&S.sidx, N * sizeof(int64_t));
    A(&S.stotal, sizeof(unsigned long long));
    if (e == hipSuccess) S.sweep_cap = n;
    return e;
}

// the gathered fallback sub-problem, sized by the fallback count m
static hipError_t ensure_sub(fos_sur_state& S, int64_t m, int L)
{
    if (S.sub_cap >= m && S.sub_layers >= L) return hipSuccess;
    for (void* p : S.sub) (void)hipFree(p);
    S.sub.clear();
    S.sub_cap = 0;
    hipError_t e = hipSuccess;
    auto A = [&](void* pp, size_t bytes) {
        if (e != hipSuccess) return;
        void** p = reinterpret_cast<void**>(pp);
        e = hipMalloc(p, std::max<size_t>(bytes, 256));
        if (e == hipSuccess) S.sub.push_back(*p);
    };
    const size_t M = (size_t)m;
    A(&S.sub_nl, M * sizeof(int32_t));
    for (int k = 0; k < 5; ++k) A(&S.sub_l[k], M * L * sizeof(float));
    for (int k = 0; k < 4; ++k) A(&S.sub_i[k], M * sizeof(float));
    A(&S.sub_ph, M * sizeof(uint64_t));
    A(&S.sub_tal, M * 6 * sizeof(unsigned long long));
    if (e == hipSuccess) { S.sub_cap = m; S.sub_layers = L; }
    return e;
}

fos_status fos_sweep_run(fos_ctx* c, const fos_mc_problem* p, float spread_max, uint64_t fallback_photons,
                         uint64_t seed, float* rat, float* spread, uint8_t* used_mc, int64_t* n_fallback,
                         void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    fos_sur_state& S = c->sur;
    if (!S.trained) return fail(c, FOS_E_NOT_PREPARED, "no trained or loaded surrogate");
    if (!p || !rat || !used_mc) return fail(c, FOS_E_INVALID_ARG, "problem, rat and used_mc must be non-NULL");
    if (p->n_items < 0 || p->max_layers < 1 || p->max_layers > FOS_MAX_LAYERS)
        return fail(c, FOS_E_INVALID_ARG, "bad n_items or max_layers");
    if (!(spread_max >= 0.f)) return fail(c, FOS_E_INVALID_ARG, "spread_max must be >= 0");
    if (fallback_photons < 1) return fail(c, FOS_E_INVALID_ARG, "fallback_photons must be >= 1");
    if (n_fallback) *n_fallback = 0;
    const int64_t n = p->n_items;
    if (n == 0) return FOS_OK;
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = ensure_sweep(S, n);
    if (e != hipSuccess) return hip_fail(c, e, "sweep scratch");
    fos_status s = fos_sur_features(c, p, S.sx, S.selig, hip_stream);
    if (s != FOS_OK) return s;
    float* spr = spread ? spread : S.sspread;
    s = fos_sur_predict(c, S.sx, S.selig, n, rat, spr, S.sdom, nullptr, hip_stream);
    if (s != FOS_OK) return s;
    fos::SweepSelectArgs sa{};
    sa.n = n; sa.spread = spr; sa.in_domain = S.sdom; sa.spread_max = spread_max; sa.used_mc = used_mc;
    const size_t blocks = ((size_t)n + fos::kSelectPerBlock - 1) / fos::kSelectPerBlock;
    sa.block_count = S.sblock; sa.block_offset = S.sblock + blocks + 1; sa.idx = S.sidx;
    if ((e = fos::launch_select_count(sa, st)) != hipSuccess || (e = fos::launch_select_scan(sa, S.stotal, st)) != hipSuccess ||
        (e = fos::launch_select_write(sa, st)) != hipSuccess ||
        (e = hipMemcpyAsync(S.total_host, S.stotal, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "fallback selection");
    const int64_t m = (int64_t)*S.total_host;
    if (n_fallback) *n_fallback = m;
    if (m == 0) return FOS_OK;
    if (m > 0x7FFFFFFF) return fail(c, FOS_E_UNSUPPORTED, "more than 2^31-1 fallback items");
    if ((e = ensure_sub(S, m, p->max_layers)) != hipSuccess) return hip_fail(c, e, "fallback sub-problem");
    fos::GatherArgs ga{};
    ga.m = m; ga.L = p->max_layers; ga.idx = S.sidx;
    ga.n_layers = p->n_layers; ga.mu_s = p->mu_s; ga.mu_a = p->mu_a; ga.g = p->g; ga.n_layer = p->n_layer;
    ga.thickness = p->thickness; ga.n_upper = p->n_upper; ga.n_lower = p->n_lower; ga.k_lower = p->k_lower;
    ga.mu0 = p->mu0;
    ga.o_n_layers = S.sub_nl;
    ga.o_mu_s = S.sub_l[0]; ga.o_mu_a = S.sub_l[1]; ga.o_g = S.sub_l[2]; ga.o_n_layer = S.sub_l[3];
    ga.o_thickness = S.sub_l[4];
    ga.o_n_upper = S.sub_i[0]; ga.o_n_lower = S.sub_i[1]; ga.o_k_lower = S.sub_i[2]; ga.o_mu0 = S.sub_i[3];
    ga.o_photons = S.sub_ph; ga.photons = fallback_photons;
    if ((e = fos::launch_gather_items(ga, st)) != hipSuccess) return hip_fail(c, e, "fallback gather");
    fos_mc_problem sub{};
    sub.n_items = (int32_t)m; sub.max_layers = p->max_layers; sub.n_layers = S.sub_nl;
    sub.mu_s = S.sub_l[0]; sub.mu_a = S.sub_l[1]; sub.g = S.sub_l[2]; sub.n_layer = S.sub_l[3];
    sub.thickness = S.sub_l[4];
    sub.n_upper = S.sub_i[0]; sub.n_lower = S.sub_i[1]; sub.k_lower = S.sub_i[2]; sub.mu0 = S.sub_i[3];
    sub.photons = S.sub_ph;
    s = fos_mc_run(c, &sub, seed, nullptr, reinterpret_cast<uint64_t*>(S.sub_tal), hip_stream);
    if (s != FOS_OK) return s;
    if ((e = fos::launch_scatter_mc(m, S.sidx, S.sub_tal, rat, st)) != hipSuccess)
        return hip_fail(c, e, "fallback scatter");
    return FOS_OK;
}

fos_status fos_spectral_reduce(fos_ctx* c, int32_t designs, int32_t lambdas, const float* rat, const float* w_r,
                               const float* w_e, float* out, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (designs < 0 || lambdas < 1) return fail(c, FOS_E_INVALID_ARG, "need designs >= 0 and lambdas >= 1");
    if (designs == 0) return FOS_OK;
    if (!rat || !w_r || !w_e || !out) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard guard(c->device);
    hipError_t e = fos::launch_spectral_reduce(designs, lambdas, rat, w_r, w_e, out,
                                               reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "spectral reduction");
}

static const char kMagic[8] = {'F', 'O', 'S', 'S', 'U', 'R', '0', '1'};

fos_status fos_sur_save(const fos_ctx* cc, void* blob, size_t* bytes)
{
    fos_ctx* c = const_cast<fos_ctx*>(cc);
    if (!c || !bytes) return FOS_E_INVALID_ARG;
    c->err.clear();
    fos_sur_state& S = c->sur;
    if (!S.trained) return fail(c, FOS_E_NOT_PREPARED, "no trained or loaded surrogate");
    const size_t P = (size_t)fos::kNets * fos::kParams;
    const size_t need = 8 + 6 * 4 + 32 * 4 + 3 * P * 4;
    if (!blob) { *bytes = need; return FOS_OK; }
    if (*bytes < need) { *bytes = need; return fail(c, FOS_E_INVALID_ARG, "blob too small"); }
    DeviceGuard guard(c->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "save");
    char* b = static_cast<char*>(blob);
    std::memcpy(b, kMagic, 8);
    const uint32_t hdr[6] = {(uint32_t)fos::kNets, (uint32_t)fos::kFeatures, (uint32_t)fos::kHidden,
                             (uint32_t)fos::kParams, 1u, S.adam_step};
    std::memcpy(b + 8, hdr, sizeof hdr);
    std::memcpy(b + 32, S.stats_host, 32 * 4);
    char* d = b + 32 + 128;
    if ((e = hipMemcpy(d, S.params, P * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(d + P * 4, S.m, P * 4, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(d + 2 * P * 4, S.v, P * 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "save");
    *bytes = need;
    return FOS_OK;
}

fos_status fos_sur_load(fos_ctx* c, const void* blob, size_t bytes)
{
    if (!c || !blob) return FOS_E_INVALID_ARG;
    c->err.clear();
    const char* b = static_cast<const char*>(blob);
    if (bytes < 32 + 128 || std::memcmp(b, kMagic, 8) != 0) return fail(c, FOS_E_INVALID_ARG, "not a surrogate blob");
    uint32_t hdr[6];
    std::memcpy(hdr, b + 8, sizeof hdr);
    if (hdr[0] != (uint32_t)fos::kNets || hdr[1] != (uint32_t)fos::kFeatures || hdr[2] != (uint32_t)fos::kHidden ||
        hdr[3] != (uint32_t)fos::kParams)
        return fail(c, FOS_E_UNSUPPORTED, "surrogate architecture differs from this library's");
    const size_t P = (size_t)fos::kNets * fos::kParams;
    const size_t need = 32 + 128 + (hdr[4] ? 3 : 1) * P * 4;
    if (bytes < need) return fail(c, FOS_E_INVALID_ARG, "blob truncated");
    fos_sur_state& S = c->sur;
    DeviceGuard guard(c->device);
    hipError_t e;
    if ((e = ensure_model(S)) != hipSuccess) return hip_fail(c, e, "model buffers");
    std::memcpy(S.stats_host, b + 32, 128);
    const char* d = b + 32 + 128;
    if ((e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(S.stats, S.stats_host, 128, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(S.params, d, P * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "load");
    if (hdr[4]) {
        if ((e = hipMemcpy(S.m, d + P * 4, P * 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(S.v, d + 2 * P * 4, P * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(c, e, "load");
        S.adam_step = hdr[5];
    } else {
        if ((e = hipMemset(S.m, 0, P * 4)) != hipSuccess || (e = hipMemset(S.v, 0, P * 4)) != hipSuccess)
            return hip_fail(c, e, "load");
        S.adam_step = 0;
    }
    if ((e = fos::launch_refresh_bf16(S.params, S.wb, fos::kNets, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(c, e, "load");
    S.trained = true;
    return FOS_OK;
}

}  // extern "C"
