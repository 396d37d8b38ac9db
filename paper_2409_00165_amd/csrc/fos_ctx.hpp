// fos_ctx.hpp -- the context object behind the C ABI and the host helpers
// shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fos_device.hpp"
#include "fos_kernels.hpp"
#include "fos_mc.h"
#include "fos_mlp.hpp"

struct fos_sur_state {
    bool trained = false;
    uint32_t adam_step = 0;
    float* params = nullptr;     // [4][kParams] fp32 master weights
    float* m = nullptr;          // Adam first moment
    float* v = nullptr;          // Adam second moment
    float* grads = nullptr;      // [4][kParams]
    __bf16* wb = nullptr;        // [4][kBfParams] bf16 copies
    __bf16* pk = nullptr;        // [4][kPkParams] fragment-ordered copies for fused inference
    float* stats = nullptr;      // [32] mean, 1/std, min, max (device)
    float stats_host[32] = {};
    // workspaces, sized for `rows` rows per member
    int ws_rows = 0;
    std::vector<void*> ws;       // every workspace allocation (freed together)
    float* xs = nullptr; __bf16* xb = nullptr; float* ys = nullptr;
    float* Z[4] = {}; __bf16* H[4] = {};
    float* logits = nullptr; float* probs = nullptr; float* loss_rows = nullptr;
    __bf16* dlog = nullptr;
    __bf16* dZ[2] = {};
    float* dW5pad = nullptr; float* dW1pad = nullptr;
    float* splitk = nullptr;     // [4][kMaxSplits][256][256] partial weight-gradient tiles, then
                                 // [4][kMaxSplits][256] partial bias gradients
    uint64_t* perm = nullptr;    // [epochs][4][2]
    size_t perm_cap = 0;
    // sweep scratch
    std::vector<void*> sweep;    // freed together
    int64_t sweep_cap = 0;
    std::vector<void*> sub;      // fallback sub-problem, freed together
    int64_t sub_cap = 0;
    int sub_layers = 0;
    float* sx = nullptr; uint8_t* selig = nullptr; uint8_t* sdom = nullptr; float* sspread = nullptr;
    unsigned long long* sblock = nullptr; int64_t* sidx = nullptr; unsigned long long* stotal = nullptr;
    int32_t* sub_nl = nullptr; float* sub_l[5] = {}; float* sub_i[4] = {}; uint64_t* sub_ph = nullptr;
    unsigned long long* sub_tal = nullptr;
    unsigned long long* total_host = nullptr;
};

struct fos_ctx {
    int device = 0;
    int n_cu = 0;
    std::string err;
    // prepared problem
    int32_t n_items = 0, max_layers = 0;
    bool prepared = false;
    uint64_t max_photons = 0;                // largest photon budget of the prepared problem
    float4* table = nullptr;
    size_t table_bytes = 0;
    unsigned long long* chunk_prefix = nullptr;    // [n_items + 1]
    size_t chunk_prefix_bytes = 0;
    unsigned long long* chunk_counter = nullptr;   // device, 1 word
    // device, 32 words: [0] first validation error, [1] item-table verdict (prepare) /
    // [2] optics kind flags, [4] Mie claim counter
    unsigned long long* err_dev = nullptr;
    unsigned long long* err_host = nullptr;  // pinned host, 1 word
    fos_mc_launch defaults{};
    bool chunk_set = false;                  // defaults.chunk fixed by fos_mc_set_launch or the tuner

    // optics scratch
    int* cell_of = nullptr;
    size_t cell_of_bytes = 0;
    double* mie = nullptr;
    size_t mie_bytes = 0;
    double2* mie_scratch = nullptr;
    size_t mie_scratch_bytes = 0;
    unsigned int* mie_order = nullptr;        // size units by series length, class counts, classes
    size_t mie_order_bytes = 0;
    double* ln_buf = nullptr;                 // log-normal grid cells, radii, weights, bin-sum table
    size_t ln_buf_bytes = 0;
    unsigned int* nmax_dev = nullptr;        // device, 1 word
    unsigned long long* aux_host = nullptr;  // pinned host, 4 words
    // tuning and graph
    std::string arch;                         // gcnArchName of the device
    std::string tune_cache;                   // launch cache file (empty = none)
    unsigned long long* tune_tallies = nullptr;
    size_t tune_tallies_bytes = 0;
    float4* tune_table = nullptr;             // the tuning sample's item records
    size_t tune_table_bytes = 0;
    unsigned long long* tune_prefix = nullptr;
    size_t tune_prefix_bytes = 0;
    unsigned char* tune_buf = nullptr;        // per-item cost and budget; sample indices and budgets
    size_t tune_buf_bytes = 0;
    unsigned char* hand_buf = nullptr;        // hand-off list of regrouping walks
    size_t hand_buf_bytes = 0;
    unsigned char* graph_hand = nullptr;      // the list a captured regrouping graph uses
    unsigned long long* seed_dev = nullptr;  // device, 1 word
    // output stage: weights [5][L], colour parameters [12], then the grid and the spectra
    float* out_buf = nullptr;
    size_t out_buf_bytes = 0;
    int32_t out_lambdas = 0;                  // grid size of the prepared stage (0 = not prepared)
    int32_t out_avail = 0;                    // FOS_OUTPUT_* bits of the prepared stage
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    uint64_t prepare_epoch = 0, graph_epoch = 0;
    // surrogate network
    fos_sur_state sur;
};

void fos_sur_free(fos_sur_state& S);

namespace fosrt {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline fos_status fail(fos_ctx* c, fos_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

inline fos_status hip_fail(fos_ctx* c, hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory)
        return fail(c, FOS_E_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
    return fail(c, FOS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
inline hipError_t grow(T*& p, size_t& cap, size_t need_bytes)
{
    if (need_bytes <= cap && p) return hipSuccess;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(need_bytes, 256);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), want);
    if (e == hipSuccess) cap = want;
    return e;
}

}  // namespace fosrt
