// runtime.hip -- host side of libfos_mc: contexts, argument checks, device
// scratch, the validation verdict, launch-configuration defaults and the
// C-ABI entry points declared in include/fos_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "fos_device.hpp"
#include "fos_kernels.hpp"
#include "fos_mc.h"
#include "fos_ctx.hpp"

using fosrt::DeviceGuard;
using fosrt::fail;
using fosrt::grow;
using fosrt::hip_fail;

namespace {

const char* field_name(int code)
{
    switch (code) {
    case fos::kErrNLayers: return "n_layers (must be 1..max_layers)";
    case fos::kErrMuS: return "mu_s (must be finite and >= 0)";
    case fos::kErrMuA: return "mu_a (must be finite and >= 0)";
    case fos::kErrG: return "g (must be in [-1, 1])";
    case fos::kErrNLayer: return "n_layer (must be finite and >= 1)";
    case fos::kErrThickness: return "thickness (must be finite and > 0)";
    case fos::kErrNUpper: return "n_upper (must be finite and >= 1)";
    case fos::kErrNLower: return "n_lower (must be finite and > 0)";
    case fos::kErrKLower: return "k_lower (must be finite and >= 0)";
    case fos::kErrMu0: return "mu0 (must be in (0, 1])";
    default: return "unknown field";
    }
}

fos_status check_launch(fos_ctx* c, const fos_mc_launch& L)
{
    if (L.block_size < 64 || L.block_size > 1024 || L.block_size % 64)
        return fail(c, FOS_E_INVALID_ARG, "launch.block_size must be a multiple of 64 in [64, 1024]");
    if (L.refill_min < 1 || L.refill_min > 64)
        return fail(c, FOS_E_INVALID_ARG, "launch.refill_min must be in [1, 64]");
    if (L.chunk < 1) return fail(c, FOS_E_INVALID_ARG, "launch.chunk must be >= 1");
    if (L.blocks_per_cu < 1 || L.blocks_per_cu > 64)
        return fail(c, FOS_E_INVALID_ARG, "launch.blocks_per_cu must be in [1, 64]");
    if (L.max_steps < 1 || L.max_steps > 0xFFFFFFFFull)
        return fail(c, FOS_E_INVALID_ARG, "launch.max_steps must be in [1, 2^32-1]");
    if (L.tail_lanes < -1 || L.tail_lanes > 64)
        return fail(c, FOS_E_INVALID_ARG, "launch.tail_lanes must be in [-1, 64]");
    if (L.regroup_lanes < -1 || L.regroup_lanes > 32)
        return fail(c, FOS_E_INVALID_ARG, "launch.regroup_lanes must be in [-1, 32]");
    return FOS_OK;
}

// Chunk for a launch that names none while the context default was never
// fixed: the largest power of two at most (a bound on the batch's photons) /
// (4 x resident waves), within [256, the built-in default], so that a small
// batch still hands every wave several claims.
constexpr int32_t kAutoChunkMin = 256;
constexpr int32_t kAutoChunkMax = 2048;

int32_t auto_chunk_for(int n_cu, int32_t n_items, uint64_t max_photons, const fos_mc_launch& L)
{
    const uint64_t n = (uint64_t)std::max(n_items, 1);
    const uint64_t bound = max_photons > UINT64_MAX / n ? UINT64_MAX : max_photons * n;
    const uint64_t waves = (uint64_t)n_cu * (uint64_t)L.blocks_per_cu * (uint64_t)(L.block_size / 64);
    const uint64_t per = bound / (4 * std::max<uint64_t>(waves, 1));
    int32_t chunk = kAutoChunkMax;
    while (chunk > kAutoChunkMin && (uint64_t)chunk > per) chunk /= 2;
    return chunk;
}

int32_t auto_chunk(const fos_ctx* c, const fos_mc_launch& L)
{
    return auto_chunk_for(c->n_cu, c->n_items, c->max_photons, L);
}

fos_mc_launch merge(const fos_mc_launch& d, const fos_mc_launch* o)
{
    fos_mc_launch r = d;
    if (!o) return r;
    if (o->block_size) r.block_size = o->block_size;
    if (o->refill_min) r.refill_min = o->refill_min;
    if (o->chunk) r.chunk = o->chunk;
    if (o->blocks_per_cu) r.blocks_per_cu = o->blocks_per_cu;
    if (o->max_steps) r.max_steps = o->max_steps;
    if (o->tail_lanes) r.tail_lanes = o->tail_lanes;
    if (o->regroup_lanes) r.regroup_lanes = o->regroup_lanes;
    return r;
}


// The launch a walk runs with: the caller's non-zero knobs over the context
// defaults, and the per-problem chunk where neither fixes one.
fos_mc_launch resolve(const fos_ctx* c, const fos_mc_launch* o)
{
    fos_mc_launch r = merge(c->defaults, o);
    if (!(o && o->chunk) && !c->chunk_set) r.chunk = auto_chunk(c, r);
    return r;
}

// Scratch of the allocation-free walk (fos_mc_run_noalloc): the packed item
// table, the chunk prefix and the status and queue words live in this
// file-scope device array instead of context allocations.  Each device that
// loads the library holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives for that
// device (kept per device below), never through the array's name.
constexpr size_t kNoAllocWordsBytes = 256;   // [0] validation verdict, [1] largest budget, [2] chunk counter
static __device__ __align__(256) unsigned char scratch[FOS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// With `device` current: the device address of its copy of `scratch`, taken
// once per device.
hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch[device] = static_cast<unsigned char*>(p);
    return e;
}

unsigned char* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// --- launch cache of the tuner: a JSON object, one entry per (device
// architecture, item class), each the tuned knobs and their time --------------
struct CachedLaunch {
    fos_mc_launch L{};
    double ms = 0.0;
};

std::map<std::string, CachedLaunch> read_launch_cache(const std::string& path)
{
    std::map<std::string, CachedLaunch> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    while ((pos = t.find('"', pos)) != std::string::npos) {
        const size_t kend = t.find('"', pos + 1);
        if (kend == std::string::npos) break;
        const std::string key = t.substr(pos + 1, kend - pos - 1);
        const size_t ob = t.find('{', kend), cb = t.find('}', kend);
        if (ob == std::string::npos || cb == std::string::npos || cb < ob) break;
        const std::string body = t.substr(ob + 1, cb - ob - 1);
        auto field = [&](const char* name, double& v) {
            const std::string pat = std::string("\"") + name + "\":";
            const size_t p = body.find(pat);
            if (p == std::string::npos) return false;
            return std::sscanf(body.c_str() + p + pat.size(), "%lf", &v) == 1;
        };
        double bs, rm, ch, bpc, tl, ms;
        if (field("block_size", bs) && field("refill_min", rm) && field("chunk", ch) &&
            field("blocks_per_cu", bpc) && field("tail_lanes", tl) && field("ms", ms)) {
            CachedLaunch e;
            e.L.block_size = (int32_t)bs; e.L.refill_min = (int32_t)rm; e.L.chunk = (int32_t)ch;
            e.L.blocks_per_cu = (int32_t)bpc; e.L.tail_lanes = (int32_t)tl;
            e.ms = ms;
            out[key] = e;
        }
        pos = cb + 1;
    }
    return out;
}

bool write_launch_cache(const std::string& path, const std::map<std::string, CachedLaunch>& entries)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t k = 0;
        for (const auto& kv : entries) {
            const fos_mc_launch& L = kv.second.L;
            char buf[512];
            std::snprintf(buf, sizeof buf,
                          " \"%s\": {\"block_size\": %d, \"refill_min\": %d, \"chunk\": %d, \"blocks_per_cu\": %d, "
                          "\"tail_lanes\": %d, \"ms\": %.4f}%s\n",
                          kv.first.c_str(), L.block_size, L.refill_min, L.chunk, L.blocks_per_cu, L.tail_lanes,
                          kv.second.ms, ++k < entries.size() ? "," : "");
            f << buf;
        }
        f << "}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

extern "C" {

int fos_abi_version(void) { return FOS_ABI_VERSION; }

const char* fos_status_string(fos_status s)
{
    switch (s) {
    case FOS_OK: return "FOS_OK";
    case FOS_E_INVALID_ARG: return "FOS_E_INVALID_ARG";
    case FOS_E_UNSUPPORTED: return "FOS_E_UNSUPPORTED";
    case FOS_E_DEVICE: return "FOS_E_DEVICE";
    case FOS_E_OUT_OF_MEMORY: return "FOS_E_OUT_OF_MEMORY";
    case FOS_E_INTERNAL: return "FOS_E_INTERNAL";
    case FOS_E_NOT_PREPARED: return "FOS_E_NOT_PREPARED";
    }
    return "FOS_E_UNKNOWN";
}

fos_status fos_create(int hip_device, fos_ctx** out)
{
    if (!out) return FOS_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return FOS_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return FOS_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FOS_E_DEVICE;
    fos_ctx* c = new (std::nothrow) fos_ctx();
    if (!c) return FOS_E_OUT_OF_MEMORY;
    c->device = hip_device;
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    c->defaults.block_size = 256;
    c->defaults.refill_min = 8;
    c->defaults.chunk = 2048;
    c->defaults.blocks_per_cu = 8;
    c->defaults.max_steps = 100000000ull;
    c->defaults.tail_lanes = -1;
    c->defaults.regroup_lanes = -1;
    DeviceGuard g(hip_device);
    if (hipMalloc(reinterpret_cast<void**>(&c->chunk_counter), 256) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->err_dev), 256) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->nmax_dev), 256) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->seed_dev), 256) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->aux_host), 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->err_host), sizeof(unsigned long long)) != hipSuccess) {
        fos_destroy(c);
        return FOS_E_OUT_OF_MEMORY;
    }
    if (scratch_init(hip_device) != hipSuccess) {
        fos_destroy(c);
        return FOS_E_DEVICE;
    }
    *out = c;
    return FOS_OK;
}

void fos_destroy(fos_ctx* c)
{
    if (!c) return;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        if (c->table) (void)hipFree(c->table);
        if (c->chunk_prefix) (void)hipFree(c->chunk_prefix);
        if (c->chunk_counter) (void)hipFree(c->chunk_counter);
        if (c->err_dev) (void)hipFree(c->err_dev);
        if (c->err_host) (void)hipHostFree(c->err_host);
        if (c->aux_host) (void)hipHostFree(c->aux_host);
        if (c->nmax_dev) (void)hipFree(c->nmax_dev);
        if (c->cell_of) (void)hipFree(c->cell_of);
        if (c->mie) (void)hipFree(c->mie);
        if (c->mie_scratch) (void)hipFree(c->mie_scratch);
        if (c->mie_order) (void)hipFree(c->mie_order);
        if (c->ln_buf) (void)hipFree(c->ln_buf);
        if (c->tune_tallies) (void)hipFree(c->tune_tallies);
        if (c->tune_table) (void)hipFree(c->tune_table);
        if (c->tune_prefix) (void)hipFree(c->tune_prefix);
        if (c->tune_buf) (void)hipFree(c->tune_buf);
        if (c->hand_buf) (void)hipFree(c->hand_buf);
        if (c->seed_dev) (void)hipFree(c->seed_dev);
        if (c->out_buf) (void)hipFree(c->out_buf);
        if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
        fos_sur_free(c->sur);
    }
    delete c;
}

const char* fos_last_error(const fos_ctx* c) { return c ? c->err.c_str() : "null context"; }

fos_status fos_mc_get_launch(const fos_ctx* c, fos_mc_launch* out)
{
    if (!c || !out) return FOS_E_INVALID_ARG;
    *out = c->defaults;
    return FOS_OK;
}

fos_status fos_mc_set_launch(fos_ctx* c, const fos_mc_launch* L)
{
    if (!c || !L) return FOS_E_INVALID_ARG;
    c->err.clear();
    fos_mc_launch m = merge(c->defaults, L);
    fos_status s = check_launch(c, m);
    if (s != FOS_OK) return s;
    c->defaults = m;
    if (L->chunk) c->chunk_set = true;
    return FOS_OK;
}

int32_t fos_mc_prepared_items(const fos_ctx* c) { return (c && c->prepared) ? c->n_items : 0; }

fos_status fos_mc_prepare(fos_ctx* c, const fos_mc_problem* p, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!p) return fail(c, FOS_E_INVALID_ARG, "problem is NULL");
    if (p->n_items < 0) return fail(c, FOS_E_INVALID_ARG, "n_items must be >= 0");
    if (p->max_layers < 1 || p->max_layers > FOS_MAX_LAYERS)
        return fail(c, FOS_E_INVALID_ARG, "max_layers must be in [1, FOS_MAX_LAYERS]");
    if (p->n_items > 0 &&
        (!p->n_layers || !p->mu_s || !p->mu_a || !p->g || !p->n_layer || !p->thickness || !p->n_upper ||
         !p->n_lower || !p->k_lower || !p->mu0 || !p->photons))
        return fail(c, FOS_E_INVALID_ARG, "a problem array pointer is NULL");
    c->prepared = false;
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int rf = fos::rec_f4(p->max_layers);
    hipError_t e = grow(c->table, c->table_bytes, (size_t)std::max(p->n_items, 1) * rf * sizeof(float4));
    if (e != hipSuccess) return hip_fail(c, e, "item table");
    e = grow(c->chunk_prefix, c->chunk_prefix_bytes, ((size_t)p->n_items + 1) * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(c, e, "work queue");
    if (p->n_items > 0) {
        if ((e = fos::launch_fill_u64(c->err_dev, ~0ull, 1, st)) != hipSuccess ||
            (e = fos::launch_fill_u64(c->err_dev + 1, 0ull, 1, st)) != hipSuccess)
            return hip_fail(c, e, "reset");
        fos::PackArgs a{p->n_items, p->max_layers, p->n_layers, p->mu_s, p->mu_a, p->g, p->n_layer,
                        p->thickness, p->n_upper, p->n_lower, p->k_lower, p->mu0, p->photons, c->table,
                        c->err_dev, c->err_dev + 1};
        if ((e = fos::launch_pack(a, st)) != hipSuccess) return hip_fail(c, e, "pack kernel");
        if ((e = hipMemcpyAsync(c->err_host, c->err_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(&c->aux_host[3], c->err_dev + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                st)) != hipSuccess)
            return hip_fail(c, e, "verdict copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "prepare");
        const unsigned long long w = *c->err_host;
        if (w != ~0ull) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "item %llu layer %llu: invalid %s", w >> 16, (w >> 8) & 0xFF,
                          field_name((int)(w & 0xFF)));
            return fail(c, FOS_E_INVALID_ARG, buf);
        }
    }
    c->n_items = p->n_items;
    c->max_layers = p->max_layers;
    c->max_photons = p->n_items > 0 ? (uint64_t)c->aux_host[3] : 0;
    c->prepared = true;
    c->prepare_epoch++;
    return FOS_OK;
}

// Zero the tallies and the chunk counter, then rebuild the chunk prefix for
// this launch's chunk size and photon cap (kernels only: graph-capturable).
static hipError_t enqueue_queue_reset(fos_ctx* c, unsigned long long* tal, int chunk, uint64_t cap, hipStream_t st,
                                      int n_tally = fos::kNTally)
{
    hipError_t e = fos::launch_reset(tal, c->chunk_counter, c->n_items, n_tally, st);
    if (e != hipSuccess) return e;
    return fos::launch_chunk_scan(c->table, fos::rec_f4(c->max_layers), c->n_items, chunk, cap, c->chunk_prefix, st);
}

// Waves of a launch, and records its hand-off list needs (0 without regrouping).
static uint64_t hand_records(const fos_ctx* c, const fos_mc_launch& L)
{
    if (L.regroup_lanes <= 0) return 0;
    return (uint64_t)c->n_cu * (uint64_t)L.blocks_per_cu * (uint64_t)(L.block_size / 64) * (uint64_t)L.regroup_lanes;
}

// Grow the context's hand-off list to what launch L needs (before any
// capture: allocation happens here, never in the enqueued work).
static hipError_t ensure_hand(fos_ctx* c, const fos_mc_launch& L, bool weighted)
{
    const uint64_t cap = hand_records(c, L);
    if (cap == 0) return hipSuccess;
    return grow(c->hand_buf, c->hand_buf_bytes, fos::hand_bytes(cap, weighted));
}

fos_status fos_mc_handoff_counts(fos_ctx* c, uint64_t* handed, uint64_t* lost, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    unsigned long long w[4] = {0, 0, 0, 0};
    if (c->hand_buf) {
        DeviceGuard g(c->device);
        hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
        hipError_t e = hipMemcpyAsync(w, c->hand_buf, sizeof w, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "hand-off counters");
    }
    if (handed) *handed = w[0];
    if (lost) *lost = w[3];
    return FOS_OK;
}

static fos::WalkArgs walk_args(fos_ctx* c, const fos_mc_launch& L, uint64_t seed, unsigned long long* tal)
{
    fos::WalkArgs a{};
    a.table = c->table;
    a.n_items = c->n_items;
    a.max_layers = c->max_layers;
    a.rec_f4 = fos::rec_f4(c->max_layers);
    a.chunk_prefix = c->chunk_prefix;
    a.chunk_counter = c->chunk_counter;
    a.tallies = tal;
    a.seed = seed;
    a.seed_ptr = nullptr;
    a.photon_cap = 0;
    a.max_steps = (uint32_t)L.max_steps;
    a.chunk = L.chunk;
    a.refill_min = L.refill_min;
    a.tail_lanes = L.tail_lanes < 0 ? 0 : L.tail_lanes;
    a.regroup_lanes = L.regroup_lanes < 0 ? 0 : L.regroup_lanes;
    a.regroup_min_waves = c->n_cu;            // one wave per CU
    a.hand = c->hand_buf;
    a.hand_cap = (uint32_t)hand_records(c, L);
    return a;
}

static fos_status execute(fos_ctx* c, uint64_t seed, const fos_mc_launch* launch, uint64_t* tallies, bool weighted,
                          void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!c->prepared) return fail(c, FOS_E_NOT_PREPARED, "no prepared problem (call fos_mc_prepare)");
    if (c->n_items == 0) return FOS_OK;
    if (!tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    const fos_mc_launch L = resolve(c, launch);
    fos_status s = check_launch(c, L);
    if (s != FOS_OK) return s;
    if (weighted && c->max_photons > (1ull << 27))
        return fail(c, FOS_E_UNSUPPORTED, "weighted walk: at most 2^27 photons per item (2^-36 weight units)");
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned long long* tal = reinterpret_cast<unsigned long long*>(tallies);
    hipError_t e = ensure_hand(c, L, weighted);
    if (e != hipSuccess) return hip_fail(c, e, "hand-off list");
    e = enqueue_queue_reset(c, tal, L.chunk, 0, st, weighted ? fos::kNTallyW : fos::kNTally);
    if (e != hipSuccess) return hip_fail(c, e, "reset kernels");
    const fos::WalkArgs a = walk_args(c, L, seed, tal);
    if ((e = fos::launch_reset_handoff(a, st)) != hipSuccess) return hip_fail(c, e, "reset kernels");
    const int grid = c->n_cu * L.blocks_per_cu;
    if ((e = fos::launch_walk(a, grid, L.block_size, st, weighted)) != hipSuccess)
        return hip_fail(c, e, "walk kernel");
    return FOS_OK;
}

fos_status fos_mc_execute(fos_ctx* c, uint64_t seed, const fos_mc_launch* launch, uint64_t* tallies,
                          void* hip_stream)
{
    return execute(c, seed, launch, tallies, false, hip_stream);
}

fos_status fos_mc_execute_weighted(fos_ctx* c, uint64_t seed, const fos_mc_launch* launch, uint64_t* tallies,
                                   void* hip_stream)
{
    return execute(c, seed, launch, tallies, true, hip_stream);
}

fos_status fos_mc_run_weighted(fos_ctx* c, const fos_mc_problem* p, uint64_t seed, const fos_mc_launch* launch,
                               uint64_t* tallies, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    if (launch) {
        const fos_mc_launch L = merge(c->defaults, launch);
        fos_status s = check_launch(c, L);
        if (s != FOS_OK) return s;
    }
    if (p && p->n_items > 0 && !tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    fos_status s = fos_mc_prepare(c, p, hip_stream);
    if (s != FOS_OK) return s;
    return execute(c, seed, launch, tallies, true, hip_stream);
}

fos_status fos_mc_weighted_fractions(fos_ctx* c, int32_t n, const uint64_t* tallies, float* rat, float* se,
                                     void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return FOS_OK;
    if (!tallies || !rat) return fail(c, FOS_E_INVALID_ARG, "tallies and rat must be non-NULL");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_weighted_fractions(n, reinterpret_cast<const unsigned long long*>(tallies), rat, se,
                                                  reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "weighted fractions kernel");
}

fos_status fos_mc_autotune_cache(fos_ctx* c, const char* path)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    c->tune_cache = path ? path : "";
    return FOS_OK;
}

fos_status fos_mc_autotune(fos_ctx* c, uint64_t seed, uint64_t sample_photons, fos_mc_launch* best, float* best_ms,
                           void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!c->prepared) return fail(c, FOS_E_NOT_PREPARED, "no prepared problem (call fos_mc_prepare)");
    if (c->n_items == 0) {
        if (best) *best = c->defaults;
        if (best_ms) *best_ms = 0.f;
        return FOS_OK;
    }
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int n = c->n_items, rf = fos::rec_f4(c->max_layers);
    // 1. estimated photon-steps per photon and budget of every item
    hipError_t e = grow(c->tune_buf, c->tune_buf_bytes, round256((size_t)n * sizeof(float)) + (size_t)n * 8);
    if (e != hipSuccess) return hip_fail(c, e, "tuning scratch");
    float* d_cost = reinterpret_cast<float*>(c->tune_buf);
    uint64_t* d_ph = reinterpret_cast<uint64_t*>(c->tune_buf + round256((size_t)n * sizeof(float)));
    std::vector<float> cost(n);
    std::vector<uint64_t> ph(n);
    if ((e = fos::launch_item_cost(c->table, rf, n, d_cost, d_ph, st)) != hipSuccess ||
        (e = hipMemcpyAsync(cost.data(), d_cost, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ph.data(), d_ph, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "tuning estimates");
    // the item class: layers, mean budget and photon-weighted mean walk
    // length, each on a log2 scale
    double sum_ph = 0.0, sum_steps = 0.0;
    for (int i = 0; i < n; ++i) {
        sum_ph += (double)ph[i];
        sum_steps += (double)ph[i] * (double)cost[i];
    }
    const double mean_ph = sum_ph / n, mean_steps = sum_ph > 0 ? sum_steps / sum_ph : 1.0;
    char key[256];
    std::snprintf(key, sizeof key, "%s|L%d|I%d|N%d|S%d", c->arch.c_str(), c->max_layers,
                  (int)std::lround(std::log2((double)n)), (int)std::lround(std::log2(std::max(mean_ph, 1.0))),
                  (int)std::lround(std::log2(std::max(mean_steps, 1.0))));
    if (!c->tune_cache.empty()) {
        const auto cache = read_launch_cache(c->tune_cache);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            fos_mc_launch L = c->defaults;
            L.block_size = it->second.L.block_size; L.refill_min = it->second.L.refill_min;
            L.chunk = it->second.L.chunk; L.blocks_per_cu = it->second.L.blocks_per_cu;
            L.tail_lanes = it->second.L.tail_lanes;
            if (check_launch(c, L) == FOS_OK) {
                c->defaults = L;
                c->chunk_set = true;
                if (best) *best = L;
                if (best_ms) *best_ms = (float)it->second.ms;
                return FOS_OK;
            }
            c->err.clear();
        }
    }
    // 2. the sample: kTuneItems items in kTuneStrata strata of equal item count
    // by estimated walk length (longest walks included), at their own budgets
    // scaled by one common factor to at most sample_photons in all
    constexpr int kTuneItems = 2048, kTuneStrata = 16;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] < cost[b]; });
    const int m = std::min(n, kTuneItems), strata = std::min(m, kTuneStrata);
    std::vector<int32_t> idx;
    idx.reserve(m);
    for (int s_ = 0; s_ < strata; ++s_) {
        const size_t lo = (size_t)s_ * n / strata, hi = (size_t)(s_ + 1) * n / strata;
        const int k = m / strata + (s_ < m % strata ? 1 : 0);
        for (int j = 0; j < k; ++j) idx.push_back(order[lo + (size_t)j * (hi - lo) / k + (hi - lo) / (2 * k)]);
    }
    double total = 0.0;
    for (int i : idx) total += (double)ph[i];
    const double cap = sample_photons ? (double)sample_photons : (double)(1ull << 30);
    const double f = total > cap ? cap / total : 1.0;
    std::vector<uint64_t> sph(m);
    for (int j = 0; j < m; ++j) {
        const uint64_t N = ph[idx[j]];
        sph[j] = N == 0 ? 0 : std::max<uint64_t>(1, (uint64_t)std::llround((double)N * f));
    }
    if ((e = grow(c->tune_table, c->tune_table_bytes, (size_t)m * rf * sizeof(float4))) != hipSuccess ||
        (e = grow(c->tune_prefix, c->tune_prefix_bytes, ((size_t)m + 1) * sizeof(unsigned long long))) !=
            hipSuccess ||
        (e = grow(c->tune_tallies, c->tune_tallies_bytes, (size_t)m * fos::kNTally * sizeof(unsigned long long))) !=
            hipSuccess)
        return hip_fail(c, e, "tuning scratch");
    // the sample's indices and budgets reuse the estimate buffers
    int32_t* d_idx = reinterpret_cast<int32_t*>(c->tune_buf);
    uint64_t* d_sph = d_ph;
    if ((e = hipMemcpyAsync(d_idx, idx.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(d_sph, sph.data(), (size_t)m * sizeof(uint64_t), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = fos::launch_gather_records(c->table, rf, d_idx, d_sph, m, c->tune_table, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "tuning sample");
    // 3. one knob at a time from the current launch, each candidate timed
    // three times on the sample (best of the last two)
    hipEvent_t ev0, ev1;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
        return fail(c, FOS_E_DEVICE, "event creation failed");
    auto time_one = [&](const fos_mc_launch& L, float& ms) -> hipError_t {
        hipError_t r0 = ensure_hand(c, L, false);
        if (r0 != hipSuccess) return r0;
        fos::WalkArgs a = walk_args(c, L, seed, c->tune_tallies);
        a.table = c->tune_table;
        a.n_items = m;
        a.chunk_prefix = c->tune_prefix;
        const int grid = c->n_cu * L.blocks_per_cu;
        float bestv = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipError_t r;
            if ((r = fos::launch_reset(c->tune_tallies, c->chunk_counter, m, fos::kNTally, st)) != hipSuccess ||
                (r = fos::launch_chunk_scan(c->tune_table, rf, m, L.chunk, 0, c->tune_prefix, st)) != hipSuccess ||
                (r = fos::launch_reset_handoff(a, st)) != hipSuccess)
                return r;
            if ((r = hipEventRecord(ev0, st)) != hipSuccess) return r;
            if ((r = fos::launch_walk(a, grid, L.block_size, st)) != hipSuccess) return r;
            if ((r = hipEventRecord(ev1, st)) != hipSuccess) return r;
            if ((r = hipEventSynchronize(ev1)) != hipSuccess) return r;
            float t = 0.f;
            if ((r = hipEventElapsedTime(&t, ev0, ev1)) != hipSuccess) return r;
            if (rep > 0 && t < bestv) bestv = t;   // first run is a warm-up
        }
        ms = bestv;
        return hipSuccess;
    };
    fos_mc_launch cur = resolve(c, nullptr);
    float cur_ms = 0.f;
    e = time_one(cur, cur_ms);
    const int32_t refills[] = {4, 6, 8, 12, 16};
    const int32_t chunks[] = {512, 1024, 2048, 4096, 8192};
    const int32_t blocks[] = {128, 256, 512};
    const int32_t per_cu[] = {8, 16};
    const int32_t tails[] = {-1, 16};
    for (int knob = 0; knob < 5 && e == hipSuccess; ++knob) {
        const int32_t* vals = knob == 0 ? refills : knob == 1 ? chunks : knob == 2 ? blocks : knob == 3 ? per_cu : tails;
        const int nv = knob == 0 ? 5 : knob == 1 ? 5 : knob == 2 ? 3 : 2;
        for (int i = 0; i < nv && e == hipSuccess; ++i) {
            fos_mc_launch L = cur;
            if (knob == 0) L.refill_min = vals[i];
            if (knob == 1) L.chunk = vals[i];
            if (knob == 2) L.block_size = vals[i];
            if (knob == 3) L.blocks_per_cu = vals[i];
            if (knob == 4) L.tail_lanes = vals[i];
            if (std::memcmp(&L, &cur, sizeof L) == 0) continue;
            float ms = 0.f;
            e = time_one(L, ms);
            if (e == hipSuccess && ms < cur_ms) { cur = L; cur_ms = ms; }
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return hip_fail(c, e, "autotune");
    c->defaults = cur;
    c->chunk_set = true;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (!c->tune_cache.empty()) {
        auto cache = read_launch_cache(c->tune_cache);
        CachedLaunch entry;
        entry.L = cur;
        entry.ms = cur_ms;
        cache[key] = entry;
        if (!write_launch_cache(c->tune_cache, cache))
            return fail(c, FOS_E_INVALID_ARG, "cannot write the launch cache " + c->tune_cache);
    }
    return FOS_OK;
}

fos_status fos_mc_graph_capture(fos_ctx* c, const fos_mc_launch* launch, uint64_t* tallies, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!c->prepared) return fail(c, FOS_E_NOT_PREPARED, "no prepared problem (call fos_mc_prepare)");
    if (c->n_items > 0 && !tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    const fos_mc_launch L = resolve(c, launch);
    fos_status s = check_launch(c, L);
    if (s != FOS_OK) return s;
    DeviceGuard g(c->device);
    hipError_t e;
    if (!c->capture_stream && (e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(c, e, "capture stream");
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    if ((e = ensure_hand(c, L, false)) != hipSuccess) return hip_fail(c, e, "hand-off list");
    c->graph_hand = L.regroup_lanes > 0 ? c->hand_buf : nullptr;
    // order the capture after the caller's work (the prepared table)
    if ((e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream))) != hipSuccess)
        return hip_fail(c, e, "graph capture");
    unsigned long long* tal = reinterpret_cast<unsigned long long*>(tallies);
    if ((e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(c, e, "begin capture");
    hipError_t e1 = hipSuccess;
    if (c->n_items > 0) {
        fos::WalkArgs a = walk_args(c, L, 0, tal);
        a.seed_ptr = reinterpret_cast<const uint64_t*>(c->seed_dev);
        e1 = enqueue_queue_reset(c, tal, L.chunk, 0, c->capture_stream);
        if (e1 == hipSuccess) e1 = fos::launch_reset_handoff(a, c->capture_stream);
        if (e1 == hipSuccess) e1 = fos::launch_walk(a, c->n_cu * L.blocks_per_cu, L.block_size, c->capture_stream);
    }
    e = hipStreamEndCapture(c->capture_stream, &c->graph);
    if (e1 != hipSuccess) return hip_fail(c, e1, "graph capture launch");
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    if ((e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(c, e, "graph instantiate");
    c->graph_epoch = c->prepare_epoch;
    return FOS_OK;
}

fos_status fos_mc_graph_launch(fos_ctx* c, uint64_t seed, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!c->graph_exec) return fail(c, FOS_E_NOT_PREPARED, "no captured graph (call fos_mc_graph_capture)");
    if (c->graph_epoch != c->prepare_epoch)
        return fail(c, FOS_E_NOT_PREPARED, "problem re-prepared since the graph was captured");
    if (c->graph_hand && c->graph_hand != c->hand_buf)
        return fail(c, FOS_E_NOT_PREPARED, "hand-off list reallocated since the graph was captured (capture again)");
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = fos::launch_fill_u64(c->seed_dev, (unsigned long long)seed, 1, st);
    if (e == hipSuccess) e = hipGraphLaunch(c->graph_exec, st);
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "graph launch");
}

fos_status fos_mc_fractions(fos_ctx* c, int32_t n, const uint64_t* tallies, float* rat, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!tallies || !rat)) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_fractions(n, reinterpret_cast<const unsigned long long*>(tallies), rat,
                                         reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "fractions kernel");
}

fos_status fos_mc_run(fos_ctx* c, const fos_mc_problem* p, uint64_t seed, const fos_mc_launch* launch,
                      uint64_t* tallies, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    if (launch) {
        const fos_mc_launch L = merge(c->defaults, launch);
        fos_status s = check_launch(c, L);
        if (s != FOS_OK) return s;
    }
    if (p && p->n_items > 0 && !tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    fos_status s = fos_mc_prepare(c, p, hip_stream);
    if (s != FOS_OK) return s;
    return fos_mc_execute(c, seed, launch, tallies, hip_stream);
}

fos_status fos_mc_run_noalloc(fos_ctx* c, const fos_mc_problem* p, uint64_t seed, const fos_mc_launch* launch,
                              uint64_t* tallies, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!p) return fail(c, FOS_E_INVALID_ARG, "problem is NULL");
    if (p->n_items < 0) return fail(c, FOS_E_INVALID_ARG, "n_items must be >= 0");
    if (p->max_layers < 1 || p->max_layers > FOS_MAX_LAYERS)
        return fail(c, FOS_E_INVALID_ARG, "max_layers must be in [1, FOS_MAX_LAYERS]");
    if (launch) {
        const fos_mc_launch L = merge(c->defaults, launch);
        fos_status s = check_launch(c, L);
        if (s != FOS_OK) return s;
    }
    if (p->n_items == 0) return FOS_OK;
    if (!p->n_layers || !p->mu_s || !p->mu_a || !p->g || !p->n_layer || !p->thickness || !p->n_upper ||
        !p->n_lower || !p->k_lower || !p->mu0 || !p->photons)
        return fail(c, FOS_E_INVALID_ARG, "a problem array pointer is NULL");
    if (!tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    const int rf = fos::rec_f4(p->max_layers);
    const size_t table_bytes = round256((size_t)p->n_items * rf * sizeof(float4));
    const size_t need = kNoAllocWordsBytes + table_bytes + ((size_t)p->n_items + 1) * sizeof(unsigned long long);
    if (need > FOS_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "problem needs %zu bytes of scratch; fos_mc_run_noalloc holds %zu",
                      need, (size_t)FOS_NOALLOC_SCRATCH_BYTES);
        return fail(c, FOS_E_INVALID_ARG, buf);
    }
    unsigned char* base = scratch_of(c->device);
    if (!base) return fail(c, FOS_E_DEVICE, "scratch address of the device unknown");
    unsigned long long* words = reinterpret_cast<unsigned long long*>(base);
    float4* table = reinterpret_cast<float4*>(base + kNoAllocWordsBytes);
    unsigned long long* prefix = reinterpret_cast<unsigned long long*>(base + kNoAllocWordsBytes + table_bytes);
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e;
    // validate and pack into the scratch table; the verdict comes back
    // through the context's pinned words
    if ((e = fos::launch_fill_u64(words, ~0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_fill_u64(words + 1, 0ull, 1, st)) != hipSuccess)
        return hip_fail(c, e, "reset");
    fos::PackArgs pa{p->n_items, p->max_layers, p->n_layers, p->mu_s, p->mu_a, p->g, p->n_layer, p->thickness,
                     p->n_upper, p->n_lower, p->k_lower, p->mu0, p->photons, table, words, words + 1};
    if ((e = fos::launch_pack(pa, st)) != hipSuccess) return hip_fail(c, e, "pack kernel");
    if ((e = hipMemcpyAsync(c->err_host, words, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&c->aux_host[3], words + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
        return hip_fail(c, e, "verdict copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "validation");
    const unsigned long long w = *c->err_host;
    if (w != ~0ull) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "item %llu layer %llu: invalid %s", w >> 16, (w >> 8) & 0xFF,
                      field_name((int)(w & 0xFF)));
        return fail(c, FOS_E_INVALID_ARG, buf);
    }
    fos_mc_launch L = merge(c->defaults, launch);
    if (!(launch && launch->chunk) && !c->chunk_set)
        L.chunk = auto_chunk_for(c->n_cu, p->n_items, (uint64_t)c->aux_host[3], L);
    fos_status s = check_launch(c, L);
    if (s != FOS_OK) return s;
    if (L.regroup_lanes > 0)
        return fail(c, FOS_E_INVALID_ARG, "launch.regroup_lanes: regrouping needs the context's hand-off list, "
                                          "which the allocation-free walk does not use");
    // queue and walk, as fos_mc_execute does, on the scratch buffers
    unsigned long long* tal = reinterpret_cast<unsigned long long*>(tallies);
    if ((e = fos::launch_reset(tal, words + 2, p->n_items, fos::kNTally, st)) != hipSuccess ||
        (e = fos::launch_chunk_scan(table, rf, p->n_items, L.chunk, 0, prefix, st)) != hipSuccess)
        return hip_fail(c, e, "reset kernels");
    fos::WalkArgs a{};
    a.table = table;
    a.n_items = p->n_items;
    a.max_layers = p->max_layers;
    a.rec_f4 = rf;
    a.chunk_prefix = prefix;
    a.chunk_counter = words + 2;
    a.tallies = tal;
    a.seed = seed;
    a.seed_ptr = nullptr;
    a.photon_cap = 0;
    a.max_steps = (uint32_t)L.max_steps;
    a.chunk = L.chunk;
    a.refill_min = L.refill_min;
    a.tail_lanes = L.tail_lanes < 0 ? 0 : L.tail_lanes;
    if ((e = fos::launch_walk(a, c->n_cu * L.blocks_per_cu, L.block_size, st)) != hipSuccess)
        return hip_fail(c, e, "walk kernel");
    return FOS_OK;
}

int64_t fos_issue_threads(const fos_ctx* c) { return c ? (int64_t)c->n_cu * 8 * 256 : 0; }

fos_status fos_issue_run(fos_ctx* c, int32_t kind, int32_t iters, float* sink, uint64_t* ops, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (kind < FOS_ISSUE_FMA || kind > FOS_ISSUE_MUL) return fail(c, FOS_E_INVALID_ARG, "unknown issue kind");
    if (iters < 1) return fail(c, FOS_E_INVALID_ARG, "iters must be >= 1");
    if (!sink) return fail(c, FOS_E_INVALID_ARG, "sink is NULL");
    DeviceGuard g(c->device);
    const int grid = c->n_cu * 8, block = 256;
    hipError_t e = fos::launch_issue(kind, iters, grid, block, sink, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(c, e, "issue kernel");
    if (ops) *ops = (uint64_t)grid * block * (uint64_t)iters * (uint64_t)fos::issue_ops_per_iteration(kind);
    return FOS_OK;
}

static const char* optics_field_name(int code)
{
    switch (code) {
    case fos::kOptErrLambda: return "lam (must be finite and > 0)";
    case fos::kOptErrNm: return "n_m (must be finite and > 0)";
    case fos::kOptErrKm: return "k_m (must be finite and >= 0)";
    case fos::kOptErrOffsets: return "offsets (must be non-decreasing within [0, offsets[n_cells]])";
    case fos::kOptErrNp: return "n_p (must be finite and > 0)";
    case fos::kOptErrKp: return "k_p (must be finite and >= 0)";
    case fos::kOptErrRadius: return "r (must be finite and > 0)";
    case fos::kOptErrFraction: return "f (must be finite and >= 0)";
    case fos::kOptErrSpread: return "sd (must be finite and >= 0)";
    case fos::kOptErrCore: return "core (0 <= r_core <= r, n_core > 0, k_core >= 0, finite)";
    case fos::kOptErrSpreadCore: return "sd with a core (coated spheres take no size spread)";
    default: return "unknown field";
    }
}

fos_status fos_optics_run(fos_ctx* c, const fos_optics_problem* p, float* mu_s, float* mu_a, float* g,
                          double* out_f64, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!p) return fail(c, FOS_E_INVALID_ARG, "problem is NULL");
    if (p->n_cells < 0) return fail(c, FOS_E_INVALID_ARG, "n_cells must be >= 0");
    if (p->n_cells == 0) return FOS_OK;
    if (!p->lam || !p->n_m || !p->k_m || !p->offsets)
        return fail(c, FOS_E_INVALID_ARG, "a cell array pointer is NULL");
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e;
    // number of particle entries and offsets[0]
    if ((e = hipMemcpyAsync(&c->aux_host[0], p->offsets + p->n_cells, sizeof(int64_t), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(&c->aux_host[1], p->offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "optics offsets");
    const int64_t P = (int64_t)c->aux_host[0];
    if ((int64_t)c->aux_host[1] != 0 || P < 0)
        return fail(c, FOS_E_INVALID_ARG, "offsets[0] must be 0 and offsets[n_cells] >= 0");
    if (P > 0 && (!p->n_p || !p->k_p || !p->r || !p->f))
        return fail(c, FOS_E_INVALID_ARG, "a particle array pointer is NULL");
    if ((e = grow(c->cell_of, c->cell_of_bytes, (size_t)std::max<int64_t>(P, 1) * sizeof(int))) != hipSuccess)
        return hip_fail(c, e, "optics scratch");

    fos::OpticsArgs a{};
    a.n_cells = p->n_cells;
    a.n_entries = P;
    a.lam = p->lam; a.n_m = p->n_m; a.k_m = p->k_m; a.offsets = p->offsets;
    a.n_p = p->n_p; a.k_p = p->k_p; a.r = p->r; a.f = p->f;
    a.sd = p->sd; a.r_core = p->r_core; a.n_core = p->n_core; a.k_core = p->k_core;
    if (a.r_core && (!a.n_core || !a.k_core)) return fail(c, FOS_E_INVALID_ARG, "r_core given without n_core, k_core");
    a.flags = reinterpret_cast<unsigned int*>(c->err_dev + 2);
    a.cell_of = c->cell_of;
    a.mie = c->mie;
    a.nmax = c->nmax_dev;
    a.err = c->err_dev;
    a.out_mu_s = mu_s; a.out_mu_a = mu_a; a.out_g = g; a.out_f64 = out_f64;
    if ((e = fos::launch_fill_u64(c->err_dev, ~0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_fill_u64(c->err_dev + 2, 0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_fill_u64(reinterpret_cast<unsigned long long*>(c->nmax_dev), 0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_optics_scan(a, st)) != hipSuccess)
        return hip_fail(c, e, "optics scan");
    if ((e = hipMemcpyAsync(c->err_host, c->err_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&c->aux_host[2], c->nmax_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipMemcpyAsync(&c->aux_host[1], c->err_dev + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "optics verdict");
    const unsigned int oflags = (unsigned int)(c->aux_host[1] & 0xFFFFFFFFull);
    a.units = (oflags & fos::kOptHasSpread) ? fos::kSpreadSizes : 1;
    a.d_arrays = (oflags & fos::kOptHasCore) ? 3 : 1;
    const unsigned long long w = *c->err_host;
    if (w != ~0ull) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "cell %llu: invalid %s", w >> 8, optics_field_name((int)(w & 0xFF)));
        return fail(c, FOS_E_INVALID_ARG, buf);
    }
    const int nn_cap = (int)(c->aux_host[2] & 0xFFFFFFFFull);
    if (nn_cap > (1 << 20)) return fail(c, FOS_E_UNSUPPORTED, "Mie series longer than 2^20 terms");
    if ((e = grow(c->mie, c->mie_bytes, (size_t)std::max<int64_t>(P, 1) * a.units * 3 * sizeof(double))) !=
        hipSuccess)
        return hip_fail(c, e, "optics scratch");
    a.mie = c->mie;
    const int block = 256;
    int grid = c->n_cu * 4;
    const int64_t need = (P * a.units + block - 1) / block;
    if (need < grid) grid = (int)std::max<int64_t>(need, 1);
    a.nn_cap = std::max(nn_cap, 1);
    const size_t nthreads = (size_t)grid * block;
    if ((e = grow(c->mie_scratch, c->mie_scratch_bytes,
                  (size_t)a.d_arrays * ((size_t)a.nn_cap + 1) * nthreads * sizeof(double2))) != hipSuccess)
        return hip_fail(c, e, "Mie scratch");
    a.scratch = c->mie_scratch;
    // size units sorted by series length when there are enough to matter
    a.order = nullptr;
    const int64_t n_units = P * a.units;
    if (n_units > 4096 && n_units < 0xFFFFFFFFll) {
        if ((e = grow(c->mie_order, c->mie_order_bytes, fos::mie_order_bytes(n_units))) != hipSuccess)
            return hip_fail(c, e, "Mie order scratch");
        if ((e = fos::launch_mie_order(a, n_units, c->mie_order, st)) != hipSuccess) return hip_fail(c, e, "Mie order");
        a.order = c->mie_order;
    }
    a.queue = c->err_dev + 4;
    if ((e = fos::launch_fill_u64(a.queue, 0ull, 1, st)) != hipSuccess) return hip_fail(c, e, "Mie queue");
    if ((e = fos::launch_mie(a, grid, block, st)) != hipSuccess) return hip_fail(c, e, "Mie kernel");
    if ((e = fos::launch_emt(a, st)) != hipSuccess) return hip_fail(c, e, "effective-medium kernel");
    return FOS_OK;
}

static const char* lognormal_field_name(int code)
{
    switch (code) {
    case fos::kLnErrSpecies: return "species index";
    case fos::kLnErrMatrix: return "matrix index";
    case fos::kLnErrRmed: return "median-radius index";
    case fos::kLnErrFraction: return "f (must be within [0, 1])";
    default: return "unknown field";
    }
}

fos_status fos_optics_lognormal(fos_ctx* c, const fos_lognormal_problem* p, float* mu_s, float* mu_a, float* g,
                                void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!p) return fail(c, FOS_E_INVALID_ARG, "problem is NULL");
    const int L = p->n_lambda, S = p->n_species, M = p->n_matrix, K = p->n_rmed, B = p->n_bins;
    if (L < 1 || S < 1 || M < 1 || K < 1 || B < 1 || p->n_designs < 0)
        return fail(c, FOS_E_INVALID_ARG, "n_lambda, n_species, n_matrix, n_rmed, n_bins must be >= 1, n_designs >= 0");
    if (!p->lambda || !p->n_p || !p->k_p || !p->n_m || !p->w)
        return fail(c, FOS_E_INVALID_ARG, "a table array pointer is NULL");
    if (p->n_designs > 0 && (!p->species || !p->matrix || !p->rmed || !p->f))
        return fail(c, FOS_E_INVALID_ARG, "a design array pointer is NULL");
    if (!(p->r0 > 0.0) || !std::isfinite(p->r0) || !(p->dlnr > 0.0) || !std::isfinite(p->dlnr))
        return fail(c, FOS_E_INVALID_ARG, "r0 and dlnr must be finite and > 0");
    if (!(p->k_m >= 0.0) || !std::isfinite(p->k_m)) return fail(c, FOS_E_INVALID_ARG, "k_m must be finite and >= 0");
    for (int l = 0; l < L; ++l)
        if (!(p->lambda[l] > 0.0) || !std::isfinite(p->lambda[l]))
            return fail(c, FOS_E_INVALID_ARG, "lambda must be finite and > 0");
    for (int i = 0; i < S * L; ++i)
        if (!(p->n_p[i] > 0.0) || !std::isfinite(p->n_p[i]) || !(p->k_p[i] >= 0.0) || !std::isfinite(p->k_p[i]))
            return fail(c, FOS_E_INVALID_ARG, "particle index must have n_p > 0, k_p >= 0, finite");
    for (int h = 0; h < M; ++h)
        if (!(p->n_m[h] > 0.0) || !std::isfinite(p->n_m[h])) return fail(c, FOS_E_INVALID_ARG, "n_m must be finite and > 0");
    for (int b = 0; b < B; ++b)
        if (!(p->w[b] >= 0.0) || !std::isfinite(p->w[b])) return fail(c, FOS_E_INVALID_ARG, "w must be finite and >= 0");
    const int J = K + B - 1;
    const double half = 0.5 * (double)(B - 1);
    std::vector<double> radii(J);
    for (int j = 0; j < J; ++j) radii[j] = p->r0 * std::exp(((double)j - half) * p->dlnr);
    if (!std::isfinite(radii[J - 1])) return fail(c, FOS_E_INVALID_ARG, "radius grid overflows");
    // one optics cell per (species, matrix, wavelength, grid radius), one entry each
    const size_t C = (size_t)S * M * L * J;
    if (C > 0x7FFFFFFFull) return fail(c, FOS_E_UNSUPPORTED, "radius grid too large");
    const size_t T = (size_t)S * M * L * K;
    // layout of ln_buf (doubles): lam, n_m, k_m, n_p, k_p, r, f [C each], offsets [C + 1] (int64),
    // radii [J], w [B], lambda [L], table [3 T]
    const size_t n_dbl = 7 * C + (C + 1) + J + B + L + 3 * T;
    std::vector<double> h(n_dbl - 3 * T);
    double* lamc = h.data();
    double *nmc = lamc + C, *kmc = nmc + C, *npc = kmc + C, *kpc = npc + C, *rc = kpc + C, *fc = rc + C;
    int64_t* offc = reinterpret_cast<int64_t*>(fc + C);
    double* rad = reinterpret_cast<double*>(offc + C + 1);
    double *wv = rad + J, *lv = wv + B;
    size_t e = 0;
    for (int s = 0; s < S; ++s)
        for (int hm = 0; hm < M; ++hm)
            for (int l = 0; l < L; ++l)
                for (int j = 0; j < J; ++j, ++e) {
                    lamc[e] = p->lambda[l]; nmc[e] = p->n_m[hm]; kmc[e] = p->k_m;
                    npc[e] = p->n_p[(size_t)s * L + l]; kpc[e] = p->k_p[(size_t)s * L + l];
                    rc[e] = radii[j]; fc[e] = 1.0; offc[e] = (int64_t)e;
                }
    offc[C] = (int64_t)C;
    std::copy(radii.begin(), radii.end(), rad);
    std::copy(p->w, p->w + B, wv);
    std::copy(p->lambda, p->lambda + L, lv);
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t err;
    if ((err = grow(c->ln_buf, c->ln_buf_bytes, n_dbl * sizeof(double))) != hipSuccess)
        return hip_fail(c, err, "log-normal scratch");
    if ((err = hipMemcpyAsync(c->ln_buf, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (err = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, err, "log-normal upload");
    double* d_lamc = c->ln_buf;
    fos_optics_problem grid{};
    grid.n_cells = (int32_t)C;
    grid.lam = d_lamc; grid.n_m = d_lamc + C; grid.k_m = d_lamc + 2 * C;
    grid.n_p = d_lamc + 3 * C; grid.k_p = d_lamc + 4 * C; grid.r = d_lamc + 5 * C; grid.f = d_lamc + 6 * C;
    grid.offsets = reinterpret_cast<const int64_t*>(d_lamc + 7 * C);
    // efficiencies of every grid cell into c->mie (the effective-medium pass writes nothing)
    fos_status st_mie = fos_optics_run(c, &grid, nullptr, nullptr, nullptr, nullptr, hip_stream);
    if (st_mie != FOS_OK) return st_mie;
    fos::LognormalArgs a{};
    a.n_lambda = L; a.n_species = S; a.n_matrix = M; a.n_rmed = K; a.n_bins = B; a.n_radii = J;
    a.mie = c->mie;
    a.radii = d_lamc + 7 * C + (C + 1);
    a.w = a.radii + J;
    a.lam = a.w + B;
    a.k_m = p->k_m;
    a.table = const_cast<double*>(a.lam) + L;
    a.n_designs = p->n_designs;
    a.species = p->species; a.matrix = p->matrix; a.rmed = p->rmed; a.f = p->f;
    a.err = c->err_dev;
    a.out_mu_s = mu_s; a.out_mu_a = mu_a; a.out_g = g;
    if ((err = fos::launch_fill_u64(c->err_dev, ~0ull, 1, st)) != hipSuccess ||
        (err = fos::launch_lognormal_check(a, st)) != hipSuccess ||
        (err = hipMemcpyAsync(c->err_host, c->err_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (err = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, err, "log-normal validation");
    const unsigned long long v = *c->err_host;
    if (v != ~0ull) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "design %llu: invalid %s", v >> 8, lognormal_field_name((int)(v & 0xFF)));
        return fail(c, FOS_E_INVALID_ARG, buf);
    }
    if ((err = fos::launch_lognormal_table(a, st)) != hipSuccess || (err = fos::launch_lognormal_cells(a, st)) != hipSuccess)
        return hip_fail(c, err, "log-normal optics");
    return FOS_OK;
}

fos_status fos_philox_words(fos_ctx* c, int32_t n, const uint64_t* photon, const uint32_t* step,
                            const uint32_t* stream, uint64_t seed, uint32_t* out, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!photon || !step || !stream || !out)) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_philox_words(n, photon, step, stream, seed, out,
                                            reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "philox kernel");
}

fos_status fos_eval_fresnel(fos_ctx* c, int32_t n, const float* ci, const float* ni, const float* nt,
                            const float* kt, float* out, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!ci || !ni || !nt || !kt || !out)) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_eval_fresnel(n, ci, ni, nt, kt, out, reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "fresnel kernel");
}

fos_status fos_eval_hg(fos_ctx* c, int32_t n, const float* g_, const float* u01, float* out, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (n < 0) return fail(c, FOS_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!g_ || !u01 || !out)) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard g(c->device);
    hipError_t e = fos::launch_eval_hg(n, g_, u01, out, reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "hg kernel");
}

}  // extern "C"
