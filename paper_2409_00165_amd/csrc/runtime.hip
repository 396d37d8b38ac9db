// runtime.hip -- host side of libfos_mc: contexts, argument checks, device
// scratch, the validation verdict, launch-configuration defaults and the
// C-ABI entry points declared in include/fos_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "fos_device.hpp"
#include "fos_kernels.hpp"
#include "fos_mc.h"

struct fos_ctx {
    int device = 0;
    int n_cu = 0;
    std::string err;
    // prepared problem
    int32_t n_items = 0, max_layers = 0;
    bool prepared = false;
    float4* table = nullptr;
    size_t table_bytes = 0;
    unsigned long long* cursors = nullptr;
    size_t cursors_n = 0;
    uint32_t* cur_item = nullptr;            // device, 1 word
    unsigned long long* err_dev = nullptr;   // device, 1 word
    unsigned long long* err_host = nullptr;  // pinned host, 1 word
    fos_mc_launch defaults{};
    // optics scratch
    int* cell_of = nullptr;
    size_t cell_of_bytes = 0;
    double* mie = nullptr;
    size_t mie_bytes = 0;
    double2* mie_scratch = nullptr;
    size_t mie_scratch_bytes = 0;
    unsigned int* nmax_dev = nullptr;        // device, 1 word
    unsigned long long* aux_host = nullptr;  // pinned host, 4 words
};

namespace {

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

fos_status fail(fos_ctx* c, fos_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

fos_status hip_fail(fos_ctx* c, hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory)
        return fail(c, FOS_E_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
    return fail(c, FOS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

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
    return FOS_OK;
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
    return r;
}

template <class T>
hipError_t grow(T*& p, size_t& cap, size_t need_bytes)
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
    c->defaults.block_size = 256;
    c->defaults.refill_min = 8;
    c->defaults.chunk = 4096;
    c->defaults.blocks_per_cu = 8;
    c->defaults.max_steps = 100000000ull;
    DeviceGuard g(hip_device);
    if (hipMalloc(reinterpret_cast<void**>(&c->cur_item), 256) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->err_dev), 256) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->nmax_dev), 256) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->aux_host), 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->err_host), sizeof(unsigned long long)) != hipSuccess) {
        fos_destroy(c);
        return FOS_E_OUT_OF_MEMORY;
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
        if (c->cursors) (void)hipFree(c->cursors);
        if (c->cur_item) (void)hipFree(c->cur_item);
        if (c->err_dev) (void)hipFree(c->err_dev);
        if (c->err_host) (void)hipHostFree(c->err_host);
        if (c->aux_host) (void)hipHostFree(c->aux_host);
        if (c->nmax_dev) (void)hipFree(c->nmax_dev);
        if (c->cell_of) (void)hipFree(c->cell_of);
        if (c->mie) (void)hipFree(c->mie);
        if (c->mie_scratch) (void)hipFree(c->mie_scratch);
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
    size_t cur_bytes = c->cursors_n * sizeof(unsigned long long);
    e = grow(c->cursors, cur_bytes, (size_t)std::max(p->n_items, 1) * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(c, e, "work cursors");
    c->cursors_n = cur_bytes / sizeof(unsigned long long);
    if (p->n_items > 0) {
        if ((e = fos::launch_fill_u64(c->err_dev, ~0ull, 1, st)) != hipSuccess) return hip_fail(c, e, "reset");
        fos::PackArgs a{p->n_items, p->max_layers, p->n_layers, p->mu_s, p->mu_a, p->g, p->n_layer,
                        p->thickness, p->n_upper, p->n_lower, p->k_lower, p->mu0, p->photons, c->table,
                        c->err_dev};
        if ((e = fos::launch_pack(a, st)) != hipSuccess) return hip_fail(c, e, "pack kernel");
        if ((e = hipMemcpyAsync(c->err_host, c->err_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
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
    c->prepared = true;
    return FOS_OK;
}

fos_status fos_mc_execute(fos_ctx* c, uint64_t seed, const fos_mc_launch* launch, uint64_t* tallies,
                          void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (!c->prepared) return fail(c, FOS_E_NOT_PREPARED, "no prepared problem (call fos_mc_prepare)");
    if (c->n_items == 0) return FOS_OK;
    if (!tallies) return fail(c, FOS_E_INVALID_ARG, "tallies is NULL");
    const fos_mc_launch L = merge(c->defaults, launch);
    fos_status s = check_launch(c, L);
    if (s != FOS_OK) return s;
    DeviceGuard g(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned long long* tal = reinterpret_cast<unsigned long long*>(tallies);
    hipError_t e = fos::launch_reset(tal, c->cursors, c->cur_item, c->n_items, st);
    if (e != hipSuccess) return hip_fail(c, e, "reset kernel");
    fos::WalkArgs a{};
    a.table = c->table;
    a.n_items = c->n_items;
    a.max_layers = c->max_layers;
    a.rec_f4 = fos::rec_f4(c->max_layers);
    a.cursors = c->cursors;
    a.cur_item = c->cur_item;
    a.tallies = tal;
    a.seed = seed;
    a.max_steps = (uint32_t)L.max_steps;
    a.chunk = L.chunk;
    a.refill_min = L.refill_min;
    const int grid = c->n_cu * L.blocks_per_cu;
    if ((e = fos::launch_walk(a, grid, L.block_size, st)) != hipSuccess) return hip_fail(c, e, "walk kernel");
    return FOS_OK;
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
    if ((e = grow(c->mie, c->mie_bytes, (size_t)std::max<int64_t>(P, 1) * 3 * sizeof(double))) != hipSuccess)
        return hip_fail(c, e, "optics scratch");
    fos::OpticsArgs a{};
    a.n_cells = p->n_cells;
    a.n_entries = P;
    a.lam = p->lam; a.n_m = p->n_m; a.k_m = p->k_m; a.offsets = p->offsets;
    a.n_p = p->n_p; a.k_p = p->k_p; a.r = p->r; a.f = p->f;
    a.cell_of = c->cell_of;
    a.mie = c->mie;
    a.nmax = c->nmax_dev;
    a.err = c->err_dev;
    a.out_mu_s = mu_s; a.out_mu_a = mu_a; a.out_g = g; a.out_f64 = out_f64;
    if ((e = fos::launch_fill_u64(c->err_dev, ~0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_fill_u64(reinterpret_cast<unsigned long long*>(c->nmax_dev), 0ull, 1, st)) != hipSuccess ||
        (e = fos::launch_optics_scan(a, st)) != hipSuccess)
        return hip_fail(c, e, "optics scan");
    if ((e = hipMemcpyAsync(c->err_host, c->err_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&c->aux_host[2], c->nmax_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "optics verdict");
    const unsigned long long w = *c->err_host;
    if (w != ~0ull) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "cell %llu: invalid %s", w >> 8, optics_field_name((int)(w & 0xFF)));
        return fail(c, FOS_E_INVALID_ARG, buf);
    }
    const int nn_cap = (int)(c->aux_host[2] & 0xFFFFFFFFull);
    if (nn_cap > (1 << 20)) return fail(c, FOS_E_UNSUPPORTED, "Mie series longer than 2^20 terms");
    const int block = 256;
    int grid = c->n_cu * 4;
    const int64_t need = (P + block - 1) / block;
    if (need < grid) grid = (int)std::max<int64_t>(need, 1);
    a.nn_cap = std::max(nn_cap, 1);
    const size_t nthreads = (size_t)grid * block;
    if ((e = grow(c->mie_scratch, c->mie_scratch_bytes, ((size_t)a.nn_cap + 1) * nthreads * sizeof(double2))) !=
        hipSuccess)
        return hip_fail(c, e, "Mie scratch");
    a.scratch = c->mie_scratch;
    if ((e = fos::launch_mie(a, grid, block, st)) != hipSuccess) return hip_fail(c, e, "Mie kernel");
    if ((e = fos::launch_emt(a, st)) != hipSuccess) return hip_fail(c, e, "effective-medium kernel");
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
