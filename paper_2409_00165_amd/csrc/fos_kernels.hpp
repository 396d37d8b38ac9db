// fos_kernels.hpp -- kernel argument blocks and launchers shared by the
// kernels and the host runtime of libfos_mc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fos {

enum ErrCode : int {
    kErrNLayers = 1,
    kErrMuS = 2,
    kErrMuA = 3,
    kErrG = 4,
    kErrNLayer = 5,
    kErrThickness = 6,
    kErrNUpper = 7,
    kErrNLower = 8,
    kErrKLower = 9,
    kErrMu0 = 10,
};

struct PackArgs {
    int n_items, max_layers;
    const int32_t* n_layers;
    const float *mu_s, *mu_a, *g, *n_layer, *thickness;
    const float *n_upper, *n_lower, *k_lower, *mu0;
    const uint64_t* photons;
    float4* table;
    unsigned long long* err;
    unsigned long long* max_photons;   // largest photon budget of the batch
};

struct WalkArgs {
    const float4* table;
    int n_items, max_layers, rec_f4;
    const unsigned long long* chunk_prefix;   // [n_items + 1] chunks before each item
    unsigned long long* chunk_counter;        // next global chunk to hand out
    unsigned long long* tallies;
    uint64_t seed;
    const uint64_t* seed_ptr;     // if non-null the seed is read here (graph replays)
    uint64_t photon_cap;          // if non-zero, at most this many photons per item
    uint32_t max_steps;
    int chunk;
    int refill_min;
    int tail_lanes;               // > 0: the build of the walk with the tail phase; a wave with no
                                  // chunk left and at most this many photons in flight prepares
                                  // their draws on all its lanes (0 = the build without it)
    // regrouping (the tail build's drain phase): a wave with no chunk left and
    // at most regroup_lanes photons in flight hands them off through the list
    // below while more than regroup_min_waves waves are alive (0 = off)
    int regroup_lanes;
    int regroup_min_waves;
    // the hand-off list, one allocation: [4] control words (reserved, taken,
    // waves alive, timed-out takes), padded to 256 B; [hand_cap] ready flags,
    // padded to 256 B; [hand_cap][2 or 3] float4 records
    unsigned char* hand;
    uint32_t hand_cap;            // records: waves of the launch x regroup_lanes
};

// byte offsets of the parts of the hand-off list
__host__ __device__ inline size_t hand_flags_offset() { return 256; }
__host__ __device__ inline size_t hand_records_offset(uint64_t cap) { return 256 + ((cap * 4 + 255) / 256) * 256; }
__host__ __device__ inline size_t hand_bytes(uint64_t cap, bool weighted)
{
    return hand_records_offset(cap) + cap * (weighted ? 3 : 2) * 16;
}

enum OptErrCode : int {
    kOptErrLambda = 1,
    kOptErrNm = 2,
    kOptErrKm = 3,
    kOptErrOffsets = 4,
    kOptErrNp = 5,
    kOptErrKp = 6,
    kOptErrRadius = 7,
    kOptErrFraction = 8,
    kOptErrSpread = 9,
    kOptErrCore = 10,
    kOptErrSpreadCore = 11,
};
// optics_scan flags: some entry has a diameter spread / a core
constexpr unsigned int kOptHasSpread = 1u, kOptHasCore = 2u;
constexpr int kSpreadSizes = 101;   // sizes of a Gaussian diameter spread

struct OpticsArgs {
    int n_cells;
    int64_t n_entries;
    const double *lam, *n_m, *k_m;
    const int64_t* offsets;
    const double *n_p, *k_p, *r, *f;
    const double *sd, *r_core, *n_core, *k_core;   // optional per entry (null = none)
    int* cell_of;                 // [n_entries]
    double* mie;                  // [n_entries * units * 3]: q_ext, q_sca, g per size unit
    int units;                    // size units per entry: 1, or kSpreadSizes when any entry has a spread
    int d_arrays;                 // logarithmic-derivative arrays per thread in scratch: 1, or 3 with cores
    unsigned int* flags;          // kOptHas* (optics_scan)
    double2* scratch;             // [(nn_cap + 1) * mie threads]
    const unsigned int* order;    // size units by series length (null = unit order)
    unsigned long long* queue;    // next 64-unit claim of mie_entries to hand out (zeroed before it)
    unsigned int* nmax;           // largest series length + 1
    int nn_cap;
    unsigned long long* err;
    float *out_mu_s, *out_mu_a, *out_g;
    double* out_f64;              // [n_cells * 3] or NULL
};

// log-normal populations on a shared radius grid (fos_optics_lognormal)
enum LnErrCode : int { kLnErrSpecies = 1, kLnErrMatrix = 2, kLnErrRmed = 3, kLnErrFraction = 4 };

struct LognormalArgs {
    int n_lambda, n_species, n_matrix, n_rmed, n_bins, n_radii;
    const double* mie;      // [(species * n_matrix + matrix) * n_lambda + l][n_radii][3] efficiencies
    const double* radii;    // [n_radii]
    const double* w;        // [n_bins]
    const double* lam;      // [n_lambda]
    double k_m;
    double* table;          // [(species * n_matrix + matrix) * n_lambda + l][n_rmed][3] bin sums
    int n_designs;
    const int32_t *species, *matrix, *rmed;
    const double* f;
    unsigned long long* err;
    float *out_mu_s, *out_mu_a, *out_g;
};

hipError_t launch_lognormal_check(const LognormalArgs& a, hipStream_t st);
hipError_t launch_lognormal_table(const LognormalArgs& a, hipStream_t st);
hipError_t launch_lognormal_cells(const LognormalArgs& a, hipStream_t st);

hipError_t launch_optics_scan(const OpticsArgs& a, hipStream_t st);
hipError_t launch_mie(const OpticsArgs& a, int grid, int block, hipStream_t st);
// Size units sorted by series length, so that the lanes of a wave run
// series of similar length; buf holds mie_order_bytes(n_units) bytes and
// starts with the order (n_units words).  Needs a.cell_of (optics_scan).
size_t mie_order_bytes(int64_t n_units);
hipError_t launch_mie_order(const OpticsArgs& a, int64_t n_units, void* buf, hipStream_t st);
hipError_t launch_emt(const OpticsArgs& a, hipStream_t st);

// launch tuner (tune_kernels.hip): estimated photon-steps per photon of every
// item, and a rescaled sample of item records in a table of its own
hipError_t launch_item_cost(const float4* table, int rf, int n, float* cost, uint64_t* photons, hipStream_t st);
hipError_t launch_gather_records(const float4* table, int rf, const int32_t* idx, const uint64_t* photons, int m,
                                 float4* out, hipStream_t st);

// instruction-throughput kernels (issue_kernels.hip)
enum IssueKind : int {
    kIssueFma = 0, kIssueRcp = 1, kIssueSqrt = 2, kIssueLog = 3, kIssueCos = 4, kIssuePhilox = 5, kIssueFmac = 6,
    kIssueMul = 7
};
int issue_ops_per_iteration(int kind);
hipError_t launch_issue(int kind, int iters, int grid, int block, float* sink, hipStream_t st);

hipError_t launch_pack(const PackArgs& a, hipStream_t st);
hipError_t launch_reset(unsigned long long* tallies, unsigned long long* counter, int n_items, int nt,
                        hipStream_t st);
hipError_t launch_chunk_scan(const float4* table, int rec_f4, int n_items, int chunk, uint64_t photon_cap,
                             unsigned long long* prefix, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t st);
hipError_t launch_walk(const WalkArgs& a, int grid, int block, hipStream_t st, bool weighted = false);
// clears the hand-off list of a regrouping walk (nothing when regroup_lanes <= 0)
hipError_t launch_reset_handoff(const WalkArgs& a, hipStream_t st);
hipError_t launch_fractions(int n, const unsigned long long* tallies, float* rat, hipStream_t st);
hipError_t launch_weighted_fractions(int n, const unsigned long long* tallies, float* rat, float* se, hipStream_t st);
size_t walk_lds_bytes(int block_size, int max_layers, bool weighted = false, bool tail = false);
hipError_t launch_philox_words(int n, const uint64_t* photon, const uint32_t* step, const uint32_t* stream,
                               uint64_t seed, uint32_t* out, hipStream_t st);
hipError_t launch_eval_fresnel(int n, const float* c, const float* ni, const float* nt, const float* kt,
                               float* out, hipStream_t st);
hipError_t launch_eval_hg(int n, const float* g, const float* u01, float* out, hipStream_t st);

}  // namespace fos
