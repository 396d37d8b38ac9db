/*
 * fos_mc.h -- C ABI of libfos_mc: Monte Carlo photon transport through
 * particle-laden multi-layer slabs on AMD Instinct MI355X (gfx950).
 *
 * The operation follows the paper "FOS: Fast Optical Spectrum calculations
 * of nanoparticle media" (arXiv 2409.00165):
 *   - inputs per wavelength are the effective scattering coefficient mu_s,
 *     absorption coefficient mu_a and asymmetry parameter g of every layer
 *     (Methodology, Scattering properties, eqs. (13)-(20); the four-column
 *     material file of the Input section carries exactly these), layer
 *     thicknesses with "Layer 1" on top, the real matrix index of every layer
 *     and the upper/lower boundary media (Input section: air, n = 1, unless
 *     set; the Monte Carlo method accepts any lower medium, conductors
 *     included -- Methodology, Photon transport);
 *   - outputs are photon counts reflected, absorbed and transmitted per
 *     wavelength (Methodology, Photon transport: an MCML-style walk that
 *     tracks only depth and the direction cosine to the surface normal;
 *     step size from the extinction, scatter-versus-absorb from the albedo,
 *     new direction from g; Fresnel reflection at every boundary using the
 *     matrix index).
 *
 * Units: lengths in micrometres, coefficients in 1/micrometre.
 *
 * Conventions for every entry point
 *   - Pointers marked DEVICE are caller-owned device memory on the context's
 *     device; pointers marked HOST are host memory.  The library never frees
 *     or keeps caller memory beyond the call's completion on the stream.
 *   - `hip_stream` is a hipStream_t (NULL = the legacy default stream).
 *   - Status codes only; no exception crosses the ABI.  After a failure
 *     fos_last_error(ctx) describes it (valid until the next call on ctx).
 *   - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef FOS_MC_H
#define FOS_MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FOS_ABI_VERSION 5
#define FOS_MAX_LAYERS 8

/* tally slots per item, in this order, uint64 each */
#define FOS_TALLY_R_SPECULAR   0  /* reflected at the first face on entry       */
#define FOS_TALLY_R_DIFFUSE    1  /* left through the top face after entering   */
#define FOS_TALLY_ABSORBED     2  /* absorbed inside a layer                    */
#define FOS_TALLY_TRANSMITTED  3  /* entered the lower medium                   */
#define FOS_TALLY_CAPPED       4  /* stopped by the per-photon step cap         */
#define FOS_TALLY_STEPS        5  /* photon-steps taken (free-path iterations)  */
#define FOS_N_TALLY            6

typedef enum {
    FOS_OK = 0,
    FOS_E_INVALID_ARG = 1,
    FOS_E_UNSUPPORTED = 2,
    FOS_E_DEVICE = 3,
    FOS_E_OUT_OF_MEMORY = 4,
    FOS_E_INTERNAL = 5,
    FOS_E_NOT_PREPARED = 6
} fos_status;

typedef struct fos_ctx fos_ctx;

/* Library ABI version (FOS_ABI_VERSION of the build). */
int fos_abi_version(void);

/* Human-readable name of a status code (static string). */
const char* fos_status_string(fos_status s);

/* Create a context bound to HIP device `hip_device`.  The context owns all
 * internal device scratch (packed item tables, work cursors).  Fails with
 * FOS_E_DEVICE if the device is absent or not gfx950. */
fos_status fos_create(int hip_device, fos_ctx** out);

/* Release a context and its scratch; NULL-safe.  Synchronises the device
 * before freeing. */
void fos_destroy(fos_ctx* ctx);

/* Message for the last failing call on ctx ("" if none). */
const char* fos_last_error(const fos_ctx* ctx);

/* ------------------------------------------------------------------------- */
/* Monte Carlo transport                                                      */
/* ------------------------------------------------------------------------- */

/* One batch of independent items.  An item is one (design, wavelength)
 * pair: a stack of n_layers[i] layers between an upper medium of real index
 * n_upper[i] (light arrives from there at incidence cosine mu0[i]) and a
 * lower half-space of complex index n_lower[i] + i k_lower[i].  Per-layer
 * arrays are row-major [n_items][max_layers]; entries beyond n_layers[i] are
 * ignored.  All pointers are DEVICE.
 *
 * Valid values: 1 <= n_layers <= max_layers <= FOS_MAX_LAYERS; mu_s, mu_a
 * >= 0 and finite (mu_s + mu_a = 0, a clear layer, is allowed); -1 <= g <= 1;
 * n_layer >= 1; thickness > 0 and finite; n_upper >= 1; n_lower > 0;
 * k_lower >= 0; 0 < mu0 <= 1; photons >= 0 (an item with 0 photons
 * yields zero tallies). */
typedef struct {
    int32_t n_items;
    int32_t max_layers;
    const int32_t* n_layers;   /* [n_items]              */
    const float* mu_s;         /* [n_items * max_layers] */
    const float* mu_a;         /* [n_items * max_layers] */
    const float* g;            /* [n_items * max_layers] */
    const float* n_layer;      /* [n_items * max_layers] real matrix index */
    const float* thickness;    /* [n_items * max_layers] */
    const float* n_upper;      /* [n_items] */
    const float* n_lower;      /* [n_items] */
    const float* k_lower;      /* [n_items] */
    const float* mu0;          /* [n_items] */
    const uint64_t* photons;   /* [n_items] */
} fos_mc_problem;

/* Launch knobs of the persistent walk kernel; a zero field takes the
 * context's current default (set by fos_mc_set_launch or fos_mc_autotune,
 * else built-in).  Until a chunk default is set that way, a launch without a
 * chunk sizes it per problem: the largest power of two at most
 * n_items * (largest photon budget) / (4 * resident waves), within
 * [256, built-in default 2048], so that small batches still give every wave
 * several claims.  Tallies never depend on these knobs. */
typedef struct {
    int32_t block_size;     /* threads per workgroup, multiple of 64, 64..1024   */
    int32_t refill_min;     /* refill a wave when >= this many lanes idle, 1..64 */
    int32_t chunk;          /* photons a wave claims from the queue at once      */
    int32_t blocks_per_cu;  /* persistent grid = CUs * blocks_per_cu             */
    uint64_t max_steps;     /* per-photon step cap (photons beyond it -> CAPPED) */
    int32_t tail_lanes;     /* > 0: a wave with no photons left to claim and at
                               most this many in flight computes their next
                               random draws on all 64 lanes ahead of the steps
                               that use them (a build of the walk with that
                               phase); -1: the build without it; 1..64, -1     */
    int32_t regroup_lanes;  /* > 0: regrouping in the tail build of the walk.  A
                               wave with no photons left to claim and at most this
                               many in flight writes their state to a hand-off
                               list in HBM and leaves, and waves with idle lanes
                               take them over, while more than one wave per CU
                               is alive; -1: off; 1..32, -1.  Needs a context
                               hand-off list of (CUs x blocks_per_cu x waves per
                               block x regroup_lanes) records of 32 B (48 B
                               weighted) plus 4 B each, grown on first use       */
} fos_mc_launch;

/* Validate `problem` and pack it into the context's device item table
 * (per item: entry Fresnel reflectance and refracted cosine; per layer:
 * extinction, albedo, Henyey-Greenstein constants, interface index ratios).
 * Runs a validation kernel on `hip_stream` and synchronises that stream to
 * read its verdict; an invalid problem returns FOS_E_INVALID_ARG naming the
 * first offending item and field, and leaves caller memory untouched.  The
 * packed table stays in the context until the next prepare. */
fos_status fos_mc_prepare(fos_ctx* ctx, const fos_mc_problem* problem, void* hip_stream);

/* Walk every photon of the prepared problem and write the tallies.
 * `tallies` is DEVICE uint64 [n_items * FOS_N_TALLY], overwritten.  The
 * random stream of photon p of item i under `seed` is Philox4x32-10 with
 * counter (p lo, p hi, step, i) and key (seed lo, seed hi), so tallies are
 * bit-identical for every launch configuration, chunking, scheduling and
 * hand-off between waves.  Asynchronous on `hip_stream`; never synchronises,
 * and may be captured into a HIP graph.  It allocates nothing, except that a
 * launch with regroup_lanes > 0 grows the context's hand-off list the first
 * time it needs more (do one such call before capturing one).  `launch` may
 * be NULL. */
fos_status fos_mc_execute(fos_ctx* ctx, uint64_t seed, const fos_mc_launch* launch,
                          uint64_t* tallies, void* hip_stream);

/* fos_mc_prepare followed by fos_mc_execute. */
fos_status fos_mc_run(fos_ctx* ctx, const fos_mc_problem* problem, uint64_t seed,
                      const fos_mc_launch* launch, uint64_t* tallies, void* hip_stream);

/* Allocation-free fos_mc_run, for callers that cannot allocate device or
 * pinned memory at call time (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same problem, seed, launch,
 * tallies and results as fos_mc_run -- bit for bit -- but the packed item
 * table, the work queue and the validation words live in a fixed device
 * array of FOS_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library is
 * loaded, instead of the context's scratch; the context's prepared problem
 * is left as it was.  A problem needing more than that (256 B + its packed
 * table, 32 B per item plus 64 B per layer slot, rounded up to 256 B, + 8 B
 * per item + 8 B) is rejected with FOS_E_INVALID_ARG before any work is
 * enqueued: about 160,000 single-layer or 30,000 eight-layer items.  Every
 * call on one GPU uses that GPU's one array and leaves it holding its table:
 * calls that overlap on one GPU (other threads, other contexts, or another
 * stream before this call's walk has finished) race and give wrong tallies.
 * Validation synchronises `hip_stream` once, as fos_mc_prepare does; the
 * walk is then asynchronous on it.  A launch with regroup_lanes > 0 is
 * rejected (its hand-off list is a context allocation). */
#define FOS_NOALLOC_SCRATCH_BYTES (16u << 20)
fos_status fos_mc_run_noalloc(fos_ctx* ctx, const fos_mc_problem* problem, uint64_t seed,
                              const fos_mc_launch* launch, uint64_t* tallies, void* hip_stream);

/* Launch tuning for the prepared problem.  The trial launches walk a sample
 * of it: up to 2048 items chosen evenly from 16 strata of equal item count
 * by an estimate of their walk length (photon-steps per photon from the
 * layers' scattering and absorption depths and g, so the longest walks are
 * in the sample), at their own photon budgets scaled by one common factor to
 * at most `sample_photons` photons in all (0 = 2^30).  A coordinate search
 * over refill_min x chunk x block_size x blocks_per_cu x tail_lanes times
 * each candidate with HIP events on `hip_stream` (best of two after a
 * warm-up) and makes the fastest the context's default.  With a launch
 * cache set (fos_mc_autotune_cache), a problem whose class -- device
 * architecture, layer slots, and the log2 of the item count, of the mean
 * budget and of the photon-weighted mean walk estimate -- has an entry takes
 * that launch without trials, and a tuned launch is written back under its
 * class.  Tallies do not depend on the launch configuration, so tuning never
 * changes results.  Synchronises the stream; uses context-owned scratch.
 * best (HOST, may be NULL) receives the chosen configuration and best_ms
 * (HOST, may be NULL) its time on the sample. */
fos_status fos_mc_autotune(fos_ctx* ctx, uint64_t seed, uint64_t sample_photons, fos_mc_launch* best,
                           float* best_ms, void* hip_stream);

/* Launch cache of fos_mc_autotune for this context: a JSON file (created if
 * absent) of tuned launches keyed by (architecture, item class); NULL or ""
 * turns it off.  The file is read and rewritten by each tuning call. */
fos_status fos_mc_autotune_cache(fos_ctx* ctx, const char* path);

/* Hand-off counts of the last regrouping walk (regroup_lanes > 0) on this
 * context: photons handed from one wave to another (HOST, may be NULL) and
 * hand-offs whose record a taking wave did not see written within its wait
 * bound (HOST, may be NULL; each such photon is missing from the tallies, so
 * anything but 0 means those tallies are short).  Both 0 before any
 * regrouping walk.  Synchronises `hip_stream`, which must order the call
 * after that walk. */
fos_status fos_mc_handoff_counts(fos_ctx* ctx, uint64_t* handed, uint64_t* lost, void* hip_stream);

/* Capture the execute sequence of the prepared problem (tally and cursor
 * reset, persistent walk) into a HIP graph owned by the context, writing to
 * `tallies` (DEVICE uint64 [n_items * FOS_N_TALLY]) with launch `launch`
 * (NULL = defaults).  The graph reads its seed from context memory, so one
 * captured sweep is replayed with any seed.  Replaces a previous graph.
 * Uses a context-owned capture stream; `hip_stream` orders the capture after
 * the caller's prior work. */
fos_status fos_mc_graph_capture(fos_ctx* ctx, const fos_mc_launch* launch, uint64_t* tallies,
                                void* hip_stream);

/* Replay the captured sweep with `seed` on `hip_stream` (asynchronous; the
 * seed is set by a kernel, so the call itself may be captured).  Tallies are
 * bit-identical to fos_mc_execute with the same seed and prepared problem. */
fos_status fos_mc_graph_launch(fos_ctx* ctx, uint64_t seed, void* hip_stream);

/* (R, A, T) fractions from tallies: rat[3i..3i+2] = ((specular + diffuse)/N,
 * absorbed/N, transmitted/N) with N the photons of item i (the paper's
 * reflectance, absorptance and transmittance, Methodology, Photon
 * transport).  tallies DEVICE uint64 [n * FOS_N_TALLY], rat DEVICE float
 * [n * 3].  Asynchronous. */
fos_status fos_mc_fractions(fos_ctx* ctx, int32_t n, const uint64_t* tallies, float* rat, void* hip_stream);

/* Weighted-packet walk: the variance-reduction form of the walk in MCML
 * (ref. [45], which the paper's Monte Carlo follows, Methodology, Photon
 * transport).  Same problem, launch, counter-based random numbers and
 * boundaries as fos_mc_execute, but each photon is a packet of weight W:
 * it enters with W = 1 - R0 (the specular part R0 is tallied as weight, no
 * draw); at each interaction it deposits W mu_a/mu_t and always scatters; it
 * leaves through a face with its whole weight (all-or-none Fresnel decision
 * as in the analog walk); below a weight of 1e-4 it survives a roulette with
 * probability 0.1 and ten times the weight.  Estimates are unbiased;
 * R + A + T = 1 holds in expectation.  tallies DEVICE uint64
 * [n_items * FOS_N_TALLY_W]: specular R, diffuse R, A, T, and the sums of
 * squares of each photon's diffuse-R, A and T totals, all in units of 2^-36
 * of a photon's weight (integer sums: results are bit-identical for any
 * launch), then roulette ends, capped photons, photon-steps and photons.  An
 * item must not exceed 2^27 photons.  Asynchronous, allocates nothing. */
#define FOS_N_TALLY_W 11
fos_status fos_mc_execute_weighted(fos_ctx* ctx, uint64_t seed, const fos_mc_launch* launch, uint64_t* tallies,
                                   void* hip_stream);

/* fos_mc_prepare + fos_mc_execute_weighted. */
fos_status fos_mc_run_weighted(fos_ctx* ctx, const fos_mc_problem* problem, uint64_t seed,
                               const fos_mc_launch* launch, uint64_t* tallies, void* hip_stream);

/* (R, A, T) means from weighted tallies, rat DEVICE float [n * 3], and the
 * standard errors of those estimates from the per-photon sums of squares, se
 * DEVICE float [n * 3] (may be NULL).  Asynchronous. */
fos_status fos_mc_weighted_fractions(fos_ctx* ctx, int32_t n, const uint64_t* tallies, float* rat, float* se,
                                     void* hip_stream);

/* Number of items of the prepared problem (0 if none). */
int32_t fos_mc_prepared_items(const fos_ctx* ctx);

/* Current launch defaults of the context (HOST out). */
fos_status fos_mc_get_launch(const fos_ctx* ctx, fos_mc_launch* out);

/* Set the context's launch defaults; fields equal to 0 keep their value. */
fos_status fos_mc_set_launch(fos_ctx* ctx, const fos_mc_launch* launch);

/* ------------------------------------------------------------------------- */
/* Effective optics (Methodology, Scattering properties)                      */
/* ------------------------------------------------------------------------- */

/* Layer cells and their particle populations.  A cell is one (layer,
 * wavelength) pair: vacuum wavelength lam, matrix index n_m + i k_m, and the
 * particle entries offsets[c] .. offsets[c+1]-1 of the CSR arrays (one entry
 * per particle size of each species: index n_p + i k_p, radius r, volume
 * fraction f as a fraction, not a percentage).  All pointers DEVICE, double.
 * Valid values: lam > 0, n_m > 0, k_m >= 0, n_p > 0, k_p >= 0, r > 0,
 * f >= 0, offsets non-decreasing from offsets[0] = 0. */
typedef struct {
    int32_t n_cells;
    const double* lam;        /* [n_cells] micrometres */
    const double* n_m;        /* [n_cells] */
    const double* k_m;        /* [n_cells] */
    const int64_t* offsets;   /* [n_cells + 1] */
    const double* n_p;        /* [offsets[n_cells]] */
    const double* k_p;
    const double* r;          /* micrometres */
    const double* f;
    /* optional per-entry arrays (NULL = none), Scattering properties section
     * and supplementary eqs. (S1)-(S9): */
    const double* sd;         /* standard deviation of the diameter 2r (micrometres): the entry becomes 101
                                 diameters evenly over 2r - 3 sd .. 2r + 3 sd with Gaussian weights,
                                 renormalised over the positive ones, as volume fractions f w; 0 = one size */
    const double* r_core;     /* core radius (micrometres), 0 <= r_core <= r: > 0 makes the entry a coated
                                 sphere, core n_core + i k_core inside a shell n_p + i k_p out to r (cross
                                 sections and eqs. (13)-(16) use r); not combined with sd > 0 */
    const double* n_core;
    const double* k_core;
} fos_optics_problem;

/* Effective mu_s, mu_a (1/micrometre) and g of every cell: Lorenz-Mie
 * coefficients of each sphere in the absorbing host, eqs. (1)-(5), in the
 * logarithmic-derivative form (the printed closed forms (6)-(9) are not
 * used); efficiencies eqs. (10)-(12) with alpha = 4 pi r k_m / lambda;
 * asymmetry eq. (15); the volume-fraction sums eqs. (13), (14), (16);
 * negative sums set to zero; the dependent-scattering factor eqs. (17)-(19)
 * when the cell's total volume fraction exceeds 0.08; matrix absorption
 * eq. (20).  Outputs (DEVICE, any may be NULL): mu_s, mu_a, g float
 * [n_cells] (cell c of a stack of max_layers layers laid out item-major is
 * exactly the per-layer problem array element of fos_mc_problem), and
 * out_f64 double [n_cells * 3] = (mu_s, mu_a, g).  Validates on the device
 * and synchronises `hip_stream` for the verdict and the series length;
 * FOS_E_INVALID_ARG names the first bad cell. */
fos_status fos_optics_run(fos_ctx* ctx, const fos_optics_problem* problem, float* mu_s, float* mu_a,
                          float* g, double* out_f64, void* hip_stream);

/* Log-normal particle populations on a shared size grid: the same optics
 * as fos_optics_run for designs whose particles are one species in log-normal
 * sizes binned as the workloads bin them (n_bins equal bins of width dlnr in
 * ln r, centred on ln r_med, volume weights w[b]), with the median radius on
 * the grid r_med = r0 exp(k dlnr).  Every bin of every design then lies on the
 * radius grid r_j = r0 exp((j - (n_bins - 1)/2) dlnr), j = 0 .. n_rmed +
 * n_bins - 2, so the Lorenz-Mie efficiencies are evaluated once per (species,
 * matrix, wavelength, r_j) and eqs. (13)-(16) become per-(median, wavelength)
 * bin sums times the design's volume fraction f (f_i = f w[b]); the clamp,
 * eqs. (17)-(19) and (20) follow per design exactly as in fos_optics_run.
 * HOST arrays: lambda, n_p, k_p, n_m, w.  DEVICE arrays: species, matrix,
 * rmed, f.  Outputs DEVICE float [n_designs * n_lambda], design-major: the
 * per-layer arrays of single-layer items (item = design * n_lambda + l).
 * Valid: lambda > 0, n_p > 0, k_p >= 0, n_m > 0, k_m >= 0, r0 > 0,
 * dlnr > 0, n_bins >= 1, w >= 0, indices in range, 0 <= f <= 1.
 * Synchronises `hip_stream` (validation verdict); FOS_E_INVALID_ARG names the
 * first bad design or table field. */
typedef struct {
    int32_t n_lambda;
    const double* lambda;    /* HOST [n_lambda] micrometres */
    int32_t n_species;
    const double* n_p;       /* HOST [n_species * n_lambda] particle index, real part */
    const double* k_p;       /* HOST [n_species * n_lambda] particle index, imaginary part */
    int32_t n_matrix;
    const double* n_m;       /* HOST [n_matrix] matrix index, real part */
    double k_m;              /* matrix index, imaginary part (all matrices) */
    double r0;               /* smallest median radius, micrometres */
    double dlnr;             /* bin width and median-grid spacing in ln r */
    int32_t n_rmed;          /* median radii on the grid */
    int32_t n_bins;
    const double* w;         /* HOST [n_bins] volume weights of the bins */
    int32_t n_designs;
    const int32_t* species;  /* DEVICE [n_designs] */
    const int32_t* matrix;   /* DEVICE [n_designs] index into n_m */
    const int32_t* rmed;     /* DEVICE [n_designs] median-radius index */
    const double* f;         /* DEVICE [n_designs] total particle volume fraction */
} fos_lognormal_problem;

fos_status fos_optics_lognormal(fos_ctx* ctx, const fos_lognormal_problem* problem, float* mu_s, float* mu_a,
                                float* g, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Surrogate network (the paper's neural-network alternative to Monte Carlo,  */
/* Methodology, Photon transport; trained here on this library's own walk)    */
/* ------------------------------------------------------------------------- */

#define FOS_SUR_FEATURES 8
#define FOS_SUR_MEMBERS 4
#define FOS_SUR_PARAMS 200451    /* fp32 parameters per ensemble member */

/* Training options.  The network of every member is 8 standardised inputs ->
 * 4 hidden layers of 256 with tanh-form GELU -> 3 logits -> softmax (R, A,
 * T); bf16 operands on the matrix cores with fp32 accumulation and fp32
 * master weights; loss = cross-entropy against the Monte Carlo fractions;
 * Adam (0.9, 0.999, 1e-8) with a cosine learning-rate decay. */
typedef struct {
    int32_t epochs;        /* passes over the data, >= 1 */
    int32_t batch;         /* rows per step and member, a multiple of 64 */
    float lr;              /* peak learning rate */
    float lr_min;          /* final learning rate of the cosine decay */
    uint64_t seed;         /* He initialisation and per-member shuffles */
    int32_t resume;        /* 1: continue from the context's model and optimiser state */
    float* loss_history;   /* DEVICE [epochs * 4] mean loss per epoch and member, or NULL */
} fos_train_opts;

/* The 8 raw surrogate features of every item of a transport problem
 * (DEVICE arrays as in fos_mc_problem, layer 0 of each item):
 * log10(mu_s t + 1e-6), log10(mu_a t + 1e-6), -log10(1 - g + 1e-3), n_layer,
 * n_lower, log10(k_lower + 1e-4), mu0, layer index (0).  x DEVICE float [n_items * 8];
 * eligible DEVICE uint8 [n_items] (may be NULL) = 1 for single-layer items
 * lit from an upper medium of index 1 -- the only items the surrogate serves
 * (the paper's network likewise needs air or vacuum boundaries).
 * Asynchronous. */
fos_status fos_sur_features(fos_ctx* ctx, const fos_mc_problem* problem, float* x, uint8_t* eligible,
                            void* hip_stream);

/* Train the 4-member ensemble on n rows: x DEVICE float [n * 8] raw
 * features, y DEVICE float [n * 3] Monte Carlo (R, A, T) fractions.  Unless
 * resuming, computes the feature mean/std (standardisation) and min/max (the
 * validity box of fos_sur_predict), initialises the members from `seed` and
 * zeroes the optimiser.  Each member sees its own shuffle of the rows every
 * epoch.  Enqueued on `hip_stream` (the call returns before the work ends);
 * n must be >= batch. */
fos_status fos_sur_train(fos_ctx* ctx, const float* x, const float* y, int64_t n, const fos_train_opts* opts,
                         void* hip_stream);

/* Ensemble prediction and gate for n rows of raw features x (DEVICE float
 * [n * 8]): rat (DEVICE float [n * 3]) = member mean of (R, A, T); spread
 * (DEVICE float [n]) = max over channels of (max - min across members);
 * in_domain (DEVICE uint8 [n]) = 1 if every feature lies inside the training
 * box and eligible[i] (DEVICE uint8, may be NULL) is set; members (DEVICE
 * float [4 * n * 3], may be NULL) = each member's prediction.  Any output may
 * be NULL.  Asynchronous. */
fos_status fos_sur_predict(fos_ctx* ctx, const float* x, const uint8_t* eligible, int64_t n, float* rat,
                           float* spread, uint8_t* in_domain, float* members, void* hip_stream);

/* Test hook: gradient of the mean loss over the first n rows (n a multiple
 * of 64, no shuffle) for every member, without updating: grads DEVICE float
 * [4 * FOS_SUR_PARAMS] in the flat layout of fos_sur_save (W1 [8][256], b1,
 * W2 [256][256], b2, W3, b3, W4, b4, W5 [256][3], b5), loss DEVICE float [4]. */
fos_status fos_sur_grad(fos_ctx* ctx, const float* x, const float* y, int64_t n, float* grads, float* loss,
                        void* hip_stream);

/* Serialise the model (and optimiser state) to HOST memory.  With blob NULL
 * only *bytes is set to the size needed.  Layout (little endian): 8-byte
 * magic "FOSSUR01", uint32 members, features, hidden, params, has_opt,
 * adam_step, then float32 stats [32] (mean, 1/std, min, max of the 8
 * features), params [members * params], and if has_opt Adam m and v. */
fos_status fos_sur_save(const fos_ctx* ctx, void* blob, size_t* bytes);

/* Load a model written by fos_sur_save (HOST blob; copies). */
fos_status fos_sur_load(fos_ctx* ctx, const void* blob, size_t bytes);

/* Surrogate design sweep with Monte Carlo fallback.  For every item of
 * `problem` (DEVICE arrays as for fos_mc_run): features, ensemble prediction
 * and gate (fos_sur_features, fos_sur_predict); items that are ineligible,
 * outside the training box or whose ensemble spread exceeds `spread_max` are
 * compacted and walked by the Monte Carlo path with `fallback_photons`
 * photons each under `seed` (stream id = position in the compacted list),
 * and their fractions replace the prediction.  Outputs (DEVICE): rat float
 * [n * 3] = (R, A, T); spread float [n] (may be NULL); used_mc uint8 [n].
 * *n_fallback (HOST, may be NULL) = number of Monte Carlo items.  Replaces
 * the context's prepared transport problem; synchronises `hip_stream` to
 * size the fallback batch. */
fos_status fos_sweep_run(fos_ctx* ctx, const fos_mc_problem* problem, float spread_max, uint64_t fallback_photons,
                         uint64_t seed, float* rat, float* spread, uint8_t* used_mc, int64_t* n_fallback,
                         void* hip_stream);

/* Spectral reductions of a sweep (the paper's solar-weighted integral,
 * eq. (21), and band emittance): for each design d of `designs` rows of
 * `lambdas` wavelengths, out[2d] = sum_l w_r[l] R[d][l] and out[2d+1] =
 * sum_l w_e[l] A[d][l] (by Kirchhoff's law the absorptance is the
 * emittance).  rat DEVICE float [designs * lambdas * 3]; weights DEVICE float
 * [lambdas] (normalised quadrature weights); out DEVICE float [2 designs]. */
fos_status fos_spectral_reduce(fos_ctx* ctx, int32_t designs, int32_t lambdas, const float* rat, const float* w_r,
                               const float* w_e, float* out, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Output stage                                                               */
/* ------------------------------------------------------------------------- */

/* What a finished spectrum turns into (Output section and Results):
 *   - the solar totals of eq. (21): R_s = int R G dlambda / int G dlambda
 *     over the simulated range, and likewise A_s and T_s, where G is the
 *     spectral solar irradiation.  As in the paper they exist only when a
 *     solar spectrum is given and the grid covers at least 0.28 - 2.5 um;
 *   - the emittance of a band (e.g. the 8 - 13 um sky window): by Kirchhoff's
 *     law the absorptance, weighted by a blackbody spectrum at a given
 *     temperature over the grid points inside the band (at least two);
 *   - the colour of the reflectance spectrum, which the paper computes but
 *     does not define.  Here: CIE 1931 XYZ under an illuminant (the
 *     colour-matching functions from the multi-lobe analytic fit of Wyman,
 *     Sloan and Shirley, JCGT 2013), scaled so that a perfect reflector has
 *     Y = 1; CIE 1976 L*a*b* against the illuminant's white; and sRGB
 *     (IEC 61966-2-1) after a Bradford adaptation of that white to D65,
 *     linear values clipped to [0, 1] before encoding.  The grid must cover
 *     0.38 - 0.78 um.
 * Coverage and band membership are decided on the single-precision grid
 * values.  Spectra are linear between their samples and zero outside them
 * (the paper interpolates input files linearly onto the simulated grid);
 * integrals are trapezoid sums over the grid. */

/* A sampled spectrum: value[j] at um[j] micrometres.  HOST arrays, 2 <= n <=
 * 2^20, um finite, positive and strictly increasing, value finite and >= 0.
 * The units of value do not matter (only ratios of integrals are used). */
typedef struct {
    int32_t n;
    const float* um;
    const float* value;
} fos_spectrum;

/* What to integrate.  solar: G of eq. (21), or NULL (no solar totals).
 * illuminant: the light the colour is seen under, or NULL (equal energy).
 * band_temperature_k > 0 asks for the band emittance over [band_lo_um,
 * band_hi_um] (finite, 0 < lo < hi); <= 0 leaves it out. */
typedef struct {
    const fos_spectrum* solar;
    const fos_spectrum* illuminant;
    float band_lo_um;
    float band_hi_um;
    float band_temperature_k;
} fos_output_spec;

#define FOS_OUTPUT_SOLAR  1   /* solar totals available           */
#define FOS_OUTPUT_BAND   2   /* band emittance available         */
#define FOS_OUTPUT_COLOUR 4   /* colour available                 */

/* Prepare the output stage for a wavelength grid: lambda_um HOST [lambdas]
 * (1 <= lambdas <= 2^20; finite, positive, strictly increasing), spec HOST
 * (NULL: no solar totals, equal-energy illuminant, no band).  The context
 * keeps five rows of quadrature weights computed on the device from the grid
 * and the spectra, and the colour white point and matrix.  *available (HOST,
 * may be NULL) receives the FOS_OUTPUT_* bits the grid allows.  The host
 * arrays are copied before the call returns (it synchronises `hip_stream`).
 * Replaces any earlier preparation; a failed call leaves the stage
 * unprepared.  A run still in flight on another stream must finish first. */
fos_status fos_output_prepare(fos_ctx* ctx, int32_t lambdas, const float* lambda_um, const fos_output_spec* spec,
                              int32_t* available, void* hip_stream);

/* Run the prepared stage on `designs` spectra: rat DEVICE float
 * [designs][lambdas][3] (R, A, T per wavelength of the prepared grid;
 * `lambdas` must equal the prepared grid's size, else FOS_E_INVALID_ARG).
 * totals DEVICE float [designs][4] = (R_s, A_s, T_s, band emittance);
 * colour DEVICE float [designs][9] = (X, Y, Z, L*, a*, b*, sRGB r, g, b), or
 * NULL.  Outputs the preparation does not allow are NaN, as are solar totals
 * when the solar spectrum has no power on the grid.  Asynchronous on
 * `hip_stream`; FOS_E_NOT_PREPARED without a successful fos_output_prepare. */
fos_status fos_output_run(fos_ctx* ctx, int32_t designs, int32_t lambdas, const float* rat, float* totals,
                          float* colour, void* hip_stream);

/* The prepared stage's weights, for inspection: weights DEVICE float
 * [5][lambdas] (rows: solar, band, x, y, z; each a normalised quadrature
 * rule, zero when that output is not available), params DEVICE float [12]
 * (white X, Y, Z, then the 3 x 3 row-major matrix from XYZ to linear sRGB),
 * either may be NULL; *available HOST (may be NULL).  Asynchronous copies on
 * `hip_stream`. */
fos_status fos_output_weights(fos_ctx* ctx, float* weights, float* params, int32_t* available, void* hip_stream);

/* Measurement hook: one launch of a kernel that issues one instruction form
 * of the walk back to back on the walk's launch shape (CUs x 8 workgroups of
 * 256 threads, 8 waves per SIMD), each thread running independent chains so
 * that issue, not latency, sets the time: kind FOS_ISSUE_FMA (v_fma_f32),
 * FOS_ISSUE_FMAC (v_fmac_f32, the accumulating encoding), FOS_ISSUE_MUL
 * (v_mul_f32), FOS_ISSUE_RCP, _SQRT, _LOG, _COS (the step's transcendental
 * forms) or FOS_ISSUE_PHILOX (whole Philox4x32-10 blocks, the walk's
 * generator: 20 32x32->64 products and 20 three-input xors each).
 * `iters` iterations per thread; sink DEVICE float [fos_issue_threads(ctx)]
 * receives each thread's result; *ops (HOST) = instructions per lane summed
 * over all lanes (Philox: blocks).  Asynchronous on `hip_stream`; time it with
 * events on that stream. */
#define FOS_ISSUE_FMA 0
#define FOS_ISSUE_RCP 1
#define FOS_ISSUE_SQRT 2
#define FOS_ISSUE_LOG 3
#define FOS_ISSUE_COS 4
#define FOS_ISSUE_PHILOX 5
#define FOS_ISSUE_FMAC 6
#define FOS_ISSUE_MUL 7
int64_t fos_issue_threads(const fos_ctx* ctx);
fos_status fos_issue_run(fos_ctx* ctx, int32_t kind, int32_t iters, float* sink, uint64_t* ops, void* hip_stream);

/* Raw Philox4x32-10 words for testing the generator: out[4*j + w] =
 * word w of counter (p lo, p hi, step, stream) with p = photon[j],
 * key (seed lo, seed hi).  photon, step, stream DEVICE [n]; out DEVICE
 * [4n].  Asynchronous on hip_stream. */
fos_status fos_philox_words(fos_ctx* ctx, int32_t n, const uint64_t* photon, const uint32_t* step,
                            const uint32_t* stream, uint64_t seed, uint32_t* out, void* hip_stream);

/* Fresnel reflectance exactly as the walk evaluates it, for testing:
 * out[j] = unpolarised reflectance from real index ni[j] into nt[j] +
 * i kt[j] at incidence cosine c[j] (Methodology, Photon transport: Fresnel
 * at the boundaries with the matrix index; any lower medium, conductors
 * included).  All arrays DEVICE [n]. */
fos_status fos_eval_fresnel(fos_ctx* ctx, int32_t n, const float* c, const float* ni, const float* nt,
                            const float* kt, float* out, void* hip_stream);

/* Henyey-Greenstein polar cosine exactly as the walk samples it, for
 * testing: out[j] = cos theta drawn with asymmetry g[j] from the uniform
 * u01[j] in [0,1) (the new direction angle from g, Methodology, Photon
 * transport).  All arrays DEVICE [n]. */
fos_status fos_eval_hg(fos_ctx* ctx, int32_t n, const float* g, const float* u01, float* out,
                       void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FOS_MC_H */
