/*
 * fos_oracle.c -- plain, slow, FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP library) never
 * links, loads or calls it, and the two share no source.
 *
 * Contents (paper: "FOS: Fast Optical Spectrum calculations of nanoparticle
 * media", arXiv 2409.00165):
 *   - Philox4x32-10 counter-based generator, from its published definition
 *     (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers: as easy as
 *     1, 2, 3").
 *   - Unpolarised Fresnel reflectance for a real incident index and a complex
 *     transmitted index (Methodology, Photon transport; boundary media in the
 *     Input section).
 *   - Henyey-Greenstein cosine sampling, textbook inversion (the sampler used
 *     by MCML, ref. [45]).
 *   - The analog photon walk through a multi-layer slab tracking only depth z
 *     and the direction cosine to the z axis (Methodology, Photon transport),
 *     and its weighted-packet form with Russian roulette (MCML, ref. [45]).
 *   - Lorenz-Mie coefficients of a sphere in an absorbing host, eqs. (1)-(5),
 *     evaluated with the Bohren-Huffman logarithmic-derivative recursion
 *     instead of the garbled closed forms (6)-(9); cross sections eqs.
 *     (10)-(12); asymmetry eq. (15); effective medium eqs. (13), (14), (16);
 *     clamp, dependent-scattering correction eqs. (17)-(19) and matrix
 *     absorption eq. (20); coated (core-shell) spheres by supplementary eqs.
 *     (S1)-(S9) and the 101-size Gaussian diameter spread of the
 *     Scattering-properties section.
 *
 * Everything is double precision.  Complex arithmetic uses C99 <complex.h>.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LAYERS 8

/* ------------------------------------------------------------------------- */
/* Philox4x32-10                                                              */
/* ------------------------------------------------------------------------- */
/* One round: two 32x32->64 products of counter words 0 and 2 with the
 * multipliers, the high halves xor-ed with the other counter words and the
 * key, the low halves passed through; the key is bumped by the Weyl constants
 * between rounds.  Ten rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = M0 * (uint64_t)c0;
        uint64_t p1 = M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on [0,1) with 24 random bits: (x >> 8) * 2^-24.  The free path uses
 * 1 - U, which lies in (0,1]. */
static inline double u24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* The draw block of photon p, step k, stream (item) s:
 * counter = (p lo, p hi, k, s), key = (seed lo, seed hi). */
static inline void draw_block(uint64_t p, uint32_t k, uint32_t s, uint64_t seed, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), k, s};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = u24(o[i]);
}

/* exposed for the generator tests */
void orc_uniforms(uint64_t p, uint32_t k, uint32_t s, uint64_t seed, double u[4])
{
    draw_block(p, k, s, seed, u);
}

/* ------------------------------------------------------------------------- */
/* Fresnel                                                                    */
/* ------------------------------------------------------------------------- */
/* Unpolarised reflectance R = (|r_s|^2 + |r_p|^2)/2 for light going from a
 * medium of real index ni into a medium of index nt + i kt, at incidence
 * cosine ci in [0,1].  With N = nt + i kt and q = N cos(theta_t) =
 * sqrt(N^2 - ni^2 sin^2(theta_i)) (principal root, Im q >= 0):
 *   r_s = (ni ci - q) / (ni ci + q),   r_p = (N^2 ci - ni q) / (N^2 ci + ni q).
 * A real medium beyond the critical angle gives q purely imaginary and
 * R = 1 (total internal reflection). */
double orc_fresnel(double ci, double ni, double nt, double kt)
{
    if (kt == 0.0 && nt == ni) return 0.0;
    double complex N = nt + I * kt;
    double complex N2 = N * N;
    double s2 = 1.0 - ci * ci;
    if (s2 < 0.0) s2 = 0.0;
    if (kt == 0.0 && ni * ni * s2 >= nt * nt) return 1.0;   /* total internal reflection */
    double complex q = csqrt(N2 - ni * ni * s2);
    if (cimag(q) < 0.0) q = -q;
    double complex rs = (ni * ci - q) / (ni * ci + q);
    double complex rp = (N2 * ci - ni * q) / (N2 * ci + ni * q);
    double R = 0.5 * (creal(rs * conj(rs)) + creal(rp * conj(rp)));
    if (R > 1.0) R = 1.0;
    return R;
}

/* ------------------------------------------------------------------------- */
/* Henyey-Greenstein                                                          */
/* ------------------------------------------------------------------------- */
/* Inverse-CDF sample of the HG phase function with asymmetry g from a
 * uniform u in [0,1):  cos = (1 + g^2 - ((1 - g^2)/(1 - g + 2 g u))^2) / (2 g),
 * isotropic cos = 2u - 1 at g = 0; a delta at cos = g when |g| = 1.  Below
 * |g| = 1e-9 the isotropic form is used (the difference is O(g)). */
double orc_hg_cos(double g, double u)
{
    double c;
    if (fabs(g) < 1e-9) {
        c = 2.0 * u - 1.0;
    } else if (fabs(g) >= 1.0) {
        c = g > 0 ? 1.0 : -1.0;
    } else {
        double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        c = (1.0 + g * g - t * t) / (2.0 * g);
    }
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return c;
}

/* ------------------------------------------------------------------------- */
/* Photon walk                                                                */
/* ------------------------------------------------------------------------- */
/* Tally layout (uint64 per item): 0 specular reflection, 1 diffuse
 * reflection, 2 absorbed, 3 transmitted, 4 terminated by the step cap,
 * 5 photon-steps. */
enum { T_RSPEC = 0, T_RDIFF, T_ABS, T_TRANS, T_CAP, T_STEPS, T_N };

typedef struct {
    int L;
    double mus[ORC_MAX_LAYERS], mua[ORC_MAX_LAYERS], g[ORC_MAX_LAYERS];
    double n[ORC_MAX_LAYERS], ztop[ORC_MAX_LAYERS], zbot[ORC_MAX_LAYERS];
    double n_up, n_lo, k_lo, mu0;
    uint32_t stream;
} orc_stack;

/* Walk photons [p_begin, p_end) of one stack; accumulate into tal[T_N].
 *
 * Depth z grows into the stack, z = 0 is the top face.  One draw block per
 * event: block 0 decides specular reflection at entry; block k >= 1 is the
 * k-th photon-step.  A step: (re)draw the optical path s = -ln(1-U0) when
 * none is left; if the path reaches the layer boundary along the direction,
 * move there, spend that optical depth and meet the interface (Fresnel with
 * U1: reflect, refract into the neighbour layer, or leave through the top
 * (diffuse reflection) or bottom (transmission)); otherwise move by s/mu_t,
 * and interact: scatter with probability mu_s/mu_t (U1), drawing the HG
 * polar cosine from U2 and the azimuth 2 pi U3, else absorb. */
static void walk_range(const orc_stack* S, uint64_t seed, uint64_t p_begin, uint64_t p_end,
                       uint64_t max_steps, uint64_t tal[T_N])
{
    double u[4];
    for (uint64_t p = p_begin; p < p_end; ++p) {
        /* launch: specular reflection at the top face */
        draw_block(p, 0u, S->stream, seed, u);
        double R0 = orc_fresnel(S->mu0, S->n_up, S->n[0], 0.0);
        if (u[1] < R0) { tal[T_RSPEC]++; continue; }
        double r = S->n_up / S->n[0];
        double uz = sqrt(1.0 - r * r * (1.0 - S->mu0 * S->mu0));
        int l = 0;
        double z = 0.0, s = 0.0;
        uint64_t k = 0;
        for (;;) {
            ++k;
            if (k > max_steps) { tal[T_CAP]++; k = max_steps; break; }
            draw_block(p, (uint32_t)k, S->stream, seed, u);
            if (s == 0.0) s = -log(1.0 - u[0]);
            double mut = S->mus[l] + S->mua[l];
            if (uz == 0.0) {
                if (mut == 0.0) { tal[T_CAP]++; break; }  /* can never move */
                goto interact;
            }
            {
                double db = (uz > 0.0) ? (S->zbot[l] - z) / uz : (S->ztop[l] - z) / uz;
                if (mut * db <= s) {
                    /* reach the interface */
                    s -= mut * db;
                    if (s < 0.0) s = 0.0;
                    int down = uz > 0.0;
                    z = down ? S->zbot[l] : S->ztop[l];
                    int exit_ = down ? (l == S->L - 1) : (l == 0);
                    double nt, kt = 0.0;
                    if (down) {
                        if (exit_) { nt = S->n_lo; kt = S->k_lo; }
                        else nt = S->n[l + 1];
                    } else {
                        nt = exit_ ? S->n_up : S->n[l - 1];
                    }
                    double ci = fabs(uz);
                    double R = orc_fresnel(ci, S->n[l], nt, kt);
                    if (u[1] < R) {
                        uz = -uz;
                    } else if (exit_) {
                        tal[down ? T_TRANS : T_RDIFF]++;
                        break;
                    } else {
                        double rr = S->n[l] / nt;
                        double ct = sqrt(1.0 - rr * rr * (1.0 - ci * ci));
                        uz = down ? ct : -ct;
                        l += down ? 1 : -1;
                    }
                    continue;
                }
                z += uz * s / mut;
                s = 0.0;
            }
        interact:
            if (u[1] < S->mus[l] / mut) {
                double ct = orc_hg_cos(S->g[l], u[2]);
                double st = sqrt(fmax(0.0, 1.0 - ct * ct));
                double so = sqrt(fmax(0.0, 1.0 - uz * uz));
                uz = uz * ct + so * st * cos(2.0 * M_PI * u[3]);
                if (uz > 1.0) uz = 1.0;
                if (uz < -1.0) uz = -1.0;
            } else {
                tal[T_ABS]++;
                break;
            }
        }
        tal[T_STEPS] += k;
    }
}

static void build_stack(orc_stack* S, int L, const double* mus, const double* mua, const double* g,
                        const double* n, const double* t, double n_up, double n_lo, double k_lo,
                        double mu0, uint32_t stream)
{
    S->L = L;
    double z = 0.0;
    for (int l = 0; l < L; ++l) {
        S->mus[l] = mus[l]; S->mua[l] = mua[l]; S->g[l] = g[l]; S->n[l] = n[l];
        S->ztop[l] = z; z += t[l]; S->zbot[l] = z;
    }
    S->n_up = n_up; S->n_lo = n_lo; S->k_lo = k_lo; S->mu0 = mu0; S->stream = stream;
}

/* Single stack, single thread. */
void orc_walk(int L, const double* mus, const double* mua, const double* g, const double* n,
              const double* t, double n_up, double n_lo, double k_lo, double mu0, uint32_t stream,
              uint64_t seed, uint64_t p_begin, uint64_t p_end, uint64_t max_steps, uint64_t* tal)
{
    orc_stack S;
    build_stack(&S, L, mus, mua, g, n, t, n_up, n_lo, k_lo, mu0, stream);
    memset(tal, 0, sizeof(uint64_t) * T_N);
    walk_range(&S, seed, p_begin, p_end, max_steps, tal);
}

/* --- thread-parallel driver over (item, photon chunk) units --------------- */
typedef struct {
    int n_items, max_layers;
    const int32_t* n_layers;
    const double *mus, *mua, *g, *n, *t, *n_up, *n_lo, *k_lo, *mu0;
    const uint64_t* photons;
    const uint32_t* streams;
    uint64_t seed, max_steps, chunk;
    const uint64_t* unit_start;   /* [n_items + 1] prefix of unit counts */
    uint64_t n_units;
    uint64_t next;                /* shared unit cursor */
    uint64_t* tallies;            /* [n_items * T_N] */
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* J = (batch_job*)arg;
    for (;;) {
        uint64_t u = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (u >= J->n_units) break;
        /* item of unit u: largest i with unit_start[i] <= u */
        int lo = 0, hi = J->n_items;
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (J->unit_start[mid] <= u) lo = mid; else hi = mid;
        }
        int i = lo;
        uint64_t c = u - J->unit_start[i];
        uint64_t p0 = c * J->chunk;
        uint64_t p1 = p0 + J->chunk;
        if (p1 > J->photons[i]) p1 = J->photons[i];
        size_t o = (size_t)i * J->max_layers;
        orc_stack S;
        build_stack(&S, J->n_layers[i], J->mus + o, J->mua + o, J->g + o, J->n + o, J->t + o,
                    J->n_up[i], J->n_lo[i], J->k_lo[i], J->mu0[i],
                    J->streams ? J->streams[i] : (uint32_t)i);
        uint64_t tal[T_N] = {0};
        walk_range(&S, J->seed, p0, p1, J->max_steps, tal);
        for (int k = 0; k < T_N; ++k)
            __atomic_fetch_add(&J->tallies[(size_t)i * T_N + k], tal[k], __ATOMIC_RELAXED);
    }
    return NULL;
}

/* Walk a batch of items with n_threads POSIX threads.  Arrays are
 * [n_items * max_layers] row-major (per-layer) or [n_items].  streams may be
 * NULL (stream id = item index).  tallies [n_items * 6] are overwritten. */
int orc_walk_batch(int n_items, int max_layers, const int32_t* n_layers, const double* mus,
                   const double* mua, const double* g, const double* n, const double* t,
                   const double* n_up, const double* n_lo, const double* k_lo, const double* mu0,
                   const uint64_t* photons, const uint32_t* streams, uint64_t seed,
                   uint64_t max_steps, int n_threads, uint64_t* tallies)
{
    if (n_items < 0 || max_layers < 1 || max_layers > ORC_MAX_LAYERS || n_threads < 1) return -1;
    memset(tallies, 0, sizeof(uint64_t) * (size_t)n_items * T_N);
    const uint64_t chunk = 8192;
    uint64_t* us = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n_items + 1));
    us[0] = 0;
    for (int i = 0; i < n_items; ++i) us[i + 1] = us[i] + (photons[i] + chunk - 1) / chunk;
    batch_job J = {n_items, max_layers, n_layers, mus, mua, g, n, t, n_up, n_lo, k_lo, mu0,
                   photons, streams, seed, max_steps, chunk, us, us[n_items], 0, tallies};
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int k = 0; k < n_threads; ++k) pthread_create(&th[k], NULL, batch_worker, &J);
    for (int k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    free(th);
    free(us);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Weighted-packet walk (the MCML form of ref. [45])                          */
/* ------------------------------------------------------------------------- */
/* The same stacks, boundaries and counter layout as the analog walk, with the
 * photon carried as a packet of weight W instead of being absorbed whole:
 *   - launch: the specular part R0 is tallied deterministically (no draw) and
 *     the packet enters with W = 1 - R0;
 *   - boundaries: as in the analog walk (all-or-none Fresnel decision with
 *     U1); an exiting packet tallies its whole weight;
 *   - interaction: the fraction mu_a/mu_t of W is deposited (absorbed), the
 *     rest scatters (HG with U2, azimuth U3) -- there is no albedo draw;
 *   - roulette: when W falls below WT_THRESHOLD the packet survives with
 *     probability WT_CHANCE (decided by U1) and weight W / WT_CHANCE, else it
 *     ends; a packet whose weight became exactly zero ends at once.
 * Tallies per item (double): specular R (sum of R0), diffuse R, A, T (sums of
 * weight), the sums of squares of each photon's diffuse-R, A and T totals
 * (variances), and the number of photons ended by roulette.  Every estimate
 * is unbiased; R + A + T = 1 holds in expectation, not photon by photon. */
#define WT_THRESHOLD 1e-4
#define WT_CHANCE 0.1
enum { WT_RSPEC = 0, WT_RDIFF, WT_ABS, WT_TRANS, WT_RDIFF2, WT_ABS2, WT_TRANS2, WT_ROULETTE, WT_N };

static void walk_range_weighted(const orc_stack* S, uint64_t seed, uint64_t p_begin, uint64_t p_end,
                                uint64_t max_steps, double wt[WT_N], uint64_t* steps, uint64_t* capped)
{
    double u[4];
    const double R0 = orc_fresnel(S->mu0, S->n_up, S->n[0], 0.0);
    for (uint64_t p = p_begin; p < p_end; ++p) {
        wt[WT_RSPEC] += R0;
        double w = 1.0 - R0, a = 0.0;
        double r = S->n_up / S->n[0];
        double uz = sqrt(1.0 - r * r * (1.0 - S->mu0 * S->mu0));
        int l = 0;
        double z = 0.0, s = 0.0;
        uint64_t k = 0;
        int out = -1;   /* WT_RDIFF or WT_TRANS when the packet leaves the stack */
        if (w > 0.0) {
            for (;;) {
                ++k;
                if (k > max_steps) { ++*capped; k = max_steps; break; }
                draw_block(p, (uint32_t)k, S->stream, seed, u);
                if (s == 0.0) s = -log(1.0 - u[0]);
                double mut = S->mus[l] + S->mua[l];
                if (uz == 0.0) {
                    if (mut == 0.0) { ++*capped; break; }
                    goto interact;
                }
                {
                    double db = (uz > 0.0) ? (S->zbot[l] - z) / uz : (S->ztop[l] - z) / uz;
                    if (mut * db <= s) {
                        s -= mut * db;
                        if (s < 0.0) s = 0.0;
                        int down = uz > 0.0;
                        z = down ? S->zbot[l] : S->ztop[l];
                        int exit_ = down ? (l == S->L - 1) : (l == 0);
                        double nt, kt = 0.0;
                        if (down) {
                            if (exit_) { nt = S->n_lo; kt = S->k_lo; }
                            else nt = S->n[l + 1];
                        } else {
                            nt = exit_ ? S->n_up : S->n[l - 1];
                        }
                        double ci = fabs(uz);
                        double R = orc_fresnel(ci, S->n[l], nt, kt);
                        if (u[1] < R) {
                            uz = -uz;
                        } else if (exit_) {
                            out = down ? WT_TRANS : WT_RDIFF;
                            break;
                        } else {
                            double rr = S->n[l] / nt;
                            double ct = sqrt(1.0 - rr * rr * (1.0 - ci * ci));
                            uz = down ? ct : -ct;
                            l += down ? 1 : -1;
                        }
                        continue;
                    }
                    z += uz * s / mut;
                    s = 0.0;
                }
            interact:
                {
                    double dw = w * (S->mua[l] / mut);   /* exactly w without scattering */
                    a += dw;
                    w -= dw;
                    if (w <= 0.0) { w = 0.0; break; }
                    double ct = orc_hg_cos(S->g[l], u[2]);
                    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
                    double so = sqrt(fmax(0.0, 1.0 - uz * uz));
                    uz = uz * ct + so * st * cos(2.0 * M_PI * u[3]);
                    if (uz > 1.0) uz = 1.0;
                    if (uz < -1.0) uz = -1.0;
                    if (w < WT_THRESHOLD) {
                        if (u[1] < WT_CHANCE) w /= WT_CHANCE;
                        else { w = 0.0; wt[WT_ROULETTE] += 1.0; break; }
                    }
                }
            }
        }
        if (out >= 0) {
            wt[out] += w;
            wt[out == WT_TRANS ? WT_TRANS2 : WT_RDIFF2] += w * w;
        }
        wt[WT_ABS] += a;
        wt[WT_ABS2] += a * a;
        *steps += k;
    }
}

typedef struct {
    batch_job B;
    double* wtallies;             /* [n_items * WT_N] */
    uint64_t* wsteps;             /* [n_items * 2]: photon-steps, capped photons */
    pthread_mutex_t lock;
} wbatch_job;

static void* wbatch_worker(void* arg)
{
    wbatch_job* WJ = (wbatch_job*)arg;
    batch_job* J = &WJ->B;
    for (;;) {
        uint64_t u = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (u >= J->n_units) break;
        int lo = 0, hi = J->n_items;
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (J->unit_start[mid] <= u) lo = mid; else hi = mid;
        }
        int i = lo;
        uint64_t c = u - J->unit_start[i];
        uint64_t p0 = c * J->chunk;
        uint64_t p1 = p0 + J->chunk;
        if (p1 > J->photons[i]) p1 = J->photons[i];
        size_t o = (size_t)i * J->max_layers;
        orc_stack S;
        build_stack(&S, J->n_layers[i], J->mus + o, J->mua + o, J->g + o, J->n + o, J->t + o,
                    J->n_up[i], J->n_lo[i], J->k_lo[i], J->mu0[i],
                    J->streams ? J->streams[i] : (uint32_t)i);
        double wt[WT_N] = {0};
        uint64_t st = 0, cap = 0;
        walk_range_weighted(&S, J->seed, p0, p1, J->max_steps, wt, &st, &cap);
        pthread_mutex_lock(&WJ->lock);
        for (int k = 0; k < WT_N; ++k) WJ->wtallies[(size_t)i * WT_N + k] += wt[k];
        WJ->wsteps[2 * (size_t)i] += st;
        WJ->wsteps[2 * (size_t)i + 1] += cap;
        pthread_mutex_unlock(&WJ->lock);
    }
    return NULL;
}

/* Weighted-packet walk of a batch (arrays as orc_walk_batch).  tallies
 * [n_items * 8] (doubles, see WT_*) and steps [n_items * 2] (photon-steps,
 * capped photons) are overwritten.  Sums over photon chunks are added in an
 * order that depends on thread timing, so results agree to rounding. */
int orc_walk_weighted_batch(int n_items, int max_layers, const int32_t* n_layers, const double* mus,
                            const double* mua, const double* g, const double* n, const double* t,
                            const double* n_up, const double* n_lo, const double* k_lo, const double* mu0,
                            const uint64_t* photons, const uint32_t* streams, uint64_t seed,
                            uint64_t max_steps, int n_threads, double* tallies, uint64_t* steps)
{
    if (n_items < 0 || max_layers < 1 || max_layers > ORC_MAX_LAYERS || n_threads < 1) return -1;
    memset(tallies, 0, sizeof(double) * (size_t)n_items * WT_N);
    memset(steps, 0, sizeof(uint64_t) * (size_t)n_items * 2);
    const uint64_t chunk = 8192;
    uint64_t* us = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n_items + 1));
    us[0] = 0;
    for (int i = 0; i < n_items; ++i) us[i + 1] = us[i] + (photons[i] + chunk - 1) / chunk;
    wbatch_job WJ;
    batch_job B = {n_items, max_layers, n_layers, mus, mua, g, n, t, n_up, n_lo, k_lo, mu0,
                   photons, streams, seed, max_steps, chunk, us, us[n_items], 0, NULL};
    WJ.B = B;
    WJ.wtallies = tallies;
    WJ.wsteps = steps;
    pthread_mutex_init(&WJ.lock, NULL);
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int k = 0; k < n_threads; ++k) pthread_create(&th[k], NULL, wbatch_worker, &WJ);
    for (int k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    pthread_mutex_destroy(&WJ.lock);
    free(th);
    free(us);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Mie theory, eqs. (1)-(5), (10)-(12), (15)                                  */
/* ------------------------------------------------------------------------- */
/* Logarithmic derivative D_n(z) = psi_n'(z)/psi_n(z) of the Riccati-Bessel
 * psi_n(z) = z j_n(z) (A_n of eq. (4)), by downward recurrence
 * D_{n-1} = n/z - 1/(D_n + n/z) started at zero far above n_max. */
static void log_derivative(double complex z, int nmax, double complex* D)
{
    int nstart = nmax;
    double az = cabs(z);
    if (az > nstart) nstart = (int)ceil(az);
    nstart += 16;
    double complex d = 0.0;
    for (int n = nstart; n > nmax; --n) d = n / z - 1.0 / (d + n / z);
    D[nmax] = d;
    for (int n = nmax; n >= 1; --n) D[n - 1] = n / z - 1.0 / (D[n] + n / z);
}

/* Mie coefficients a_n, b_n (n = 1..nmax) of a sphere of relative index
 * m = n_p/n_m with host size parameter x (complex for an absorbing host).
 * With psi_n = z j_n, xi_n = z h_n^(1), eqs. (2)-(5) become
 *   a_n = [(D_n(mx)/m + n/x) psi_n(x) - psi_{n-1}(x)]
 *       / [(D_n(mx)/m + n/x) xi_n(x)  - xi_{n-1}(x)]
 *   b_n = [(m D_n(mx) + n/x) psi_n(x) - psi_{n-1}(x)]
 *       / [(m D_n(mx) + n/x) xi_n(x)  - xi_{n-1}(x)].
 * psi_n(x) follows from the upward recurrence psi_{n+1} = (2n+1)/x psi_n -
 * psi_{n-1} (psi_0 = sin x, psi_{-1} = cos x) while n <= |x|, where it is
 * stable and psi_n oscillates through zeros; above |x| psi_n decays
 * monotonically and is taken from the ratio psi_{n-1}/psi_n = D_n(x) + n/x.
 * xi_n(x) by upward recurrence xi_{n+1} = (2n+1)/x xi_n - xi_{n-1} from
 * xi_0 = sin x - i cos x, xi_{-1} = cos x + i sin x. */
int orc_mie_coeffs(double xr, double xi, double mr, double mi, int nmax, double* a_out, double* b_out)
{
    if (nmax < 1) return -1;
    double complex x = xr + I * xi, m = mr + I * mi;
    double complex* Dy = (double complex*)malloc(sizeof(double complex) * (nmax + 1));
    double complex* Dx = (double complex*)malloc(sizeof(double complex) * (nmax + 1));
    log_derivative(m * x, nmax, Dy);
    log_derivative(x, nmax, Dx);
    double complex psi_prev = csin(x);                 /* psi_0 */
    double complex psi_m1 = ccos(x);                   /* psi_-1 */
    double ax = cabs(x);
    double complex xi_0 = csin(x) - I * ccos(x);       /* xi_0  */
    double complex xi_m1 = ccos(x) + I * csin(x);      /* xi_-1 */
    for (int n = 1; n <= nmax; ++n) {
        double complex psi_n = (n <= ax) ? (2.0 * n - 1.0) / x * psi_prev - psi_m1
                                         : psi_prev / (Dx[n] + n / x);
        double complex xi_n = (2.0 * n - 1.0) / x * xi_0 - xi_m1;
        if (!isfinite(cabs(xi_n)) || cabs(xi_n) > 1e250) {
            /* far above |x| xi_n overflows while psi_n/xi_n -> 0: the
             * remaining coefficients are zero to double precision */
            for (int k = n; k <= nmax; ++k) {
                a_out[2 * (k - 1)] = a_out[2 * (k - 1) + 1] = 0.0;
                b_out[2 * (k - 1)] = b_out[2 * (k - 1) + 1] = 0.0;
            }
            break;
        }
        double complex ta = Dy[n] / m + n / x;
        double complex tb = m * Dy[n] + n / x;
        double complex an = (ta * psi_n - psi_prev) / (ta * xi_n - xi_0);
        double complex bn = (tb * psi_n - psi_prev) / (tb * xi_n - xi_0);
        a_out[2 * (n - 1)] = creal(an); a_out[2 * (n - 1) + 1] = cimag(an);
        b_out[2 * (n - 1)] = creal(bn); b_out[2 * (n - 1) + 1] = cimag(bn);
        psi_m1 = psi_prev; psi_prev = psi_n;
        xi_m1 = xi_0; xi_0 = xi_n;
    }
    free(Dy); free(Dx);
    return 0;
}

/* Series length of eq. (12): ceil(2 + |y| + 4.3 |y|^(1/3)). */
int orc_mie_nmax(double yabs) { return (int)ceil(2.0 + yabs + 4.3 * cbrt(yabs)); }

/* Geometric term of eq. (10), gamma = 2(1 + (alpha-1) e^alpha)/alpha^2, with
 * alpha = 4 pi r k_m / lambda; for small alpha the cancelling form is replaced
 * by its Taylor series 1 + 2a/3 + a^2/4 + a^3/15 + a^4/72. */
double orc_gamma(double alpha)
{
    if (fabs(alpha) < 1e-3)
        return 1.0 + alpha * (2.0 / 3.0 + alpha * (0.25 + alpha * (1.0 / 15.0 + alpha / 72.0)));
    return 2.0 * (1.0 + (alpha - 1.0) * exp(alpha)) / (alpha * alpha);
}

/* Single sphere of radius r in host n_m + i k_m at vacuum wavelength lam:
 * efficiencies q_ext = C_ext/(pi r^2), q_sca = C_sca/(pi r^2) from eqs.
 * (11)-(12) and the asymmetry parameter g from eq. (15).  Outputs
 * out[0] = q_ext, out[1] = q_sca, out[2] = g, out[3] = nmax used. */
int orc_mie_sphere(double lam, double nm, double km, double np_, double kp, double r, double* out)
{
    double complex Nm = nm + I * km, Np = np_ + I * kp;
    double complex x = 2.0 * M_PI * r * Nm / lam;
    double complex y = 2.0 * M_PI * r * Np / lam;
    int nmax = orc_mie_nmax(cabs(y));
    int nn = nmax + 1;       /* eq. (15) needs a_{nmax+1} */
    double* a = (double*)malloc(sizeof(double) * 2 * nn);
    double* b = (double*)malloc(sizeof(double) * 2 * nn);
    orc_mie_coeffs(creal(x), cimag(x), creal(Np / Nm), cimag(Np / Nm), nn, a, b);
    double sext = 0.0, ssca = 0.0, sg = 0.0;
    double complex iNm2 = 1.0 / (Nm * Nm);
    for (int n = 1; n <= nmax; ++n) {
        double complex an = a[2 * (n - 1)] + I * a[2 * (n - 1) + 1];
        double complex bn = b[2 * (n - 1)] + I * b[2 * (n - 1) + 1];
        double complex an1 = a[2 * n] + I * a[2 * n + 1];
        double complex bn1 = b[2 * n] + I * b[2 * n + 1];
        sext += (2.0 * n + 1.0) * creal((an + bn) * iNm2);
        ssca += (2.0 * n + 1.0) * (creal(an * conj(an)) + creal(bn * conj(bn)));
        sg += (double)n * (n + 2.0) / (n + 1.0) * creal(an * conj(an1) + bn * conj(bn1))
            + (2.0 * n + 1.0) / ((double)n * (n + 1.0)) * creal(an * conj(bn));
    }
    double alpha = 4.0 * M_PI * r * km / lam;
    double gam = orc_gamma(alpha);
    double cext = lam * lam / (2.0 * M_PI) * sext;
    double csca = lam * lam * exp(-alpha) / (2.0 * M_PI * gam * creal(Nm * conj(Nm))) * ssca;
    double area = M_PI * r * r;
    out[0] = cext / area;
    out[1] = csca / area;
    out[2] = ssca > 0.0 ? 2.0 * sg / ssca : 0.0;
    out[3] = (double)nmax;
    free(a); free(b);
    return 0;
}

/* --- coated (core-shell) spheres, supplementary eqs. (S1)-(S9) ------------- */
/* Riccati-Bessel psi_n(z) = z j_n(z) (eq. (S7)), n = 0..nmax: upward
 * recurrence while n <= |z|, above that from the logarithmic derivative,
 * psi_n = psi_{n-1} / (D_n + n/z) (the upward form loses accuracy there). */
static void riccati_psi(double complex z, int nmax, double complex* psi)
{
    double complex* D = (double complex*)malloc(sizeof(double complex) * (nmax + 1));
    log_derivative(z, nmax, D);
    double az = cabs(z);
    double complex pm1 = ccos(z);
    psi[0] = csin(z);
    for (int n = 1; n <= nmax; ++n) {
        psi[n] = (n <= az) ? (2.0 * n - 1.0) / z * psi[n - 1] - (n == 1 ? pm1 : psi[n - 2])
                           : psi[n - 1] / (D[n] + n / z);
    }
    free(D);
}

/* chi_n(z) = z y_n(z) (eq. (S8)), n = 0..nmax, by the upward recurrence,
 * stable for this growing solution: chi_0 = -cos z, chi_1 = -cos z / z - sin z. */
static void riccati_chi(double complex z, int nmax, double complex* chi)
{
    chi[0] = -ccos(z);
    if (nmax >= 1) chi[1] = -ccos(z) / z - csin(z);
    for (int n = 2; n <= nmax; ++n) chi[n] = (2.0 * n - 1.0) / z * chi[n - 1] - chi[n - 2];
}

/* derivative of a Riccati-Bessel function: f'_n(z) = f_{n-1}(z) - (n/z) f_n(z) */
static double complex rb_deriv(const double complex* f, int n, double complex z)
{
    return f[n - 1] - (double)n / z * f[n];
}

/* Mie coefficients of a coated sphere, written out as eqs. (S1)-(S4): core
 * size parameter x = k r_core and outer y = k r_outer (k the host wave number,
 * complex in an absorbing host), m1 = core / host, m2 = shell / host (S5, S6),
 * xi_n = psi_n + i chi_n (S9, first-kind Hankel).  n = 1..nmax.  Meant for
 * moderate sizes (the literal form lets chi_n grow without bound). */
int orc_mie_coated_coeffs(double xr, double xi_, double yr, double yi, double m1r, double m1i, double m2r,
                          double m2i, int nmax, double* a_out, double* b_out)
{
    if (nmax < 1) return -1;
    double complex x = xr + I * xi_, y = yr + I * yi;
    double complex m1 = m1r + I * m1i, m2 = m2r + I * m2i;
    size_t sz = sizeof(double complex) * (nmax + 1);
    double complex *p1x = malloc(sz), *p2x = malloc(sz), *c2x = malloc(sz), *p2y = malloc(sz), *c2y = malloc(sz);
    double complex *py = malloc(sz), *cy = malloc(sz);
    riccati_psi(m1 * x, nmax, p1x);
    riccati_psi(m2 * x, nmax, p2x);
    riccati_chi(m2 * x, nmax, c2x);
    riccati_psi(m2 * y, nmax, p2y);
    riccati_chi(m2 * y, nmax, c2y);
    riccati_psi(y, nmax, py);
    riccati_chi(y, nmax, cy);
    int bad = 0;
    for (int n = 1; n <= nmax; ++n) {
        double complex dp1x = rb_deriv(p1x, n, m1 * x), dp2x = rb_deriv(p2x, n, m2 * x);
        double complex dc2x = rb_deriv(c2x, n, m2 * x), dp2y = rb_deriv(p2y, n, m2 * y);
        double complex dc2y = rb_deriv(c2y, n, m2 * y), dpy = rb_deriv(py, n, y), dcy = rb_deriv(cy, n, y);
        double complex xin = py[n] + I * cy[n], dxin = dpy + I * dcy;
        /* (S3), (S4) */
        double complex An = (m2 * p2x[n] * dp1x - m1 * dp2x * p1x[n]) / (m2 * c2x[n] * dp1x - m1 * dc2x * p1x[n]);
        double complex Bn = (m2 * p1x[n] * dp2x - m1 * p2x[n] * dp1x) / (m2 * dc2x * p1x[n] - m1 * dp1x * c2x[n]);
        /* (S1), (S2) */
        double complex ua = dp2y - An * dc2y, va = p2y[n] - An * c2y[n];
        double complex ub = dp2y - Bn * dc2y, vb = p2y[n] - Bn * c2y[n];
        double complex an = (py[n] * ua - m2 * dpy * va) / (xin * ua - m2 * dxin * va);
        double complex bn = (m2 * py[n] * ub - dpy * vb) / (m2 * xin * ub - dxin * vb);
        if (!isfinite(cabs(an)) || !isfinite(cabs(bn))) bad = 1;
        a_out[2 * (n - 1)] = creal(an); a_out[2 * (n - 1) + 1] = cimag(an);
        b_out[2 * (n - 1)] = creal(bn); b_out[2 * (n - 1) + 1] = cimag(bn);
    }
    free(p1x); free(p2x); free(c2x); free(p2y); free(c2y); free(py); free(cy);
    return bad ? -2 : 0;
}

/* Efficiencies of a coated sphere (core radius rc, index nc + i kc; shell to
 * radius r, index ns + i ks) in host nm + i km: eqs. (11), (12), (15) with the
 * coefficients of (S1)-(S4), the cross sections referred to the outer radius,
 * and alpha of eq. (10) from the outer radius.  The series length is eq. (12)
 * with |y| the larger of the core's and the shell's size parameters.
 * out = q_ext, q_sca, g, nmax; returns < 0 if the literal form overflowed. */
int orc_mie_coated(double lam, double nm, double km, double nc, double kc, double rc, double ns, double ks,
                   double r, double* out)
{
    double complex Nm = nm + I * km, Nc = nc + I * kc, Ns = ns + I * ks;
    double complex x = 2.0 * M_PI * rc * Nm / lam, y = 2.0 * M_PI * r * Nm / lam;
    double yabs = fmax(2.0 * M_PI * r * cabs(Ns) / lam, 2.0 * M_PI * rc * cabs(Nc) / lam);
    int nmax = orc_mie_nmax(yabs);
    int nn = nmax + 1;
    double* a = (double*)malloc(sizeof(double) * 2 * nn);
    double* b = (double*)malloc(sizeof(double) * 2 * nn);
    double complex m1 = Nc / Nm, m2 = Ns / Nm;
    int rc_ = orc_mie_coated_coeffs(creal(x), cimag(x), creal(y), cimag(y), creal(m1), cimag(m1), creal(m2),
                                    cimag(m2), nn, a, b);
    double sext = 0.0, ssca = 0.0, sg = 0.0;
    double complex iNm2 = 1.0 / (Nm * Nm);
    for (int n = 1; n <= nmax; ++n) {
        double complex an = a[2 * (n - 1)] + I * a[2 * (n - 1) + 1];
        double complex bn = b[2 * (n - 1)] + I * b[2 * (n - 1) + 1];
        double complex an1 = a[2 * n] + I * a[2 * n + 1];
        double complex bn1 = b[2 * n] + I * b[2 * n + 1];
        sext += (2.0 * n + 1.0) * creal((an + bn) * iNm2);
        ssca += (2.0 * n + 1.0) * (creal(an * conj(an)) + creal(bn * conj(bn)));
        sg += (double)n * (n + 2.0) / (n + 1.0) * creal(an * conj(an1) + bn * conj(bn1))
            + (2.0 * n + 1.0) / ((double)n * (n + 1.0)) * creal(an * conj(bn));
    }
    double alpha = 4.0 * M_PI * r * km / lam;
    double gam = orc_gamma(alpha);
    double cext = lam * lam / (2.0 * M_PI) * sext;
    double csca = lam * lam * exp(-alpha) / (2.0 * M_PI * gam * creal(Nm * conj(Nm))) * ssca;
    double area = M_PI * r * r;
    out[0] = cext / area;
    out[1] = csca / area;
    out[2] = ssca > 0.0 ? 2.0 * sg / ssca : 0.0;
    out[3] = (double)nmax;
    free(a); free(b);
    return rc_;
}

/* The paper's size-distribution option: one diameter D with standard
 * deviation sd becomes 101 diameters evenly spaced over D - 3 sd .. D + 3 sd
 * with Gaussian weights, renormalised to sum to one (read as volume-fraction
 * weights, like the per-size fractions of a custom distribution); diameters
 * that are not positive are left out.  Writes radii and weights, returns the
 * number of sizes (1 when sd = 0). */
int orc_gaussian_sizes(double D, double sd, double* r_out, double* w_out)
{
    if (!(sd > 0.0)) { r_out[0] = 0.5 * D; w_out[0] = 1.0; return 1; }
    int k = 0;
    double sum = 0.0;
    for (int j = 0; j <= 100; ++j) {
        double d = D - 3.0 * sd + 6.0 * sd * j / 100.0;
        if (!(d > 0.0)) continue;
        double z = (d - D) / sd;
        r_out[k] = 0.5 * d;
        w_out[k] = exp(-0.5 * z * z);
        sum += w_out[k];
        ++k;
    }
    for (int j = 0; j < k; ++j) w_out[j] /= sum;
    return k;
}

/* Effective medium of one layer at one wavelength, eqs. (13)-(20).
 * Particles i = 0..np-1 with index np_[i] + i kp[i], radius r[i], volume
 * fraction f[i].  Outputs out[0] = mu_s, out[1] = mu_a (total, eq. (20)),
 * out[2] = g (eq. (16)).
 *   mu_s = sum 1.5 q_sca,i f_i / (2 r_i),  mu_a = sum 1.5 (q_ext,i - q_sca,i) f_i / (2 r_i)
 *   g    = sum (1.5 q_sca,i f_i g_i / (2 r_i)) / mu_s      (g = 0 when mu_s = 0)
 * Negative summed coefficients are set to zero; when the total volume
 * fraction exceeds 0.08 both are multiplied by
 * C = 1 + 1.5 F - 0.75 F^2, F = sum f_i; finally the matrix absorption
 * 4 pi k_m (1 - F) / lambda is added to mu_a.
 * Optional per-particle arrays (NULL = none): sd, the standard deviation of
 * the diameter 2 r (the particle becomes orc_gaussian_sizes(); r is its mean
 * radius); rc, nc, kc, a core of radius rc > 0 and index nc + i kc inside a
 * shell of index n_p + i k_p out to r (no size spread for coated spheres, as
 * in the paper).  Returns < 0 if a coated sphere overflowed the literal form. */
int orc_layer_optics_ex(double lam, double nm, double km, int np, const double* np_, const double* kp,
                        const double* r, const double* f, const double* sd, const double* rc,
                        const double* nc, const double* kc, double* out)
{
    double mus = 0.0, mua = 0.0, gs = 0.0, F = 0.0;
    double rr[101], ww[101];
    int status = 0;
    for (int i = 0; i < np; ++i) {
        F += f[i];
        if (rc && rc[i] > 0.0) {
            /* a coated sphere: core rc, shell out to r (no size spread) */
            double q[4];
            if (orc_mie_coated(lam, nm, km, nc[i], kc[i], rc[i], np_[i], kp[i], r[i], q) < 0) status = -2;
            double ws = 1.5 * q[1] * f[i] / (2.0 * r[i]);
            mus += ws;
            mua += 1.5 * (q[0] - q[1]) * f[i] / (2.0 * r[i]);
            gs += ws * q[2];
            continue;
        }
        int k = orc_gaussian_sizes(2.0 * r[i], sd ? sd[i] : 0.0, rr, ww);
        for (int j = 0; j < k; ++j) {
            double q[4];
            orc_mie_sphere(lam, nm, km, np_[i], kp[i], rr[j], q);
            double fj = f[i] * ww[j];
            double ws = 1.5 * q[1] * fj / (2.0 * rr[j]);
            mus += ws;
            mua += 1.5 * (q[0] - q[1]) * fj / (2.0 * rr[j]);
            gs += ws * q[2];
        }
    }
    double g = mus > 0.0 ? gs / mus : 0.0;
    if (mus < 0.0) mus = 0.0;
    if (mua < 0.0) mua = 0.0;
    if (F > 0.08) {
        double C = 1.0 + 1.5 * F - 0.75 * F * F;
        mus *= C;
        mua *= C;
    }
    mua += 4.0 * M_PI * km * (1.0 - F) / lam;
    out[0] = mus; out[1] = mua; out[2] = g;
    return status;
}

int orc_layer_optics(double lam, double nm, double km, int np, const double* np_, const double* kp,
                     const double* r, const double* f, double* out)
{
    return orc_layer_optics_ex(lam, nm, km, np, np_, kp, r, f, NULL, NULL, NULL, NULL, out);
}

/* Many cells (layer x wavelength), CSR particle lists, threaded. */
typedef struct {
    int n_cells;
    const double *lam, *nm, *km;
    const int64_t* off;
    const double *np_, *kp, *r, *f;
    const double *sd, *rc, *nc, *kc;   /* optional, NULL = homogeneous, one size */
    double* out;
    int next;
    int status;
} optics_job;

static void* optics_worker(void* arg)
{
    optics_job* J = (optics_job*)arg;
    for (;;) {
        int c = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (c >= J->n_cells) break;
        int64_t o = J->off[c];
        int cnt = (int)(J->off[c + 1] - o);
        int st = orc_layer_optics_ex(J->lam[c], J->nm[c], J->km[c], cnt, J->np_ + o, J->kp + o, J->r + o,
                                     J->f + o, J->sd ? J->sd + o : NULL, J->rc ? J->rc + o : NULL,
                                     J->nc ? J->nc + o : NULL, J->kc ? J->kc + o : NULL, J->out + 3 * (size_t)c);
        if (st < 0) __atomic_store_n(&J->status, st, __ATOMIC_RELAXED);
    }
    return NULL;
}

int orc_optics_batch_ex(int n_cells, const double* lam, const double* nm, const double* km,
                        const int64_t* offsets, const double* np_, const double* kp, const double* r,
                        const double* f, const double* sd, const double* rc, const double* nc, const double* kc,
                        int n_threads, double* out)
{
    if (n_threads < 1) return -1;
    optics_job J = {n_cells, lam, nm, km, offsets, np_, kp, r, f, sd, rc, nc, kc, out, 0, 0};
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int k = 0; k < n_threads; ++k) pthread_create(&th[k], NULL, optics_worker, &J);
    for (int k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    free(th);
    return J.status;
}

int orc_optics_batch(int n_cells, const double* lam, const double* nm, const double* km,
                     const int64_t* offsets, const double* np_, const double* kp, const double* r,
                     const double* f, int n_threads, double* out)
{
    return orc_optics_batch_ex(n_cells, lam, nm, km, offsets, np_, kp, r, f, NULL, NULL, NULL, NULL, n_threads, out);
}
