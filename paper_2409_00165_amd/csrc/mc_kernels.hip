// mc_kernels.hip -- gfx950 kernels of the Monte Carlo photon walk.
//
//   pack_items    : validate one item per thread and write its packed record
//                   (entry Fresnel reflectance, refracted cosine, per-layer
//                   extinction, albedo, HG constants, interface ratios).
//   reset_run     : zero the caller's tallies and the chunk counter.
//   reset_handoff : clear the hand-off list of a regrouping walk.
//   chunk_scan    : prefix of per-item chunk counts (the work queue).
//   walk          : the persistent photon walk (one photon per lane).
//   walk_long     : the same walk built for heavy-tailed batches: once its
//                   queue is empty a wave enters a drain phase that can hand
//                   its last photons to other waves and prepare their draws
//                   on idle lanes.
//   philox_words / eval_fresnel / eval_hg : thin kernels exposing the device
//                   building blocks to the test-suite.
//
// The walk follows the paper's Monte Carlo transport (Methodology, Photon
// transport): per photon only the depth z and the direction cosine mu_z to
// the surface normal are tracked; the free path follows from the extinction
// coefficient, scatter-versus-absorb from the albedo, the new direction from
// the Henyey-Greenstein asymmetry g (MCML, ref. [45]); every boundary
// reflects or refracts by unpolarised Fresnel with the matrix index, and the
// lower medium may be absorbing (complex index).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fos_device.hpp"
#include "fos_kernels.hpp"

namespace fos {

// ---------------------------------------------------------------------------
// pack + validate
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite_(float x) { return isfinite(x); }

__device__ __forceinline__ void report(unsigned long long* err, int item, int layer, int code)
{
    unsigned long long w = ((unsigned long long)(uint32_t)item << 16) |
                           ((unsigned long long)(layer & 0xFF) << 8) | (unsigned long long)code;
    atomicMin(err, w);
}

__device__ double fresnel_real_d(double c, double ni, double nt)
{
    if (ni == nt) return 0.0;
    const double m = ni / nt;
    const double s2t = m * m * (1.0 - c * c);
    if (s2t >= 1.0) return 1.0;
    const double ct = sqrt(1.0 - s2t);
    const double rs = (m * c - ct) / (m * c + ct);
    const double rp = (c - m * ct) / (c + m * ct);
    return 0.5 * (rs * rs + rp * rp);
}

__global__ void pack_items(PackArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_items) return;
    const int L = a.n_layers[i];
    if (L < 1 || L > a.max_layers) { report(a.err, i, 0, kErrNLayers); return; }
    const size_t o = (size_t)i * a.max_layers;
    const float nu = a.n_upper[i], nl = a.n_lower[i], kl = a.k_lower[i], mu0 = a.mu0[i];
    bool bad = false;
    if (!finite_(nu) || nu < 1.0f) { report(a.err, i, 0, kErrNUpper); bad = true; }
    if (!finite_(nl) || !(nl > 0.0f)) { report(a.err, i, 0, kErrNLower); bad = true; }
    if (!finite_(kl) || kl < 0.0f) { report(a.err, i, 0, kErrKLower); bad = true; }
    if (!finite_(mu0) || !(mu0 > 0.0f) || mu0 > 1.0f) { report(a.err, i, 0, kErrMu0); bad = true; }
    for (int l = 0; l < L; ++l) {
        const float s = a.mu_s[o + l], ab = a.mu_a[o + l], g = a.g[o + l];
        const float n = a.n_layer[o + l], t = a.thickness[o + l];
        if (!finite_(s) || s < 0.0f) { report(a.err, i, l, kErrMuS); bad = true; }
        if (!finite_(ab) || ab < 0.0f) { report(a.err, i, l, kErrMuA); bad = true; }
        if (!finite_(g) || g < -1.0f || g > 1.0f) { report(a.err, i, l, kErrG); bad = true; }
        if (!finite_(n) || n < 1.0f) { report(a.err, i, l, kErrNLayer); bad = true; }
        if (!finite_(t) || !(t > 0.0f)) { report(a.err, i, l, kErrThickness); bad = true; }
    }
    if (bad) return;

    float4* rec = a.table + (size_t)i * rec_f4(a.max_layers);
    // entry: Fresnel from the upper medium into layer 1, refracted cosine
    const double n1 = a.n_layer[o];
    const double R0 = fresnel_real_d((double)mu0, (double)nu, n1);
    const double r = (double)nu / n1;
    const double s2t = r * r * (1.0 - (double)mu0 * mu0);
    const double uz0 = s2t < 1.0 ? sqrt(1.0 - s2t) : 0.0;
    rec[0] = make_float4((float)R0, (float)uz0, nl, kl);
    const uint64_t N = a.photons[i];
    atomicMax(a.max_photons, (unsigned long long)N);
    rec[1] = make_float4(__uint_as_float((uint32_t)N), __uint_as_float((uint32_t)(N >> 32)),
                         __int_as_float(L), __int_as_float(i));
    for (int l = 0; l < L; ++l) {
        const double s = a.mu_s[o + l], ab = a.mu_a[o + l], g = a.g[o + l];
        const double n = a.n_layer[o + l], t = a.thickness[o + l];
        const double mut = s + ab;
        const float alb = mut > 0.0 ? (float)(s / mut) : 0.0f;
        const float inv = mut > 0.0 ? (float)(1.0 / mut) : 0.0f;
        float hG, hh, q1, q2;
        bool mirror;
        hg_constants(g, hG, hh, q1, q2, mirror);
        const double n_up = (l == 0) ? (double)nu : (double)a.n_layer[o + l - 1];
        const double n_dn = (l == L - 1) ? (double)nl : (double)a.n_layer[o + l + 1];
        uint32_t fl = 0;
        if (l == 0) fl |= kExitUp;
        if (l == L - 1) { fl |= kExitDn; if (kl > 0.0f) fl |= kComplexDn; }
        if (n_up == n) fl |= kMatchUp;
        if (n_dn == n && !(fl & kComplexDn)) fl |= kMatchDn;
        if (mirror) fl |= kHgMirror;
        float4* lr = rec + kHdrF4 + kLayerF4 * l;
        lr[0] = make_float4((float)mut, alb, inv, (float)t);
        lr[1] = make_float4(hG, hh, q1, q2);
        lr[2] = make_float4((float)(n / n_up), (float)(n / n_dn), (float)n, __uint_as_float(fl));
        lr[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__global__ void reset_run(unsigned long long* tallies, unsigned long long* counter, int n_items, int nt)
{
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = tid; j < (size_t)n_items * nt; j += stride) tallies[j] = 0ull;
    if (tid == 0) *counter = 0ull;
}

// Clear the hand-off list of a regrouping walk: its control words and the
// ready flag of every record.
__global__ void reset_handoff(unsigned char* hand, uint64_t cap)
{
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    unsigned int* flags = reinterpret_cast<unsigned int*>(hand + hand_flags_offset());
    for (size_t j = tid; j < cap; j += stride) flags[j] = 0u;
    if (tid < 4) reinterpret_cast<unsigned long long*>(hand)[tid] = 0ull;
}

// Exclusive prefix of per-item chunk counts ceil(min(N, cap) / chunk), one
// block of 1024 threads: each thread sums a contiguous run of items, the run
// totals are scanned in LDS, and a second pass writes the prefix.
__global__ __launch_bounds__(1024) void chunk_scan(const float4* table, int rf, int n_items, int chunk,
                                                   uint64_t cap, unsigned long long* prefix)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int per = (n_items + 1023) / 1024;
    const int b = t * per;
    const int e = b + per < n_items ? b + per : n_items;
    auto chunks_of = [&](int i) -> unsigned long long {
        const float4 h1 = table[(size_t)i * rf + 1];
        uint64_t N = (uint64_t)__float_as_uint(h1.x) | ((uint64_t)__float_as_uint(h1.y) << 32);
        if (cap && N > cap) N = cap;
        return (N + (uint64_t)chunk - 1) / (uint64_t)chunk;
    };
    unsigned long long sum = 0;
    for (int i = b; i < e; ++i) sum += chunks_of(i);
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = t > 0 ? part[t - 1] : 0ull;
    for (int i = b; i < e; ++i) {
        prefix[i] = run;
        run += chunks_of(i);
    }
    if (t == 1023) prefix[n_items] = part[1023];
}

// ---------------------------------------------------------------------------
// the persistent walk
// ---------------------------------------------------------------------------
// Each wave works on its own: it claims chunks of photons of one item from a
// global queue (one chunk counter over the items' chunk prefix), stages the
// item's record into one of kSlots LDS slots of its own, and fills idle lanes
// with new photons from the chunk.  A lane keeps the parameters of its
// current layer in registers and re-reads the LDS slot only when it launches
// a photon or crosses into another layer.  Lanes that finish are refilled
// once at least refill_min of them are idle, so a wave keeps walking while
// the photons of an old chunk drain.  Outcomes and steps are counted per
// slot in LDS (one LDS add per finishing lane) and added to the item's
// uint64 tallies when a slot is recycled and at exit.  The refill check runs
// after every step that ends a photon and at least every kStepsPerCheck
// steps.
constexpr int kSlots = 4;

struct LaneLayer {
    float mut, alb, inv_mut, thick;
    float hG, hh, q1, q2;
    float m_up, m_dn, n;
    uint32_t flags;
};

__device__ __forceinline__ void load_layer(const float4* slot_rec, int l, LaneLayer& P)
{
    const float4* lr = slot_rec + kHdrF4 + kLayerF4 * l;
    const float4 a = lr[0], b = lr[1], c = lr[2];
    P.mut = a.x; P.alb = a.y; P.inv_mut = a.z; P.thick = a.w;
    P.hG = b.x; P.hh = b.y; P.q1 = b.z; P.q2 = b.w;
    P.m_up = c.x; P.m_dn = c.y; P.n = c.z; P.flags = __float_as_uint(c.w);
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// A 64-bit value of the first active lane, made wave-uniform.  The builtin
// returns a signed int: each half goes through uint32_t so that the low
// half is not sign-extended into the high one.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ int lane_rank(uint64_t mask)
{
    // number of set bits of mask below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long weight_units(double w)
{
    return (unsigned long long)__double2ull_rn(w * kWeightUnit);
}

// A finished photon's outcome, step count and (weighted form) weights added
// to its item's counters `c0` (LDS slot or HBM tallies).
template <bool WEIGHTED>
__device__ __forceinline__ void finish_photon(unsigned long long* c0, int term, uint32_t k, float wgt, float absd)
{
    if constexpr (WEIGHTED) {
        atomicAdd(c0 + kWSteps, (unsigned long long)k);
        const double ad = (double)absd;
        if (ad > 0.0) {
            atomicAdd(c0 + kWAbs, weight_units(ad));
            atomicAdd(c0 + kWAbs2, weight_units(ad * ad));
        }
        if (term == kTrans || term == kRDiff) {
            const double w = (double)wgt;
            atomicAdd(c0 + (term == kTrans ? kWTrans : kWRDiff), weight_units(w));
            atomicAdd(c0 + (term == kTrans ? kWTrans2 : kWRDiff2), weight_units(w * w));
        } else if (term == kWRoulette) {
            atomicAdd(c0 + kWRoulette, 1ull);
        } else if (term == kCap) {
            atomicAdd(c0 + kWCap, 1ull);
        }
    } else {
        atomicAdd(c0 + kSteps, (unsigned long long)k);
        atomicAdd(c0 + term, 1ull);
    }
}

// Hand-off list control words (WalkArgs::hand_ctl): records reserved and
// records taken so far, waves of the launch alive, takes that timed out.
constexpr int kHandReserved = 0, kHandClaimed = 1, kHandWaves = 2, kHandLost = 3;
constexpr int kAbsorbEvery = 4;       // drain rounds before the first look again at an empty list
constexpr int kAbsorbMax = 128;       // and at most this many
constexpr int kHandRetry = 8;         // drain rounds before a refused hand-off is tried again
constexpr int kHandSpins = 1 << 22;   // bound on the wait for a reserved record's flag

// The counters are read and updated with relaxed device-scope atomics; a
// record's contents are ordered by its flag (release store, acquire load),
// and the live-wave count's acquire-release updates order every hand-off
// before the last wave's final look at the counters.
__device__ __forceinline__ unsigned long long hand_load(unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wave with nothing in flight leaves the launch: true when it may exit.
// The wave whose leaving takes the live-wave count to zero looks at the
// list once more and, if photons are still listed, stays to take them (every
// hand-off is written and flagged before its wave leaves).
__device__ __forceinline__ bool wave_leave(unsigned long long* ctl, int lane)
{
    int stay = 0;
    if (lane == 0) {
        const unsigned long long old = __hip_atomic_fetch_add(ctl + kHandWaves, ~0ull, __ATOMIC_ACQ_REL,
                                                              __HIP_MEMORY_SCOPE_AGENT);
        if (old == 1ull && hand_load(ctl + kHandClaimed) < hand_load(ctl + kHandReserved)) {
            __hip_atomic_fetch_add(ctl + kHandWaves, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            stay = 1;
        }
    }
    return __builtin_amdgcn_readfirstlane(stay) == 0;
}

// WEIGHTED selects the weighted-packet (MCML) form: no specular or albedo
// draws; the packet deposits mu_a/mu_t of its weight at each interaction,
// always scatters, plays roulette below kRouletteThreshold, and tallies
// weights (kNTallyW counters) instead of photon counts (kNTally).
// SINGLE is for problems whose items all have one layer: a photon that is
// not reflected at a face always leaves, so the layer-change code is not
// compiled in.
// One photon-step of a lane from its Philox block X (the lane's step
// counter k already advanced): free path, then boundary or interaction;
// sets `term` when the photon ends.  REC is the lane's item record (its LDS
// slot, or the item table in HBM after a hand-off).  Written out as a macro
// so that each loop of the walk compiles it in place.
#define FOS_WALK_STEP(X, REC)                                                                \
    do {                                                                                     \
        const uint4 x_ = (X);                                                                \
        const float U1 = u24(x_.y);                                                          \
        if (s == 0.f) s = neg_ln(1.0f - u24(x_.x));                                          \
        const float aa = fabsf(uz);                                                          \
        bool interact;                                                                       \
        if (aa == 0.f) {                                                                     \
            interact = P.mut > 0.f;                                                          \
            if (!interact) term = kCap; /* parallel in a clear layer */                      \
        } else {                                                                             \
            const bool down = uz > 0.f;                                                      \
            const float dz = down ? P.thick - z : z;                                         \
            interact = !(P.mut * dz <= s * aa);                                              \
            if (!interact) {                                                                 \
/* reach the interface */                                                                    \
                s = fmaxf(s - P.mut * dz * fast_rcp(aa), 0.f);                               \
                z = down ? P.thick : 0.f;                                                    \
                const uint32_t fl = P.flags;                                                 \
                const bool ex = down ? (fl & kExitDn) : (fl & kExitUp);                      \
                const bool matched = down ? (fl & kMatchDn) : (fl & kMatchUp);               \
                float R = 0.f, ct = aa;                                                      \
                if (down && (fl & kComplexDn)) {                                             \
                    const float4 h0 = (REC)[0];                                              \
                    R = fresnel_complex(aa, P.n, h0.z, h0.w);                                \
                } else if (!matched) {                                                       \
                    const float m = down ? P.m_dn : P.m_up;                                  \
                    const float s2t = m * m * (1.f - aa * aa);                               \
                    if (s2t >= 1.f) {                                                        \
                        R = 1.f;                                                             \
                    } else {                                                                 \
                        ct = fast_sqrt(1.f - s2t);                                           \
                        R = fresnel_real(aa, ct, m);                                         \
                    }                                                                        \
                }                                                                            \
                if (U1 < R) {                                                                \
                    uz = -uz;                                                                \
                } else if (SINGLE || ex) {                                                   \
                    term = down ? kTrans : kRDiff;                                           \
                } else {                                                                     \
                    layer += down ? 1 : -1;                                                  \
                    load_layer((REC), layer, P);                                             \
                    uz = down ? ct : -ct;                                                    \
                    z = down ? 0.f : P.thick;                                                \
                }                                                                            \
            } else {                                                                         \
                z = fmaf(uz * s, P.inv_mut, z);                                              \
                s = 0.f;                                                                     \
            }                                                                                \
        }                                                                                    \
        if (interact) {                                                                      \
            bool scatter;                                                                    \
            if constexpr (WEIGHTED) {                                                        \
/* deposit mu_a/mu_t of the weight, scatter the rest */                                      \
                const float wn = wgt * P.alb;                                                \
                absd += wgt - wn;                                                            \
                wgt = wn;                                                                    \
                scatter = wgt > 0.f;                                                         \
                if (!scatter) term = kAbs;                                                   \
            } else {                                                                         \
                scatter = U1 < P.alb;                                                        \
                if (!scatter) term = kAbs;                                                   \
            }                                                                                \
            if (scatter) {                                                                   \
                const float c = hg_cos(P.hG, P.hh, P.q1, P.q2, (P.flags & kHgMirror) != 0u,  \
                                       u24(x_.z));                                           \
                const float st2 = fmaxf((1.f - uz * uz) * (1.f - c * c), 0.f);               \
                const float cp = __builtin_amdgcn_cosf(u24(x_.w)); /* cos(2 pi U3) */        \
                uz = fminf(fmaxf(fmaf(uz, c, fast_sqrt(st2) * cp), -1.f), 1.f);              \
                if constexpr (WEIGHTED) {                                                    \
                    if (wgt < kRouletteThreshold) {                                          \
                        if (U1 < kRouletteChance) wgt = wgt / kRouletteChance;               \
                        else term = kWRoulette;                                              \
                    }                                                                        \
                }                                                                            \
            }                                                                                \
        }                                                                                    \
    } while (0)

// TAIL is the build for heavy-tailed runs: once a wave has nothing left to
// claim it enters the drain phase below, where photons can be handed between
// waves (regroup_lanes) and few photons in flight get their draws prepared
// on all 64 lanes (tail_lanes).
template <int kStepsPerCheck, bool WEIGHTED, bool SINGLE, bool TAIL>
__device__ __forceinline__ void walk_body(WalkArgs a)
{
    constexpr int NT = WEIGHTED ? kNTallyW : kNTally;
    extern __shared__ float4 smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int rf = a.rec_f4;
    float4* tab = smem + (size_t)wv * kSlots * rf;                         // [kSlots][rf]
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(smem + (size_t)nwaves * kSlots * rf) +
                              (size_t)wv * kSlots * NT;                      // [kSlots][NT]
    int* slot_item = reinterpret_cast<int*>(reinterpret_cast<unsigned long long*>(
                         smem + (size_t)nwaves * kSlots * rf) + (size_t)nwaves * kSlots * NT) +
                     wv * kSlots;                                            // [kSlots]
    // tail build: 64 prepared Philox blocks of this wave, then the wave's copy
    // of the hand-off arguments (list address, capacity, regroup_lanes and
    // regroup_min_waves), read back at the drain so that they do not occupy
    // scalar registers through the main loop
    uint4* const drw0 = reinterpret_cast<uint4*>(smem + (size_t)nwaves * kSlots * rf +
                                                 (size_t)nwaves * kSlots * NT / 2 + (size_t)nwaves * kSlots / 4);
    uint4* drw = drw0 + (size_t)wv * 64;
    uint4* harg = drw0 + (size_t)nwaves * 64 + wv;

    for (int j = lane; j < kSlots * NT; j += 64) cnt[j] = 0ull;
    if (lane < kSlots) slot_item[lane] = -1;
    if constexpr (TAIL) {
        if (lane == 0) {
            const uint64_t hp = reinterpret_cast<uint64_t>(a.hand);
            *harg = make_uint4((uint32_t)hp, (uint32_t)(hp >> 32), a.hand_cap,
                               (uint32_t)a.regroup_lanes | ((uint32_t)a.regroup_min_waves << 8));
            if (a.regroup_lanes > 0)
                __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(a.hand) + kHandWaves, 1ull,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    wave_sync_lds();

    const uint64_t seed = a.seed_ptr ? *a.seed_ptr : a.seed;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t max_steps = a.max_steps;

    // lane state
    bool alive = false;
    int slot = 0, layer = 0;
    uint32_t item = 0, p_lo = 0, p_hi = 0, k = 0;
    float z = 0.f, uz = 1.f, s = 0.f;
    float wgt = 0.f, absd = 0.f;   // weighted form: packet weight, weight deposited so far
    LaneLayer P;
    P.mut = P.alb = P.inv_mut = P.thick = P.hG = P.hh = P.q1 = P.q2 = P.m_up = P.m_dn = P.n = 0.f;
    P.flags = 0u;

    // wave-uniform source chunk
    int src_slot = -1, src_item = -1;
    uint64_t src_next = 0, src_end = 0;
    bool queue_done = false;

    for (;;) {
        // ---------------- refill ----------------
        uint64_t dead = ballot64(!alive);
        while (dead != 0ull && (__popcll(dead) >= a.refill_min || dead == ~0ull)) {
            if (src_next >= src_end) {
                if (queue_done) break;
                const int ns = (src_slot + 1) % kSlots;
                if (ballot64(alive && slot == ns) != 0ull) {   // slot still draining
                    if constexpr (TAIL) {
                        // A wave whose oldest slot holds a long walk cannot
                        // claim, so it would not learn that the queue is
                        // empty until that walk ends: it looks at the queue
                        // itself, and enters the drain phase once it is.
                        int qd = 0;
                        if (lane == 0)
                            qd = __hip_atomic_load(a.chunk_counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                 a.chunk_prefix[a.n_items];
                        queue_done = __builtin_amdgcn_readfirstlane(qd) != 0;
                    }
                    break;
                }
                // claim the next global chunk; lane 0 finds its item by
                // binary search in the chunk prefix
                int c_item = -1;
                unsigned long long c_start = 0ull, c_end = 0ull;
                if (lane == 0) {
                    const unsigned long long kc = atomicAdd(a.chunk_counter, 1ull);
                    if (kc < a.chunk_prefix[a.n_items]) {
                        int lo = 0, hi = a.n_items;   // first j in [1, n] with prefix[j] > kc
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (a.chunk_prefix[mid] <= kc) lo = mid; else hi = mid;
                        }
                        const float4 h1 = a.table[(size_t)lo * rf + 1];
                        uint64_t N = (uint64_t)__float_as_uint(h1.x) | ((uint64_t)__float_as_uint(h1.y) << 32);
                        if (a.photon_cap && N > a.photon_cap) N = a.photon_cap;
                        c_item = lo;
                        c_start = (kc - a.chunk_prefix[lo]) * (unsigned long long)a.chunk;
                        c_end = (c_start + (uint64_t)a.chunk < N) ? c_start + (uint64_t)a.chunk : N;
                    }
                }
                c_item = __builtin_amdgcn_readfirstlane(c_item);
                c_start = uniform_u64(c_start);
                c_end = uniform_u64(c_end);
                if (c_item < 0) { queue_done = true; break; }
                if (c_item != src_item) {
                    // recycle slot ns: flush its counts, stage the new item
                    const int old = slot_item[ns];
                    if (old >= 0 && lane < NT) {
                        const unsigned long long v = cnt[ns * NT + lane];
                        if (v) atomicAdd(a.tallies + (size_t)old * NT + lane, v);
                    }
                    wave_sync_lds();
                    if (lane < NT) cnt[ns * NT + lane] = 0ull;
                    for (int j = lane; j < rf; j += 64) tab[ns * rf + j] = a.table[(size_t)c_item * rf + j];
                    if (lane == 0) slot_item[ns] = c_item;
                    wave_sync_lds();
                    src_slot = ns;
                    src_item = c_item;
                }
                src_next = c_start;
                src_end = c_end;
            }
            // hand photons of the source chunk to idle lanes
            const uint64_t avail = src_end - src_next;
            const int nd = __popcll(dead);
            const int take = (uint64_t)nd < avail ? nd : (int)avail;
            const int rank = lane_rank(dead);
            const bool mine = !alive && rank < take;
            bool spec = false;
            if (mine) {
                const uint64_t p = src_next + (uint64_t)rank;
                const float4* sr = tab + src_slot * rf;
                const float4 h0 = sr[0];
                p_lo = (uint32_t)p; p_hi = (uint32_t)(p >> 32);
                item = (uint32_t)src_item;
                bool enter;
                if constexpr (WEIGHTED) {
                    // the specular part leaves as weight, no draw
                    wgt = 1.0f - h0.x;
                    absd = 0.f;
                    enter = wgt > 0.f;
                } else {
                    const uint4 x = philox4x32_10(p_lo, p_hi, 0u, item, k0, k1);
                    enter = !(u24(x.y) < h0.x);
                    spec = !enter;                      // specular reflection
                }
                if (enter) {
                    alive = true;
                    slot = src_slot;
                    layer = 0;
                    z = 0.f; uz = h0.y; s = 0.f; k = 0u;
                    load_layer(sr, 0, P);
                }
            }
            if constexpr (WEIGHTED) {
                if (take > 0 && lane == 0) {
                    atomicAdd(cnt + src_slot * NT + kWRSpec,
                              (unsigned long long)take * weight_units((double)tab[src_slot * rf].x));
                    atomicAdd(cnt + src_slot * NT + kWPhotons, (unsigned long long)take);
                }
            } else {
                const uint64_t sm = ballot64(spec);
                if (sm != 0ull && lane == 0)
                    atomicAdd(cnt + src_slot * NT + kRSpec, (unsigned long long)__popcll(sm));
            }
            src_next += (uint64_t)take;
            dead = ballot64(!alive);
        }
        if (dead == ~0ull) break;   // queue exhausted and nothing in flight
        if constexpr (TAIL) {
            if (queue_done && src_next >= src_end) break;   // nothing left to claim: drain phase
        }

        // ---------------- walk ----------------

        for (int it = 0; it < kStepsPerCheck; ++it) {
            const bool go = alive && k < max_steps;
            int term = (alive && !go) ? (int)kCap : -1;        // step budget used up
            if (go) {
                ++k;
                FOS_WALK_STEP(philox4x32_10(p_lo, p_hi, k, item, k0, k1), tab + slot * rf);
            }
            // ---- tallies of photons that finished in this step ----
            const uint64_t tm = ballot64(term >= 0);
            if (tm != 0ull) {
                if constexpr (WEIGHTED) {
                    // per-lane: the packet's deposits, its exit weight, the counts
                    if (term >= 0) {
                        alive = false;
                        unsigned long long* c0 = cnt + slot * NT;
                        atomicAdd(c0 + kWSteps, (unsigned long long)k);
                        const double ad = (double)absd;
                        if (ad > 0.0) {
                            atomicAdd(c0 + kWAbs, weight_units(ad));
                            atomicAdd(c0 + kWAbs2, weight_units(ad * ad));
                        }
                        if (term == kTrans || term == kRDiff) {
                            const double w = (double)wgt;
                            atomicAdd(c0 + (term == kTrans ? kWTrans : kWRDiff), weight_units(w));
                            atomicAdd(c0 + (term == kTrans ? kWTrans2 : kWRDiff2), weight_units(w * w));
                        } else if (term == kWRoulette) {
                            atomicAdd(c0 + kWRoulette, 1ull);
                        } else if (term == kCap) {
                            atomicAdd(c0 + kWCap, 1ull);
                        }
                    }
                } else {
                    // one LDS add per finishing lane and counter: about one
                    // photon ends per wave-step, and per-outcome ballots cost
                    // more scalar and vector issue than the adds they save
                    if (term >= 0) {
                        alive = false;
                        unsigned long long* c0 = cnt + slot * NT;
                        atomicAdd(c0 + kSteps, (unsigned long long)k);
                        atomicAdd(c0 + term, 1ull);
                    }
                }
                if (__popcll(ballot64(!alive)) >= a.refill_min) break;
            }
        }
    }

    // exit (or, in the tail build, the start of the drain phase): flush
    // every slot of this wave
    wave_sync_lds();
    for (int sl = 0; sl < kSlots; ++sl) {
        const int it = slot_item[sl];
        if (it >= 0 && lane < NT) {
            const unsigned long long v = cnt[sl * NT + lane];
            if (v) atomicAdd(a.tallies + (size_t)it * NT + lane, v);
        }
    }

    if constexpr (TAIL) {
        // ---------------- drain: nothing left to claim ----------------
        // The slots are flushed: from here on a lane reads its item's record
        // from the item table and a finishing photon adds to its item's
        // tallies in HBM, so photons can move between waves.
        //
        // Regrouping (regroup_lanes > 0).  A wave left with at most
        // regroup_lanes photons writes their whole state (item, photon,
        // step, depth, direction, remaining free path, layer, and the
        // packet's weights) to the hand-off list and leaves, freeing its
        // slot on the SIMD; waves with idle lanes take listed photons over.
        // A photon's draws depend only on (photon, step, item, seed), so it
        // continues with the same draws and decisions wherever it runs: the
        // tallies are the same bits.  A wave hands off at most once, and
        // only while more than regroup_min_waves waves are alive and the
        // list holds fewer than 64 untaken photons, so the list stays
        // within hand_cap = waves x regroup_lanes and is taken up promptly.
        // Every wave leaves through wave_leave(): the wave whose leaving
        // takes the count of live waves to zero takes whatever is still
        // listed, so no photon is left behind.
        //
        // Tail phase (tail_lanes > 0): a wave with at most tail_lanes
        // photons in flight lets its idle lanes compute their next draws.
        // With nl photons in flight each gets B = 64 / 2^ceil(log2 nl)
        // consecutive Philox blocks, one per lane, in the wave's LDS buffer,
        // and its lane reads the block of each step there instead of running
        // the ten dependent rounds.  The draws are the same bits.
        constexpr int RW = WEIGHTED ? 3 : 2;   // float4 per hand-off record
        const uint4 hv = *harg;
        unsigned char* const hbase =
            reinterpret_cast<unsigned char*>(uniform_u64(((uint64_t)hv.y << 32) | (uint64_t)hv.x));
        const uint32_t hand_cap = (uint32_t)__builtin_amdgcn_readfirstlane((int)hv.z);
        const uint32_t hw = (uint32_t)__builtin_amdgcn_readfirstlane((int)hv.w);
        const bool regroup = (hw & 0xFFu) != 0u;
        unsigned long long* const ctl = reinterpret_cast<unsigned long long*>(hbase);
        // wstate: bits 0-7, drain rounds before the next look at an empty
        // list (doubling from kAbsorbEvery up to kAbsorbMax while it stays
        // empty); bits 8-15, the current wait; bits 16-23, rounds before the
        // next hand-off attempt; kHanded: this wave has handed off (never
        // twice) or found the live-wave count at or below the floor (it only
        // falls) -- either way it does not try again.
        constexpr int kHanded = 1 << 24;
        int wstate = 0;
        for (;;) {
            uint64_t dead = ballot64(!alive);
            // ---- take over listed photons into idle lanes ----
            if (regroup && dead != 0ull && (dead == ~0ull || __popcll(dead) >= a.refill_min)) {
                if ((wstate & 0xFF) > 0 && dead != ~0ull) {
                    --wstate;
                } else {
                    int take = 0;
                    unsigned long long hb = 0ull;
                    if (lane == 0) {
                        unsigned long long h = hand_load(ctl + kHandClaimed);
                        for (int t = 0; t < 4; ++t) {
                            const unsigned long long r = hand_load(ctl + kHandReserved);
                            if (r <= h) break;
                            const unsigned long long want = (unsigned long long)__popcll(dead);
                            const unsigned long long n = r - h < want ? r - h : want;
                            if (__hip_atomic_compare_exchange_strong(ctl + kHandClaimed, &h, h + n, __ATOMIC_RELAXED,
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                take = (int)n;
                                hb = h;
                                break;
                            }
                        }
                    }
                    take = __builtin_amdgcn_readfirstlane(take);
                    hb = uniform_u64(hb);
                    if (take == 0) {
                        // list empty: wait twice as long as last time
                        int w = (wstate >> 8) & 0xFF;
                        w = w == 0 ? kAbsorbEvery : (2 * w > kAbsorbMax ? kAbsorbMax : 2 * w);
                        wstate = (wstate & ~0xFFFF) | (w << 8) | w;
                    } else {
                        wstate &= ~0xFFFF;
                        const int rank = lane_rank(dead);
                        const bool mine = !alive && rank < take;
                        const unsigned long long j = hb + (unsigned long long)rank;
                        // each record's writer sets its flag right after reserving it
                        bool ready = !mine;
                        for (int sp = 0; sp < kHandSpins; ++sp) {
                            if (!ready)
                                ready = __hip_atomic_load(
                                            reinterpret_cast<unsigned int*>(hbase + hand_flags_offset()) + j,
                                            __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u;
                            if (ballot64(!ready) == 0ull) break;
                            __builtin_amdgcn_s_sleep(2);
                        }
                        if (mine) {
                            if (ready) {
                                const float4* hr =
                                    reinterpret_cast<const float4*>(hbase + hand_records_offset(hand_cap)) + j * RW;
                                const float4 r0 = hr[0], r1 = hr[1];
                                item = __float_as_uint(r0.x);
                                p_lo = __float_as_uint(r0.y);
                                p_hi = __float_as_uint(r0.z);
                                k = __float_as_uint(r0.w);
                                z = r1.x;
                                uz = r1.y;
                                s = r1.z;
                                layer = __float_as_int(r1.w);
                                if constexpr (WEIGHTED) {
                                    const float4 r2 = hr[2];
                                    wgt = r2.x;
                                    absd = r2.y;
                                }
                                load_layer(a.table + (size_t)item * rf, layer, P);
                                alive = true;
                            } else {
                                atomicAdd(ctl + kHandLost, 1ull);
                            }
                        }
                        dead = ballot64(!alive);
                    }
                }
            }
            if (dead == ~0ull) {           // nothing in flight
                if (!regroup || wave_leave(ctl, lane)) break;
                continue;
            }
            const int nl = 64 - __popcll(dead);
            // ---- hand the few photons in flight to other waves and leave ----
            if (regroup && !(wstate & kHanded) && (uint32_t)nl <= (hw & 0xFFu) && (wstate & 0xFF0000) == 0) {
                // give: 1 handed off, 0 try again later, -1 never (too few waves alive)
                int give = 0;
                unsigned long long gb = 0ull;
                if (lane == 0) {
                    const unsigned long long aw = hand_load(ctl + kHandWaves);
                    if (aw <= (unsigned long long)(hw >> 8)) {
                        give = -1;
                    } else {
                        unsigned long long r = hand_load(ctl + kHandReserved);
                        const unsigned long long h = hand_load(ctl + kHandClaimed);
                        if (r - h < 64ull && r + (unsigned long long)nl <= (unsigned long long)hand_cap &&
                            __hip_atomic_compare_exchange_strong(ctl + kHandReserved, &r, r + (unsigned long long)nl,
                                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT)) {
                            give = 1;
                            gb = r;
                        }
                    }
                }
                give = __builtin_amdgcn_readfirstlane(give);
                if (give < 0) wstate |= kHanded;
                if (give == 0) wstate |= kHandRetry << 16;
                if (give > 0) {
                    gb = uniform_u64(gb);
                    if (alive) {
                        const unsigned long long j = gb + (unsigned long long)lane_rank(~dead);
                        float4* hr = reinterpret_cast<float4*>(hbase + hand_records_offset(hand_cap)) + j * RW;
                        hr[0] = make_float4(__uint_as_float(item), __uint_as_float(p_lo), __uint_as_float(p_hi),
                                            __uint_as_float(k));
                        hr[1] = make_float4(z, uz, s, __int_as_float(layer));
                        if constexpr (WEIGHTED) hr[2] = make_float4(wgt, absd, 0.f, 0.f);
                        __hip_atomic_store(reinterpret_cast<unsigned int*>(hbase + hand_flags_offset()) + j, 1u,
                                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        alive = false;
                    }
                    wstate |= kHanded;
                    if (wave_leave(ctl, lane)) break;
                    continue;
                }
            } else if ((wstate & 0xFF0000) != 0) {
                wstate -= 1 << 16;
            }
            if (nl <= a.tail_lanes) {
                // ---- tail phase: steps on prepared draws ----
                const uint64_t live = ballot64(alive && k < max_steps);
                const int nlive = __popcll(live);
                int lg = 0;
                while ((1 << lg) < nlive) ++lg;
                const int B = 64 >> lg;
                {
                    // this lane prepares draw o of the q-th photon in flight
                    const int q = lane >> (6 - lg);
                    const int o = lane & (B - 1);
                    uint64_t m = live;
                    for (int t = 0; t < q && m; ++t) m &= m - 1;
                    const int src = m ? (int)__builtin_ctzll(m) : 0;
                    const uint32_t sp_lo = __shfl(p_lo, src), sp_hi = __shfl(p_hi, src);
                    const uint32_t s_k = __shfl(k, src), s_item = __shfl(item, src);
                    drw[lane] = philox4x32_10(sp_lo, sp_hi, s_k + 1u + (uint32_t)o, s_item, k0, k1);
                }
                wave_sync_lds();
                const int base = (alive && k < max_steps) ? (lane_rank(live) << (6 - lg)) : 0;
                for (int j = 0; j < B; ++j) {
                    const bool go = alive && k < max_steps;
                    int term = (alive && !go) ? (int)kCap : -1;
                    if (go) {
                        ++k;
                        FOS_WALK_STEP(drw[base + j], a.table + (size_t)item * rf);
                    }
                    if (term >= 0) {
                        alive = false;
                        finish_photon<WEIGHTED>(a.tallies + (size_t)item * NT, term, k, wgt, absd);
                    }
                    if (ballot64(alive) == 0ull) break;
                }
                wave_sync_lds();
                continue;
            }
            for (int it = 0; it < kStepsPerCheck; ++it) {
                const bool go = alive && k < max_steps;
                int term = (alive && !go) ? (int)kCap : -1;
                if (go) {
                    ++k;
                    FOS_WALK_STEP(philox4x32_10(p_lo, p_hi, k, item, k0, k1), a.table + (size_t)item * rf);
                }
                if (term >= 0) {
                    alive = false;
                    finish_photon<WEIGHTED>(a.tallies + (size_t)item * NT, term, k, wgt, absd);
                }
            }
        }
    }
}

template <int kStepsPerCheck, bool WEIGHTED, bool SINGLE>
__global__ void walk(WalkArgs a)
{
    walk_body<kStepsPerCheck, WEIGHTED, SINGLE, false>(a);
}

// The drain phase lifts the tail build's scalar registers just past what 8
// waves per SIMD allow (103 of 102 for the analog one-layer build); capped at
// 102, the allocator spills one scalar (the LDS address of the drain's
// buffers) to a vector lane outside both loops and the build keeps 8 waves.
template <int kStepsPerCheck, bool WEIGHTED, bool SINGLE>
__global__ __attribute__((amdgpu_num_sgpr(102))) void walk_long(WalkArgs a)
{
    walk_body<kStepsPerCheck, WEIGHTED, SINGLE, true>(a);
}

size_t walk_lds_bytes(int block_size, int max_layers, bool weighted, bool tail)
{
    const int nw = block_size / 64;
    const int nt = weighted ? kNTallyW : kNTally;
    return (size_t)nw * kSlots * rec_f4(max_layers) * sizeof(float4) +
           (size_t)nw * kSlots * nt * sizeof(unsigned long long) + (size_t)nw * kSlots * sizeof(int) +
           (tail ? (size_t)nw * 65 * sizeof(uint4) : 0);
}

hipError_t launch_reset_handoff(const WalkArgs& a, hipStream_t st)
{
    if (a.regroup_lanes <= 0) return hipSuccess;
    uint64_t blocks = ((uint64_t)a.hand_cap + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(reset_handoff, dim3((unsigned)blocks), dim3(256), 0, st, a.hand, (uint64_t)a.hand_cap);
    return hipGetLastError();
}

hipError_t launch_walk(const WalkArgs& a, int grid, int block, hipStream_t st, bool weighted)
{
    const bool tail = a.tail_lanes > 0 || a.regroup_lanes > 0;
    const size_t lds = walk_lds_bytes(block, a.max_layers, weighted, tail);
    const bool single = a.max_layers == 1;
    if (tail) {
        if (weighted && single)
            hipLaunchKernelGGL((walk_long<16, true, true>), dim3(grid), dim3(block), lds, st, a);
        else if (weighted)
            hipLaunchKernelGGL((walk_long<16, true, false>), dim3(grid), dim3(block), lds, st, a);
        else if (single)
            hipLaunchKernelGGL((walk_long<16, false, true>), dim3(grid), dim3(block), lds, st, a);
        else
            hipLaunchKernelGGL((walk_long<16, false, false>), dim3(grid), dim3(block), lds, st, a);
    } else if (weighted && single)
        hipLaunchKernelGGL((walk<16, true, true>), dim3(grid), dim3(block), lds, st, a);
    else if (weighted)
        hipLaunchKernelGGL((walk<16, true, false>), dim3(grid), dim3(block), lds, st, a);
    else if (single)
        hipLaunchKernelGGL((walk<16, false, true>), dim3(grid), dim3(block), lds, st, a);
    else
        hipLaunchKernelGGL((walk<16, false, false>), dim3(grid), dim3(block), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t st)
{
    if (a.n_items <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(pack_items, dim3((a.n_items + b - 1) / b), dim3(b), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* tallies, unsigned long long* counter, int n_items, int nt,
                        hipStream_t st)
{
    int blocks = (int)(((size_t)n_items * nt + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(reset_run, dim3(blocks), dim3(256), 0, st, tallies, counter, n_items, nt);
    return hipGetLastError();
}

hipError_t launch_chunk_scan(const float4* table, int rec_f4, int n_items, int chunk, uint64_t photon_cap,
                             unsigned long long* prefix, hipStream_t st)
{
    hipLaunchKernelGGL(chunk_scan, dim3(1), dim3(1024), 0, st, table, rec_f4, n_items, chunk, photon_cap, prefix);
    return hipGetLastError();
}

__global__ void fill_u64(unsigned long long* p, unsigned long long v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t st)
{
    hipLaunchKernelGGL(fill_u64, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// (R, A, T) fractions of every item from its tallies: R = (specular +
// diffuse)/N, A/N, T/N with N the item's photons
__global__ void fractions_k(int n, const unsigned long long* t, float* rat)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long* ti = t + (size_t)i * kNTally;
    const double N = (double)(ti[0] + ti[1] + ti[2] + ti[3] + ti[4]);
    if (N == 0.0) {
        rat[3 * (size_t)i + 0] = rat[3 * (size_t)i + 1] = rat[3 * (size_t)i + 2] = 0.0f;
        return;
    }
    rat[3 * (size_t)i + 0] = (float)((double)(ti[0] + ti[1]) / N);
    rat[3 * (size_t)i + 1] = (float)((double)ti[2] / N);
    rat[3 * (size_t)i + 2] = (float)((double)ti[3] / N);
}

// weighted tallies -> (R, A, T) means and the standard errors of their
// estimates (the specular part is exact, so R's error is the diffuse part's)
__global__ void weighted_fractions_k(int n, const unsigned long long* t, float* rat, float* se)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long* ti = t + (size_t)i * kNTallyW;
    const double N = (double)ti[kWPhotons];
    float* r = rat + 3 * (size_t)i;
    float* e = se ? se + 3 * (size_t)i : nullptr;
    if (N == 0.0) {
        r[0] = r[1] = r[2] = 0.0f;
        if (e) e[0] = e[1] = e[2] = 0.0f;
        return;
    }
    const double u = 1.0 / kWeightUnit;
    const double mean_rd = (double)ti[kWRDiff] * u / N, mean_a = (double)ti[kWAbs] * u / N;
    const double mean_t = (double)ti[kWTrans] * u / N;
    r[0] = (float)((double)ti[kWRSpec] * u / N + mean_rd);
    r[1] = (float)mean_a;
    r[2] = (float)mean_t;
    if (e) {
        const double m2[3] = {(double)ti[kWRDiff2] * u / N, (double)ti[kWAbs2] * u / N, (double)ti[kWTrans2] * u / N};
        const double m1[3] = {mean_rd, mean_a, mean_t};
        for (int c = 0; c < 3; ++c) e[c] = (float)sqrt(fmax(m2[c] - m1[c] * m1[c], 0.0) / N);
    }
}

hipError_t launch_weighted_fractions(int n, const unsigned long long* tallies, float* rat, float* se, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(weighted_fractions_k, dim3((n + 255) / 256), dim3(256), 0, st, n, tallies, rat, se);
    return hipGetLastError();
}

hipError_t launch_fractions(int n, const unsigned long long* tallies, float* rat, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fractions_k, dim3((n + 255) / 256), dim3(256), 0, st, n, tallies, rat);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// test hooks
// ---------------------------------------------------------------------------
__global__ void philox_words_k(int n, const uint64_t* photon, const uint32_t* step, const uint32_t* stream,
                               uint64_t seed, uint32_t* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint64_t p = photon[j];
    const uint4 x = philox4x32_10((uint32_t)p, (uint32_t)(p >> 32), step[j], stream[j], (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    out[4 * j + 0] = x.x; out[4 * j + 1] = x.y; out[4 * j + 2] = x.z; out[4 * j + 3] = x.w;
}

hipError_t launch_philox_words(int n, const uint64_t* photon, const uint32_t* step, const uint32_t* stream,
                               uint64_t seed, uint32_t* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_words_k, dim3((n + 255) / 256), dim3(256), 0, st, n, photon, step, stream, seed, out);
    return hipGetLastError();
}

// Fresnel exactly as the walk evaluates it: real interfaces by ratio
// m = ni/nt (total internal reflection -> 1), complex lower media by the
// impedance form.
__global__ void eval_fresnel_k(int n, const float* c, const float* ni, const float* nt, const float* kt,
                               float* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float aa = c[j];
    float R;
    if (kt[j] > 0.f) {
        R = fresnel_complex(aa, ni[j], nt[j], kt[j]);
    } else if (ni[j] == nt[j]) {
        R = 0.f;
    } else {
        const float m = ni[j] / nt[j];
        const float s2t = m * m * (1.f - aa * aa);
        R = s2t >= 1.f ? 1.f : fresnel_real(aa, fast_sqrt(1.f - s2t), m);
    }
    out[j] = R;
}

hipError_t launch_eval_fresnel(int n, const float* c, const float* ni, const float* nt, const float* kt,
                               float* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_fresnel_k, dim3((n + 255) / 256), dim3(256), 0, st, n, c, ni, nt, kt, out);
    return hipGetLastError();
}

__global__ void eval_hg_k(int n, const float* g, const float* u01, float* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float G, h, q1, q2;
    bool mirror;
    hg_constants((double)g[j], G, h, q1, q2, mirror);
    out[j] = hg_cos(G, h, q1, q2, mirror, u01[j]);
}

hipError_t launch_eval_hg(int n, const float* g, const float* u01, float* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_hg_k, dim3((n + 255) / 256), dim3(256), 0, st, n, g, u01, out);
    return hipGetLastError();
}

}  // namespace fos
