// fos_device.hpp -- device-side building blocks of the gfx950 photon walk:
// the Philox4x32-10 counter generator, 24-bit uniforms, Fresnel
// reflectance and the Henyey-Greenstein sampler, plus the packed item-table
// layout shared by the pack kernel and the walk kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fos {

// ---------------------------------------------------------------------------
// Packed item table (float4 records, one per item, stride rec_f4(max_layers)):
//   hdr0 = (R0, uz0, n_lower, k_lower)        entry reflectance, refracted cosine
//   hdr1 = (photons lo, photons hi, n_layers, item)   (bit patterns)
//   per layer l, 4 float4 at 2 + 4 l:
//   L0 = (mu_t, albedo, 1/mu_t, thickness)
//   L1 = (hg_G, hg_h, hg_q1, hg_q2)   Henyey-Greenstein constants (hg_cos)
//   L2 = (m_up, m_dn, n_layer, flags)  m = n_layer / n_neighbour; flags bits
//   L3 = reserved
// ---------------------------------------------------------------------------
constexpr int kHdrF4 = 2;
constexpr int kLayerF4 = 4;
__host__ __device__ constexpr int rec_f4(int max_layers) { return kHdrF4 + kLayerF4 * max_layers; }

enum LayerFlags : uint32_t {
    kExitUp = 1u,      // top face of this layer is the top of the stack
    kExitDn = 2u,      // bottom face is the bottom of the stack
    kMatchUp = 4u,     // index-matched across the top face
    kMatchDn = 8u,     // index-matched across the bottom face
    kComplexDn = 16u,  // lower medium is absorbing (k > 0): complex Fresnel
    kHgMirror = 32u,   // Henyey-Greenstein sample is mirrored (see hg_cos)
};

enum Outcome : int { kRSpec = 0, kRDiff = 1, kAbs = 2, kTrans = 3, kCap = 4, kSteps = 5, kNTally = 6 };
// weighted-packet tallies: weights in units of 2^-36 (exact integer sums, so
// results do not depend on the order photons finish in), photon counts, steps
enum WOutcome : int {
    kWRSpec = 0, kWRDiff = 1, kWAbs = 2, kWTrans = 3, kWRDiff2 = 4, kWAbs2 = 5, kWTrans2 = 6,
    kWRoulette = 7, kWCap = 8, kWSteps = 9, kWPhotons = 10, kNTallyW = 11
};
constexpr double kWeightUnit = 68719476736.0;   // 2^36
constexpr float kRouletteThreshold = 1e-4f;       // packets below this weight play roulette
constexpr float kRouletteChance = 0.1f;           // and survive with this probability

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// on counter words 0 and 2 (multipliers 0xD2511F53, 0xCD9E8D57); the high
// halves are xor-ed with the other words and the round key, the low halves
// move over; the key advances by (0x9E3779B9, 0xBB67AE85) between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// uniform in [0,1) from the top 24 bits of a word (exact in FP32)
__device__ __forceinline__ float u24(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// Hardware approximations (about 1 ulp) used on the walk's hot path; their
// error is far below the binomial noise of any tally.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// -ln(xi) for xi in [2^-24, 1] via the base-2 logarithm instruction
__device__ __forceinline__ float neg_ln(float xi) { return -0.693147180559945309f * __builtin_amdgcn_logf(xi); }

// ---------------------------------------------------------------------------
// Fresnel reflectance, unpolarised.
// Real interface, m = n_i / n_t, c = |cos theta_i|, ct = cos theta_t:
//   r_s = (m c - ct)/(m c + ct),  r_p = (c - m ct)/(c + m ct).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fresnel_real(float c, float ct, float m)
{
    const float a1 = m * c - ct, d1 = m * c + ct;
    const float a2 = c - m * ct, d2 = c + m * ct;
    const float num = a1 * a1 * (d2 * d2) + a2 * a2 * (d1 * d1);
    const float den = (d1 * d1) * (d2 * d2);
    return 0.5f * num * fast_rcp(den);
}

// Absorbing lower medium N = n + i k seen from real index ni at cosine c:
// q = N cos(theta_t) = sqrt(N^2 - ni^2 (1 - c^2)) (principal root),
//   r_s = (ni c - q)/(ni c + q),  r_p = (N^2 c - ni q)/(N^2 c + ni q).
__device__ __forceinline__ float fresnel_complex(float c, float ni, float n, float k)
{
    const float A2 = n * n - k * k;         // Re N^2
    const float B = 2.0f * n * k;           // Im N^2 >= 0
    const float A = A2 - ni * ni * (1.0f - c * c);
    const float mod = fast_sqrt(A * A + B * B);
    float qr, qi;
    if (A >= 0.0f) {
        qr = fast_sqrt(0.5f * (mod + A));
        qi = (qr > 0.0f) ? 0.5f * B * fast_rcp(qr) : 0.0f;
    } else {
        qi = fast_sqrt(0.5f * (mod - A));
        qr = (qi > 0.0f) ? 0.5f * B * fast_rcp(qi) : 0.0f;
    }
    const float nc = ni * c;
    const float rs2 = ((nc - qr) * (nc - qr) + qi * qi) * fast_rcp((nc + qr) * (nc + qr) + qi * qi);
    const float pr = A2 * c, pi = B * c;
    const float sr = ni * qr, si = ni * qi;
    const float rp2 = ((pr - sr) * (pr - sr) + (pi - si) * (pi - si)) *
                      fast_rcp((pr + sr) * (pr + sr) + (pi + si) * (pi + si));
    return fminf(0.5f * (rs2 + rp2), 1.0f);
}

// ---------------------------------------------------------------------------
// Henyey-Greenstein polar cosine.  With G = |g|, h = 1 - G and the uniform
// measured from the backward end, e = 2U for g >= 0 (2(1 - U) for g < 0,
// whose sample is then mirrored), the inverse CDF
//   cos = (1 + G^2 - ((1 - G^2)/(1 - G + G e))^2) / (2G)
// rearranges to
//   cos = (-h^2 + q1 e + q2 e^2) / (h + G e)^2,  q1 = (1 + G^2) h,
//                                               q2 = G (1 + G^2) / 2,
// which has no division by g (exact isotropic limit cos = e - 1 at G = 0)
// and no cancellation near backscatter for G -> 1.  |g| = 1 (a delta) is
// stored as G = 0, h = 1, q1 = q2 = 0 with the mirror flag set for g = +1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float hg_cos(float G, float h, float q1, float q2, bool mirror, float U)
{
    const float e = 2.0f * (mirror ? 1.0f - U : U);
    const float t = fmaf(G, e, h);
    const float num = fmaf(fmaf(q2, e, q1), e, -h * h);
    float c = num * fast_rcp(t * t);
    c = mirror ? -c : c;
    return fminf(fmaxf(c, -1.0f), 1.0f);
}

// Per-layer HG constants (G, h, q1, q2) and the mirror flag, in double.
__host__ __device__ inline void hg_constants(double g, float& G, float& h, float& q1, float& q2, bool& mirror)
{
    if (g >= 1.0 || g <= -1.0) {
        G = 0.0f; h = 1.0f; q1 = 0.0f; q2 = 0.0f;
        mirror = g > 0.0;
        return;
    }
    const double a = g < 0.0 ? -g : g;
    const double hh = 1.0 - a;
    G = (float)a;
    h = (float)hh;
    q1 = (float)((1.0 + a * a) * hh);
    q2 = (float)(0.5 * a * (1.0 + a * a));
    mirror = g < 0.0;
}

}  // namespace fos
