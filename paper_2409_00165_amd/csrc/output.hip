// output.hip -- the output stage: what a finished spectrum turns into.
//   * Eq. (21): the solar-weighted totals R_s, A_s, T_s -- the spectral value
//     times the solar irradiation G integrated over the simulated range, over
//     the integral of G.  Computed when a solar spectrum is given and the
//     simulated range covers 0.28 - 2.5 um (Output section).
//   * The emittance of a band (the sky window of the Introduction): by
//     Kirchhoff's law the absorptance, weighted by a blackbody spectrum over
//     the grid points inside the band.
//   * The colour of the reflectance (the painted bilayer of Results; the
//     paper leaves the method open): CIE 1931 XYZ under an illuminant, with
//     the colour-matching functions from the multi-lobe analytic fit of
//     Wyman, Sloan and Shirley (JCGT 2013); CIE 1976 L*a*b* against the
//     illuminant's white; sRGB (IEC 61966-2-1) after a Bradford adaptation of
//     that white to D65, linear values clipped to [0, 1].
// Spectra given as samples are linear between samples and zero outside them
// (the paper interpolates every input file linearly onto the simulated grid,
// Input section); integrals are trapezoid sums over the grid.
//
// Everything before the colour transforms is linear in the spectrum, so the
// stage splits in two.  fos_output_prepare turns the grid and the spectra
// into five rows of quadrature weights once (one workgroup, FP64: sampling,
// trapezoid widths, Planck's law, the fit, the normalising integrals and the
// 3 x 3 colour matrix).  fos_output_run then reads each design's spectrum
// exactly once and reduces it against the weights: one wave per design, each
// lane a strided set of wavelengths (12-byte R, A, T records, so a wave's
// loads cover 768 contiguous bytes), a butterfly over the wave, and the
// colour transforms in the epilogue.  The run is bound by HBM reads of the
// spectra.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>
#include <string>

#include "fos_ctx.hpp"

namespace fos {

namespace {

constexpr int kPrepThreads = 256;
constexpr int kRows = 5;            // weight rows: solar, band, x, y, z
constexpr int kOutParams = 12;      // white X, Y, Z; XYZ -> linear sRGB, 3 x 3 row-major
constexpr int kMaxGrid = 1 << 20;   // wavelengths of one grid, samples of one spectrum
constexpr double kC2 = 14387.769;   // second radiation constant hc/k, um K

struct PrepArgs {
    int L;
    const float* lam;                    // [L]
    int ns; const float* s_um; const float* s_val;   // solar spectrum (ns = 0: none)
    int ni; const float* i_um; const float* i_val;   // illuminant (ni = 0: equal energy)
    float band_lo, band_hi, band_t;
    int avail;                           // FOS_OUTPUT_* bits
    float* w;                            // [kRows][L]
    float* params;                       // [kOutParams]
};

struct RunArgs {
    int64_t designs;
    int L;
    const float* rat;                    // [designs][L][3]
    const float* w;                      // [kRows][L]
    const float* params;                 // [kOutParams]
    float* totals;                       // [designs][4]
    float* colour;                       // [designs][9] or null
    int avail;
};

// value of a sampled spectrum at x: linear between samples, zero outside
__device__ double sample_at(int n, const float* um, const float* val, double x)
{
    if (x < (double)um[0] || x > (double)um[n - 1]) return 0.0;
    int lo = 0, hi = n - 1;                  // um[lo] <= x <= um[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((double)um[mid] <= x) lo = mid; else hi = mid;
    }
    const double t = (x - (double)um[lo]) / ((double)um[hi] - (double)um[lo]);
    return (double)val[lo] + t * ((double)val[hi] - (double)val[lo]);
}

// one lobe of the colour-matching fit: a Gaussian of width s1 below its
// centre and s2 above it (nm)
__device__ double lobe(double nm, double centre, double s1, double s2)
{
    const double t = (nm - centre) / (nm < centre ? s1 : s2);
    return exp(-0.5 * t * t);
}

__device__ void colour_matching(double um, double& x, double& y, double& z)
{
    const double nm = 1000.0 * um;
    x = 1.056 * lobe(nm, 599.8, 37.9, 31.0) + 0.362 * lobe(nm, 442.0, 16.0, 26.7) -
        0.065 * lobe(nm, 501.1, 20.4, 26.2);
    y = 0.821 * lobe(nm, 568.8, 46.9, 40.5) + 0.286 * lobe(nm, 530.9, 16.3, 31.1);
    z = 1.217 * lobe(nm, 437.0, 11.8, 36.0) + 0.681 * lobe(nm, 459.0, 26.0, 13.8);
}

__device__ bool in_band(const PrepArgs& a, float v) { return v >= a.band_lo && v <= a.band_hi; }

// unnormalised weights of grid point l: spectrum value x trapezoid width
__device__ void point_weights(const PrepArgs& a, int l, double (&v)[kRows])
{
    const double x = a.lam[l];
    const double left = a.lam[l > 0 ? l - 1 : l], right = a.lam[l + 1 < a.L ? l + 1 : l];
    const double width = 0.5 * (right - left);
    v[0] = a.ns > 0 ? sample_at(a.ns, a.s_um, a.s_val, x) * width : 0.0;
    v[1] = 0.0;
    if (a.band_t > 0.0f && in_band(a, a.lam[l])) {
        // the trapezoid rule on the part of the grid inside the band
        const double bl = (l > 0 && in_band(a, a.lam[l - 1])) ? (double)a.lam[l - 1] : x;
        const double br = (l + 1 < a.L && in_band(a, a.lam[l + 1])) ? (double)a.lam[l + 1] : x;
        const double planck = 1.0 / (x * x * x * x * x * expm1(kC2 / (x * (double)a.band_t)));
        v[1] = planck * 0.5 * (br - bl);
    }
    const double s = a.ni > 0 ? sample_at(a.ni, a.i_um, a.i_val, x) : 1.0;
    double cx, cy, cz;
    colour_matching(x, cx, cy, cz);
    v[2] = s * cx * width;
    v[3] = s * cy * width;
    v[4] = s * cz * width;
}

__device__ void invert3(const double (&m)[9], double (&r)[9])
{
    const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    const double id = 1.0 / det;
    r[0] = c00 * id; r[1] = (m[2] * m[7] - m[1] * m[8]) * id; r[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    r[3] = c01 * id; r[4] = (m[0] * m[8] - m[2] * m[6]) * id; r[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    r[6] = c02 * id; r[7] = (m[1] * m[6] - m[0] * m[7]) * id; r[8] = (m[0] * m[4] - m[1] * m[3]) * id;
}

__device__ void matmul3(const double (&a)[9], const double (&b)[9], double (&r)[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// XYZ -> linear sRGB for colours seen under `white`: the Bradford cone
// responses of the colour are scaled by D65's over the white's, then the
// IEC 61966-2-1 matrix
__device__ void srgb_matrix(const double (&white)[3], double (&m)[9])
{
    const double brad[9] = {0.8951, 0.2664, -0.1614, -0.7502, 1.7135, 0.0367, 0.0389, -0.0685, 1.0296};
    const double srgb[9] = {3.2406, -1.5372, -0.4986, -0.9689, 1.8758, 0.0415, 0.0557, -0.2040, 1.0570};
    const double d65[3] = {0.3127 / 0.3290, 1.0, (1.0 - 0.3127 - 0.3290) / 0.3290};
    double scaled[9], inv[9], adapt[9];
    for (int i = 0; i < 3; ++i) {
        const double src = brad[3 * i] * white[0] + brad[3 * i + 1] * white[1] + brad[3 * i + 2] * white[2];
        const double dst = brad[3 * i] * d65[0] + brad[3 * i + 1] * d65[1] + brad[3 * i + 2] * d65[2];
        for (int j = 0; j < 3; ++j) scaled[3 * i + j] = brad[3 * i + j] * (dst / src);
    }
    invert3(brad, inv);
    matmul3(inv, scaled, adapt);
    matmul3(srgb, adapt, m);
}

__global__ __launch_bounds__(kPrepThreads) void output_prepare_kernel(PrepArgs a)
{
    __shared__ double part[kRows][kPrepThreads];
    const int tid = threadIdx.x;
    double sum[kRows] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = tid; l < a.L; l += kPrepThreads) {
        double v[kRows];
        point_weights(a, l, v);
        for (int k = 0; k < kRows; ++k) sum[k] += v[k];
    }
    for (int k = 0; k < kRows; ++k) part[k][tid] = sum[k];
    __syncthreads();
    for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int k = 0; k < kRows; ++k) part[k][tid] += part[k][tid + h];
        __syncthreads();
    }
    const double solar = part[0][0], band = part[1][0], ny = part[3][0];
    const bool has_solar = (a.avail & FOS_OUTPUT_SOLAR) != 0, has_band = (a.avail & FOS_OUTPUT_BAND) != 0;
    const bool has_colour = (a.avail & FOS_OUTPUT_COLOUR) != 0;
    for (int l = tid; l < a.L; l += kPrepThreads) {
        double v[kRows];
        point_weights(a, l, v);
        a.w[l] = has_solar ? (float)(v[0] / solar) : 0.0f;
        a.w[a.L + l] = has_band ? (float)(v[1] / band) : 0.0f;
        for (int k = 2; k < kRows; ++k) a.w[(size_t)k * a.L + l] = has_colour ? (float)(v[k] / ny) : 0.0f;
    }
    if (tid == 0) {
        const double white[3] = {part[2][0] / ny, 1.0, part[4][0] / ny};
        double m[9];
        srgb_matrix(white, m);
        for (int i = 0; i < 3; ++i) a.params[i] = has_colour ? (float)white[i] : 0.0f;
        for (int i = 0; i < 9; ++i) a.params[3 + i] = has_colour ? (float)m[i] : 0.0f;
    }
}

__device__ __forceinline__ float lab_f(float t)
{
    constexpr float eps = 216.0f / 24389.0f;                 // (6/29)^3
    return t > eps ? cbrtf(t) : fmaf(t, 841.0f / 108.0f, 4.0f / 29.0f);     // 1 / (3 (6/29)^2) = 841/108
}

__device__ __forceinline__ float srgb_encode(float v)
{
    v = fminf(fmaxf(v, 0.0f), 1.0f);
    return v <= 0.0031308f ? 12.92f * v : 1.055f * powf(v, 1.0f / 2.4f) - 0.055f;
}

// the 13 outputs of design d from its 7 sums (R_s, A_s, T_s, band, X, Y, Z),
// written by the calling lane
__device__ void finish(const RunArgs& a, int64_t d, const float (&s)[7])
{
    const float nan = __builtin_nanf("");
    const bool solar = (a.avail & FOS_OUTPUT_SOLAR) != 0;
    float* t = a.totals + (size_t)d * 4;
    t[0] = solar ? s[0] : nan;
    t[1] = solar ? s[1] : nan;
    t[2] = solar ? s[2] : nan;
    t[3] = (a.avail & FOS_OUTPUT_BAND) ? s[3] : nan;
    if (!a.colour) return;
    float* c = a.colour + (size_t)d * 9;
    if (!(a.avail & FOS_OUTPUT_COLOUR)) {
        for (int i = 0; i < 9; ++i) c[i] = nan;
        return;
    }
    const float* p = a.params;
    const float X = s[4], Y = s[5], Z = s[6];
    const float fx = lab_f(X / p[0]), fy = lab_f(Y / p[1]), fz = lab_f(Z / p[2]);
    c[0] = X;
    c[1] = Y;
    c[2] = Z;
    c[3] = 116.0f * fy - 16.0f;
    c[4] = 500.0f * (fx - fy);
    c[5] = 200.0f * (fy - fz);
    for (int i = 0; i < 3; ++i) c[6 + i] = srgb_encode(p[3 + 3 * i] * X + p[4 + 3 * i] * Y + p[5 + 3 * i] * Z);
}

// the lane's 7 products of one wavelength with the weight rows, added to v
__device__ __forceinline__ void accumulate(float (&v)[8], float ws, float wb, float wx, float wy, float wz, float r,
                                           float ab, float t)
{
    v[0] = fmaf(ws, r, v[0]);
    v[1] = fmaf(ws, ab, v[1]);
    v[2] = fmaf(ws, t, v[2]);
    v[3] = fmaf(wb, ab, v[3]);
    v[4] = fmaf(wx, r, v[4]);
    v[5] = fmaf(wy, r, v[5]);
    v[6] = fmaf(wz, r, v[6]);
}

// Sums of 8 values over the wave by recursive halving: at the exchange
// across lane bit 5 each half keeps four of the values and sends the other
// four, across bit 4 two, across bit 3 one, and the last three exchanges add
// one value -- 10 shuffles where separate butterflies take 48.  Lanes
// 8k .. 8k + 7 end with the wave's sum of v[k].
__device__ __forceinline__ float wave_sums8(const float (&v)[8], int lane)
{
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0;
    float u[4], t[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = (b5 ? v[k + 4] : v[k]) + __shfl_xor(b5 ? v[k] : v[k + 4], 32);
#pragma unroll
    for (int k = 0; k < 2; ++k) t[k] = (b4 ? u[k + 2] : u[k]) + __shfl_xor(b4 ? u[k] : u[k + 2], 16);
    float z = (b3 ? t[1] : t[0]) + __shfl_xor(b3 ? t[0] : t[1], 8);
    z += __shfl_xor(z, 4);
    z += __shfl_xor(z, 2);
    z += __shfl_xor(z, 1);
    return z;
}

constexpr int kChunk = 32;      // designs per wave in output_run_kernel
constexpr int kMaxIter = 16;    // wavelengths per lane it holds in registers: grids up to 1024

// A wave takes kChunk consecutive designs.  Lane l holds wavelengths
// l, l + 64, ... (IT of them) with their five weights in registers; a lane's
// slots past the grid read the last wavelength again with zero weights, so
// every load is unconditional.  Two register sets of R, A, T alternate: the
// next design's spectrum is in flight while the current one is reduced, and
// the design's 7 sums go to lane j (its place in the chunk).  Past the
// chunk's end the loads repeat its last design (an L2 hit, result unused).
// The epilogue runs once per chunk, one design per lane.
template <int IT>
__global__ __launch_bounds__(256) void output_run_kernel(RunArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t d0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kChunk;
    if (d0 >= a.designs) return;
    const int nd = (int)(a.designs - d0 < kChunk ? a.designs - d0 : kChunk);
    const int L = a.L;
    float w[kRows][IT];
    int off[IT];                               // float offset of the lane's i-th wavelength in a row
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = lane + 64 * i;
        off[i] = 3 * (l < L ? l : L - 1);
#pragma unroll
        for (int k = 0; k < kRows; ++k) w[k][i] = l < L ? a.w[(size_t)k * L + l] : 0.0f;
    }
    const float* base = a.rat + (size_t)d0 * L * 3;
    const size_t stride = (size_t)L * 3;
    auto load = [&](float (&b)[IT][3], int j) {
        const float* row = base + (size_t)(j < nd ? j : nd - 1) * stride;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            b[i][0] = row[off[i]];
            b[i][1] = row[off[i] + 1];
            b[i][2] = row[off[i] + 2];
        }
    };
    float own[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto reduce = [&](const float (&b)[IT][3], int j) {
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < IT; ++i) accumulate(v, w[0][i], w[1][i], w[2][i], w[3][i], w[4][i], b[i][0], b[i][1], b[i][2]);
        const int z = __float_as_int(wave_sums8(v, lane));
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const float sk = __int_as_float(__builtin_amdgcn_readlane(z, 8 * k));
            own[k] = lane == j ? sk : own[k];
        }
    };
    // the scheduling barriers keep each prefetch ahead of the reduction it
    // overlaps (left alone, the scheduler sinks the loads past it)
    float A[IT][3], B[IT][3];
    load(A, 0);
    for (int j = 0; j < nd; j += 2) {
        load(B, j + 1);
        __builtin_amdgcn_sched_barrier(0);
        reduce(A, j);
        __builtin_amdgcn_sched_barrier(0);
        load(A, j + 2);
        __builtin_amdgcn_sched_barrier(0);
        reduce(B, j + 1);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane < nd) finish(a, d0 + lane, own);
}

// Grids wider than 64 x kMaxIter wavelengths: one wave per design, the
// weights read alongside the spectrum.
__global__ __launch_bounds__(256) void output_run_wide_kernel(RunArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t d = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (d >= a.designs) return;
    const int L = a.L;
    const float* row = a.rat + (size_t)d * L * 3;
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int l = lane; l < L; l += 64)
        accumulate(v, a.w[l], a.w[L + l], a.w[2 * (size_t)L + l], a.w[3 * (size_t)L + l], a.w[4 * (size_t)L + l],
                   row[3 * l], row[3 * l + 1], row[3 * l + 2]);
    const int z = __float_as_int(wave_sums8(v, lane));
    float s[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) s[k] = __int_as_float(__builtin_amdgcn_readlane(z, 8 * k));
    if (lane == 0) finish(a, d, s);
}

bool increasing_finite(const float* v, int n, bool positive)
{
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(v[i]) || (positive && !(v[i] > 0.0f))) return false;
        if (i > 0 && !(v[i] > v[i - 1])) return false;
    }
    return true;
}

bool spectrum_ok(const fos_spectrum* s, std::string& why)
{
    if (!s->um || !s->value) { why = "NULL spectrum array"; return false; }
    if (s->n < 2 || s->n > kMaxGrid) { why = "a spectrum needs 2 .. 2^20 samples"; return false; }
    if (!increasing_finite(s->um, s->n, true)) {
        why = "spectrum wavelengths must be finite, positive and strictly increasing";
        return false;
    }
    for (int i = 0; i < s->n; ++i)
        if (!std::isfinite(s->value[i]) || s->value[i] < 0.0f) {
            why = "spectrum values must be finite and non-negative";
            return false;
        }
    return true;
}

}  // namespace

}  // namespace fos

using namespace fosrt;

fos_status fos_output_prepare(fos_ctx* c, int32_t lambdas, const float* lambda_um, const fos_output_spec* spec,
                              int32_t* available, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    c->out_lambdas = 0;
    if (lambdas < 1 || lambdas > fos::kMaxGrid) return fail(c, FOS_E_INVALID_ARG, "need 1 <= lambdas <= 2^20");
    if (!lambda_um) return fail(c, FOS_E_INVALID_ARG, "NULL wavelength grid");
    if (!fos::increasing_finite(lambda_um, lambdas, true))
        return fail(c, FOS_E_INVALID_ARG, "grid wavelengths must be finite, positive and strictly increasing");
    const fos_spectrum* solar = spec ? spec->solar : nullptr;
    const fos_spectrum* illum = spec ? spec->illuminant : nullptr;
    std::string why;
    if (solar && !fos::spectrum_ok(solar, why)) return fail(c, FOS_E_INVALID_ARG, "solar: " + why);
    if (illum && !fos::spectrum_ok(illum, why)) return fail(c, FOS_E_INVALID_ARG, "illuminant: " + why);
    const float bt = spec ? spec->band_temperature_k : 0.0f;
    const float blo = spec ? spec->band_lo_um : 0.0f, bhi = spec ? spec->band_hi_um : 0.0f;
    if (!std::isfinite(bt)) return fail(c, FOS_E_INVALID_ARG, "band temperature must be finite");
    if (bt > 0.0f && !(std::isfinite(blo) && std::isfinite(bhi) && blo > 0.0f && blo < bhi))
        return fail(c, FOS_E_INVALID_ARG, "band needs finite 0 < lo < hi");

    // what the grid allows (decided on the single-precision grid values)
    const float first = lambda_um[0], last = lambda_um[lambdas - 1];
    int avail = 0;
    if (solar && lambdas >= 2 && first <= 0.28f && last >= 2.5f) avail |= FOS_OUTPUT_SOLAR;
    if (bt > 0.0f) {
        int inside = 0;
        for (int i = 0; i < lambdas; ++i) inside += lambda_um[i] >= blo && lambda_um[i] <= bhi;
        if (inside >= 2) avail |= FOS_OUTPUT_BAND;
    }
    if (lambdas >= 2 && first <= 0.38f && last >= 0.78f) avail |= FOS_OUTPUT_COLOUR;

    const int ns = solar ? solar->n : 0, ni = illum ? illum->n : 0;
    const size_t L = (size_t)lambdas;
    const size_t floats = fos::kRows * L + fos::kOutParams + L + 2 * (size_t)ns + 2 * (size_t)ni;
    DeviceGuard guard(c->device);
    hipError_t e = grow(c->out_buf, c->out_buf_bytes, floats * sizeof(float));
    if (e != hipSuccess) return hip_fail(c, e, "output-stage buffer");
    float* w = c->out_buf;
    float* params = w + fos::kRows * L;
    float* lam = params + fos::kOutParams;
    float* s_um = lam + L;
    float* s_val = s_um + ns;
    float* i_um = s_val + ns;
    float* i_val = i_um + ni;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    auto up = [&](float* dst, const float* src, size_t n) {
        return n ? hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyHostToDevice, st) : hipSuccess;
    };
    if ((e = up(lam, lambda_um, L)) != hipSuccess || (e = up(s_um, solar ? solar->um : nullptr, ns)) != hipSuccess ||
        (e = up(s_val, solar ? solar->value : nullptr, ns)) != hipSuccess ||
        (e = up(i_um, illum ? illum->um : nullptr, ni)) != hipSuccess ||
        (e = up(i_val, illum ? illum->value : nullptr, ni)) != hipSuccess)
        return hip_fail(c, e, "output-stage upload");
    // the caller's host arrays are free once this returns
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "output-stage upload");
    fos::PrepArgs a{};
    a.L = lambdas; a.lam = lam;
    a.ns = ns; a.s_um = s_um; a.s_val = s_val;
    a.ni = ni; a.i_um = i_um; a.i_val = i_val;
    a.band_lo = blo; a.band_hi = bhi; a.band_t = bt;
    a.avail = avail; a.w = w; a.params = params;
    hipLaunchKernelGGL(fos::output_prepare_kernel, dim3(1), dim3(fos::kPrepThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "output-stage weights");
    c->out_lambdas = lambdas;
    c->out_avail = avail;
    if (available) *available = avail;
    return FOS_OK;
}

fos_status fos_output_run(fos_ctx* c, int32_t designs, int32_t lambdas, const float* rat, float* totals,
                          float* colour, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (c->out_lambdas < 1) return fail(c, FOS_E_NOT_PREPARED, "fos_output_prepare has not succeeded");
    if (lambdas != c->out_lambdas)
        return fail(c, FOS_E_INVALID_ARG, "lambdas differs from the prepared grid (" +
                                              std::to_string(c->out_lambdas) + ")");
    if (designs < 0) return fail(c, FOS_E_INVALID_ARG, "need designs >= 0");
    if (designs == 0) return FOS_OK;
    if (!rat || !totals) return fail(c, FOS_E_INVALID_ARG, "NULL array");
    DeviceGuard guard(c->device);
    fos::RunArgs a{};
    a.designs = designs;
    a.L = c->out_lambdas;
    a.rat = rat;
    a.w = c->out_buf;
    a.params = c->out_buf + fos::kRows * (size_t)c->out_lambdas;
    a.totals = totals;
    a.colour = colour;
    a.avail = c->out_avail;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int iters = (a.L + 63) / 64;
    const unsigned chunked = (unsigned)((designs + 4 * fos::kChunk - 1) / (4 * fos::kChunk));
    if (iters <= 1) hipLaunchKernelGGL(fos::output_run_kernel<1>, dim3(chunked), dim3(256), 0, st, a);
    else if (iters <= 2) hipLaunchKernelGGL(fos::output_run_kernel<2>, dim3(chunked), dim3(256), 0, st, a);
    else if (iters <= 4) hipLaunchKernelGGL(fos::output_run_kernel<4>, dim3(chunked), dim3(256), 0, st, a);
    else if (iters <= 8) hipLaunchKernelGGL(fos::output_run_kernel<8>, dim3(chunked), dim3(256), 0, st, a);
    else if (iters <= fos::kMaxIter)
        hipLaunchKernelGGL(fos::output_run_kernel<fos::kMaxIter>, dim3(chunked), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(fos::output_run_wide_kernel, dim3((unsigned)((designs + 3) / 4)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FOS_OK : hip_fail(c, e, "output stage");
}

fos_status fos_output_weights(fos_ctx* c, float* weights, float* params, int32_t* available, void* hip_stream)
{
    if (!c) return FOS_E_INVALID_ARG;
    c->err.clear();
    if (c->out_lambdas < 1) return fail(c, FOS_E_NOT_PREPARED, "fos_output_prepare has not succeeded");
    DeviceGuard guard(c->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t L = (size_t)c->out_lambdas;
    hipError_t e = hipSuccess;
    if (weights) e = hipMemcpyAsync(weights, c->out_buf, fos::kRows * L * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && params)
        e = hipMemcpyAsync(params, c->out_buf + fos::kRows * L, fos::kOutParams * sizeof(float),
                           hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "output-stage weights copy");
    if (available) *available = c->out_avail;
    return FOS_OK;
}
