// optics_kernels.hip -- effective scattering properties of particle-laden
// layers on the GPU (Methodology, Scattering properties): Lorenz-Mie
// efficiencies of every (particle size, wavelength) entry in an absorbing
// host, eqs. (1)-(5), (10)-(12), (15), then the effective medium of every
// layer cell, eqs. (13)-(20).  Double precision throughout.
//
//   optics_scan : one wave per cell -- validate, record the owning cell of
//                 each particle entry, and the largest Mie series length.
//   order_units : the size units ordered by series length within contiguous
//                 ranges, so the lanes of a wave run series of similar length.
//   mie_entries : waves claim 64 sorted size units at a time, taking the
//                 ranges in turn so the longest series start first; per unit the
//                 logarithmic derivative D_n(m x) by downward recurrence (kept
//                 in a strided global scratch), psi_n(x) and xi_n(x) by upward
//                 recurrence, a_n and b_n in the Bohren-Huffman form, and the
//                 three series of eqs. (11), (12), (15).
//   emt_cells   : one wave per cell -- eqs. (13)-(16), the clamp, the dependent-
//                 scattering factor (17)-(19) and matrix absorption (20).
//   lognormal_* : log-normal populations whose bins lie on one radius grid:
//                 per (species, matrix, wavelength, median radius) the bin
//                 sums of eqs. (13), (14), (16) from efficiencies evaluated
//                 once per grid radius (by mie_entries), then per (design,
//                 wavelength) cell the same clamp / factor / matrix term as
//                 emt_cells with f_i = f w_b.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fos_kernels.hpp"


namespace fos {

struct cd {
    double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__device__ __forceinline__ cd conj_(cd a) { return cd{a.re, -a.im}; }
__device__ __forceinline__ double abs2(cd a) { return a.re * a.re + a.im * a.im; }
// 1/x for x in [1/4, 2]: the hardware estimate and two Newton steps (each
// doubles the correct bits), a few ulp from the rounded quotient.
__device__ __forceinline__ double rcp_near_one(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
// 1/b = conj(b) / |b|^2, with b first scaled by the power of two that brings
// its larger part into [1/2, 1), so |b|^2 neither overflows nor underflows and
// one reciprocal replaces the three divisions (and the branch) of Smith's
// method.
__device__ __forceinline__ cd recip(cd b)
{
    const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(b.re), fabs(b.im)));
    const double br = ldexp(b.re, -e), bi = ldexp(b.im, -e);
    const double q = rcp_near_one(br * br + bi * bi);
    return cd{ldexp(br * q, -e), ldexp(-bi * q, -e)};
}
__device__ __forceinline__ cd operator/(cd a, cd b) { return a * recip(b); }
__device__ __forceinline__ cd csin_(cd z) { return cd{sin(z.re) * cosh(z.im), cos(z.re) * sinh(z.im)}; }
__device__ __forceinline__ cd ccos_(cd z) { return cd{cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)}; }

__device__ __forceinline__ int series_length(double ay) { return (int)ceil(2.0 + ay + 4.3 * cbrt(ay)); }

__device__ __forceinline__ void optics_report(unsigned long long* err, int cell, int code)
{
    atomicMin(err, ((unsigned long long)(uint32_t)cell << 8) | (unsigned long long)code);
}

// Diameter of size unit `sub` of a Gaussian spread (mean diameter d0,
// standard deviation sd): 101 diameters evenly over d0 - 3 sd .. d0 + 3 sd.
__device__ __forceinline__ double spread_diameter(double d0, double sd, int sub)
{
    return d0 - 3.0 * sd + 6.0 * sd * (double)sub / (double)(kSpreadSizes - 1);
}

// Validation and series bound: one wave per cell, its lanes striding over the
// cell's particle entries (cells may hold hundreds), then a wave reduction of
// the longest series and of the kind flags.
__global__ void optics_scan(OpticsArgs a)
{
    const int lane = threadIdx.x & 63;
    const int c = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (c >= a.n_cells) return;   // whole waves
    const double lam = a.lam[c], nm = a.n_m[c], km = a.k_m[c];
    const int64_t b = a.offsets[c], e = a.offsets[c + 1];
    bool bad = false;
    if (!(lam > 0.0) || !isfinite(lam)) { if (lane == 0) optics_report(a.err, c, kOptErrLambda); bad = true; }
    if (!(nm > 0.0) || !isfinite(nm)) { if (lane == 0) optics_report(a.err, c, kOptErrNm); bad = true; }
    if (!(km >= 0.0) || !isfinite(km)) { if (lane == 0) optics_report(a.err, c, kOptErrKm); bad = true; }
    if (b < 0 || e < b || e > a.n_entries) {
        if (lane == 0) optics_report(a.err, c, kOptErrOffsets);
        return;
    }
    if (bad) return;
    int nmax = 0;
    unsigned int flags = 0u;
    const double two_pi = 2.0 * 3.141592653589793;
    for (int64_t j = b + lane; j < e; j += 64) {
        const double np_ = a.n_p[j], kp = a.k_p[j], r = a.r[j], f = a.f[j];
        const double sd = a.sd ? a.sd[j] : 0.0;
        const double rc = a.r_core ? a.r_core[j] : 0.0;
        int code = 0;
        if (!(np_ > 0.0) || !isfinite(np_)) code = kOptErrNp;
        else if (!(kp >= 0.0) || !isfinite(kp)) code = kOptErrKp;
        else if (!(r > 0.0) || !isfinite(r)) code = kOptErrRadius;
        else if (!(f >= 0.0) || !isfinite(f)) code = kOptErrFraction;
        else if (!(sd >= 0.0) || !isfinite(sd)) code = kOptErrSpread;
        else if (!(rc >= 0.0) || !(rc <= r)) code = kOptErrCore;
        else if (sd > 0.0 && rc > 0.0) code = kOptErrSpreadCore;
        else if (rc > 0.0) {
            const double nc = a.n_core[j], kc = a.k_core[j];
            if (!(nc > 0.0) || !isfinite(nc) || !(kc >= 0.0) || !isfinite(kc)) code = kOptErrCore;
        }
        if (code != 0) {
            optics_report(a.err, c, code);
            break;
        }
        a.cell_of[j] = c;
        // |y| of eq. (1) for the largest size of the entry, at the larger index
        double ay = two_pi * (sd > 0.0 ? 0.5 * spread_diameter(2.0 * r, sd, kSpreadSizes - 1) : r) *
                    sqrt(np_ * np_ + kp * kp) / lam;
        if (rc > 0.0) {
            ay = fmax(ay, two_pi * rc * sqrt(a.n_core[j] * a.n_core[j] + a.k_core[j] * a.k_core[j]) / lam);
            flags |= kOptHasCore;
        }
        if (sd > 0.0) flags |= kOptHasSpread;
        const int nn = series_length(ay) + 1;
        if (nn > nmax) nmax = nn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nmax = max(nmax, __shfl_xor(nmax, o));
        flags |= (unsigned int)__shfl_xor((int)flags, o);
    }
    if (lane == 0) {
        if (nmax > 0) atomicMax(a.nmax, (unsigned int)nmax);
        if (flags) atomicOr(a.flags, flags);
    }
}

// D_n(z), n = 1..nn, by downward recurrence from far above, stored strided
// (D[n * stride]); returns D_0 as well (from the n = 1 step).
__device__ cd log_derivative_strided(cd z, int nn, double az, cd* D, size_t stride)
{
    int nstart = nn;
    if (ceil(az) > nstart) nstart = (int)ceil(az);
    nstart += 16;
    const cd iz = recip(z);
    cd d = mk(0.0, 0.0);
    for (int n = nstart; n > nn; --n) {
        const cd nz = (double)n * iz;
        d = nz - recip(d + nz);
    }
    D[(size_t)nn * stride] = d;
    for (int n = nn; n >= 1; --n) {
        const cd nz = (double)n * iz;
        d = nz - recip(d + nz);
        if (n >= 2) D[(size_t)(n - 1) * stride] = d;
    }
    return d;   // D_0
}

// Efficiency series of one sphere (homogeneous, or coated when Nc is given):
// sext, ssca, sg of eqs. (11), (12), (15).  A coated sphere (core radius rc,
// index Nc, inside a shell Ns out to r) enters through the logarithmic form of
// eqs. (S1)-(S4): with D = psi'/psi and G = chi'/chi of the core and shell
// arguments, T = psi/chi, and
//   U = (m2 D(m1x) - m1 D(m2x)) / (m2 D(m1x) - m1 G(m2x)) T(m2x)/T(m2y)
//   V = (m2 D(m2x) - m1 D(m1x)) / (m2 G(m2x) - m1 D(m1x)) T(m2x)/T(m2y),
// a_n and b_n take the homogeneous form with D(my)/m replaced by
// (D(m2y) - U G(m2y)) / (m2 (1 - U)) and m D(my) by m2 (D(m2y) - V G(m2y)) /
// (1 - V); U = V = 0 gives the homogeneous sphere back.  G and T follow the
// upward recurrences G_n = 1/(n/z - G_{n-1}) - n/z and
// T_n = T_{n-1} (n/z - D_{n-1}) / (n/z - G_{n-1}), from G_0 = T_0 = -tan z.
struct Series {
    double sext, ssca, sg;
};

__device__ Series mie_series(double lam, cd Nm, cd Ns, double r, bool coated, cd Nc, double rc, int nn_cap,
                             cd* scratch, size_t stride, size_t dstride)
{
    const double pi = 3.141592653589793;
    const double k0 = 2.0 * pi / lam;
    const cd x_out = (k0 * r) * Nm;                 // host size parameter of the outer surface
    const cd m2 = Ns / Nm;
    const cd y2 = m2 * x_out;                       // shell (or particle) argument at r
    double ay = k0 * r * sqrt(abs2(Ns));
    if (coated) ay = fmax(ay, k0 * rc * sqrt(abs2(Nc)));
    int nn = series_length(ay) + 1;                 // eq. (15) needs a_{nmax+1}
    if (nn > nn_cap) nn = nn_cap;
    const int nmax = nn - 1;
    cd* D2y = scratch;                              // D_n(m2 y)
    const cd D2y0 = log_derivative_strided(y2, nn, sqrt(abs2(y2)), D2y, stride);
    cd* D1x = scratch + dstride;                    // D_n(m1 x)   (coated only)
    cd* D2x = scratch + 2 * dstride;                // D_n(m2 x)
    cd m1 = mk(0.0, 0.0), z1 = mk(0.0, 0.0), z2 = mk(0.0, 0.0);
    cd G2x = mk(0.0, 0.0), G2y = mk(0.0, 0.0), T2x = mk(0.0, 0.0), T2y = mk(0.0, 0.0);
    cd D2x0 = mk(0.0, 0.0);
    if (coated) {
        const cd x_in = (k0 * rc) * Nm;
        m1 = Nc / Nm;
        z1 = m1 * x_in;
        z2 = m2 * x_in;
        log_derivative_strided(z1, nn, sqrt(abs2(z1)), D1x, stride);
        D2x0 = log_derivative_strided(z2, nn, sqrt(abs2(z2)), D2x, stride);
        const cd t2x = csin_(z2) / ccos_(z2), t2y = csin_(y2) / ccos_(y2);
        G2x = mk(-t2x.re, -t2x.im); T2x = G2x;      // G_0 = T_0 = -tan z
        G2y = mk(-t2y.re, -t2y.im); T2y = G2y;
    }
    // upward psi_n(x), xi_n(x) = x h_n^(1)(x) of the outer host argument
    const cd ix = recip(x_out);
    const cd sx = csin_(x_out), cx = ccos_(x_out);
    cd psi_m1 = cx, psi_0 = sx;
    cd xi_m1 = mk(cx.re - sx.im, cx.im + sx.re);   // cos x + i sin x
    cd xi_0 = mk(sx.re + cx.im, sx.im - cx.re);    // sin x - i cos x
    const cd iNm2 = recip(Nm * Nm);
    const cd im2 = recip(m2);
    const cd iz2 = coated ? recip(z2) : mk(0.0, 0.0), iy2 = recip(y2);
    cd D2x_prev = D2x0, D2y_prev = D2y0;
    Series S{0.0, 0.0, 0.0};
    cd a_prev = mk(0.0, 0.0), b_prev = mk(0.0, 0.0);
    bool done = false;
    for (int n = 1; n <= nn && !done; ++n) {
        const double fn = (double)n;
        const cd psi_n = (2.0 * fn - 1.0) * ix * psi_0 - psi_m1;
        const cd xi_n = (2.0 * fn - 1.0) * ix * xi_0 - xi_m1;
        cd an, bn;
        const cd Dy = D2y[(size_t)n * stride];
        cd ta = Dy * im2, tb = m2 * Dy;            // homogeneous: D(my)/m and m D(my)
        if (coated) {
            const cd nz2 = fn * iz2, ny2 = fn * iy2;
            // upward G_n and T_n of the shell arguments
            T2x = T2x * (nz2 - D2x_prev) / (nz2 - G2x);
            T2y = T2y * (ny2 - D2y_prev) / (ny2 - G2y);
            G2x = recip(nz2 - G2x) - nz2;
            G2y = recip(ny2 - G2y) - ny2;
            const cd D1 = D1x[(size_t)n * stride], D2 = D2x[(size_t)n * stride];
            const cd ratio = T2x / T2y;
            const cd U = (m2 * D1 - m1 * D2) / (m2 * D1 - m1 * G2x) * ratio;
            const cd V = (m2 * D2 - m1 * D1) / (m2 * G2x - m1 * D1) * ratio;
            const cd one = mk(1.0, 0.0);
            ta = (Dy - U * G2y) / (m2 * (one - U));
            tb = m2 * (Dy - V * G2y) / (one - V);
            D2x_prev = D2;
            D2y_prev = Dy;
        }
        if (!isfinite(xi_n.re) || !isfinite(xi_n.im) || abs2(xi_n) > 1e300) {
            // psi_n/xi_n -> 0 far above |x|: remaining coefficients vanish
            an = mk(0.0, 0.0); bn = mk(0.0, 0.0);
            done = true;
        } else {
            const cd nx = fn * ix;
            const cd ua = ta + nx, ub = tb + nx;
            an = (ua * psi_n - psi_0) / (ua * xi_n - xi_0);
            bn = (ub * psi_n - psi_0) / (ub * xi_n - xi_0);
        }
        if (n >= 2) {   // cross term of eq. (15) for the pair (n-1, n)
            const double f1 = fn - 1.0;
            S.sg += f1 * (f1 + 2.0) / (f1 + 1.0) * ((a_prev * conj_(an)).re + (b_prev * conj_(bn)).re);
        }
        if (n <= nmax) {
            S.sext += (2.0 * fn + 1.0) * ((an + bn) * iNm2).re;
            S.ssca += (2.0 * fn + 1.0) * (abs2(an) + abs2(bn));
            S.sg += (2.0 * fn + 1.0) / (fn * (fn + 1.0)) * (an * conj_(bn)).re;
        }
        a_prev = an; b_prev = bn;
        psi_m1 = psi_0; psi_0 = psi_n;
        xi_m1 = xi_0; xi_0 = xi_n;
    }
    return S;
}

// Size units ordered by series length within contiguous ranges of about
// kOrderRange units, one block per range: a class histogram in LDS (class =
// series length, capped at kOrderClasses - 1), its exclusive prefix, then
// every unit placed at its class offset plus its rank.  With ranges this
// long a class holds dozens of units, so 64 neighbouring positions of the
// order hold series of nearly equal length, which is what the lanes of a
// wave need.  The order within a class is not fixed, and need not be: each
// unit's result is written at its own index.
constexpr int kOrderClasses = 1024;
#ifndef FOS_ORDER_RANGE
#define FOS_ORDER_RANGE 4096
#endif
constexpr int64_t kOrderRange = FOS_ORDER_RANGE;

// Units per ordered range for n_units units: about kOrderRange, one block of
// order_units per range, at most 65535 ranges.
__host__ __device__ __forceinline__ int64_t order_range(int64_t n_units)
{
    int64_t blocks = (n_units + kOrderRange - 1) / kOrderRange;
    if (blocks > 65535) blocks = 65535;
    return (n_units + blocks - 1) / blocks;
}

__device__ __forceinline__ int unit_class(const OpticsArgs& a, int64_t u)
{
    const double two_pi = 2.0 * 3.141592653589793;
    const int64_t j = u / a.units;
    const int sub = (int)(u % a.units);
    const double sd = a.sd ? a.sd[j] : 0.0;
    const double rc = a.r_core ? a.r_core[j] : 0.0;
    double r = a.r[j];
    if (sd > 0.0) {
        const double d = spread_diameter(2.0 * r, sd, sub);
        if (!(d > 0.0)) return 0;   // skipped by mie_entries
        r = 0.5 * d;
    } else if (sub > 0) {
        return 0;
    }
    const double lam = a.lam[a.cell_of[j]];
    double ay = two_pi * r * sqrt(a.n_p[j] * a.n_p[j] + a.k_p[j] * a.k_p[j]) / lam;
    if (rc > 0.0) ay = fmax(ay, two_pi * rc * sqrt(a.n_core[j] * a.n_core[j] + a.k_core[j] * a.k_core[j]) / lam);
    const int nn = series_length(ay) + 1;
    return nn < kOrderClasses ? nn : kOrderClasses - 1;
}

__global__ __launch_bounds__(256) void order_units(OpticsArgs a, int64_t n_units, int64_t per_block,
                                                   unsigned short* cls, unsigned int* order)
{
    __shared__ unsigned int next[kOrderClasses];
    __shared__ unsigned int part[256];
    const int t = threadIdx.x;
    for (int k = t; k < kOrderClasses; k += 256) next[k] = 0u;
    __syncthreads();
    const int64_t u0 = (int64_t)blockIdx.x * per_block;
    const int64_t u1 = u0 + per_block < n_units ? u0 + per_block : n_units;
    for (int64_t u = u0 + t; u < u1; u += 256) {
        const int k = kOrderClasses - 1 - unit_class(a, u);   // longest series first
        cls[u] = (unsigned short)k;
        atomicAdd(&next[k], 1u);
    }
    __syncthreads();
    // exclusive prefix of the histogram: 4 classes per thread, then across threads
    constexpr int per = kOrderClasses / 256;
    unsigned int c[per], sum = 0u;
#pragma unroll
    for (int i = 0; i < per; ++i) { c[i] = next[per * t + i]; sum += c[i]; }
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const unsigned int v = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned int run = (unsigned int)u0 + part[t] - sum;
#pragma unroll
    for (int i = 0; i < per; ++i) { next[per * t + i] = run; run += c[i]; }
    __syncthreads();
    for (int64_t u = u0 + t; u < u1; u += 256) {
        const unsigned int pos = atomicAdd(&next[cls[u]], 1u);
        order[pos] = (unsigned int)u;
    }
}

// One thread per size unit (entry, sub): Gaussian spreads give 101 units per
// entry (unused units are skipped), everything else one.  Waves claim 64
// positions at a time from a queue counter.  Without an order the positions
// are the units themselves.  With one (a.order: ranges of order_range units,
// each longest series first) claim c takes chunk c / R of range c % R, R
// ranges in all: the first chunks of every range come before the second of
// any, so the longest series of the whole request start first and the short
// ones fill the end.
__global__ __launch_bounds__(256) void mie_entries(OpticsArgs a)
{
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nthreads = (size_t)gridDim.x * blockDim.x;
    const double pi = 3.141592653589793;
    const size_t n_units = (size_t)a.n_entries * a.units;
    const size_t dstride = ((size_t)a.nn_cap + 1) * nthreads;
    const int lane = threadIdx.x & 63;
    const size_t range = a.order ? (size_t)order_range((int64_t)n_units) : n_units;
    const size_t n_ranges = (n_units + range - 1) / range;
    const size_t n_claims = n_ranges * ((range + 63) / 64);
    for (;;) {
        // each wave takes the next chunk from the queue, so waves that drew
        // short series take more of them
        unsigned long long claim = 0ull;
        if (lane == 0) claim = atomicAdd(a.queue, 1ull);
        claim = __shfl(claim, 0);
        if (claim >= n_claims) break;
        const size_t rg = (size_t)claim % n_ranges;
        const size_t r0 = rg * range;
        const size_t r1 = r0 + range < n_units ? r0 + range : n_units;
        const size_t s = r0 + 64 * ((size_t)claim / n_ranges) + lane;
        if (s >= r1) continue;
        const size_t u = a.order ? (size_t)a.order[s] : s;
        const size_t j = u / a.units;
        const int sub = (int)(u % a.units);
        const int c = a.cell_of[j];
        const double lam = a.lam[c];
        const double sd = a.sd ? a.sd[j] : 0.0;
        const double rc = a.r_core ? a.r_core[j] : 0.0;
        double r = a.r[j];
        if (sd > 0.0) {
            const double d = spread_diameter(2.0 * r, sd, sub);
            if (!(d > 0.0)) continue;                  // sizes that are not positive are left out
            r = 0.5 * d;
        } else if (sub > 0) {
            continue;
        }
        const cd Nm = mk(a.n_m[c], a.k_m[c]);
        const cd Np = mk(a.n_p[j], a.k_p[j]);
        const bool coated = rc > 0.0;
        const cd Nc = coated ? mk(a.n_core[j], a.k_core[j]) : mk(1.0, 0.0);
        cd* scratch = reinterpret_cast<cd*>(a.scratch) + tid;
        const Series S = mie_series(lam, Nm, Np, r, coated, Nc, rc, a.nn_cap, scratch, nthreads, dstride);
        // eqs. (10)-(12), cross sections referred to the (outer) radius r
        const double alpha = 4.0 * pi * r * a.k_m[c] / lam;
        double gam;
        if (fabs(alpha) < 1e-3)
            gam = 1.0 + alpha * (2.0 / 3.0 + alpha * (0.25 + alpha * (1.0 / 15.0 + alpha / 72.0)));
        else
            gam = 2.0 * (1.0 + (alpha - 1.0) * exp(alpha)) / (alpha * alpha);
        const double area = pi * r * r;
        const double cext = lam * lam / (2.0 * pi) * S.sext;
        const double csca = lam * lam * exp(-alpha) / (2.0 * pi * gam * abs2(Nm)) * S.ssca;
        a.mie[3 * u + 0] = cext / area;
        a.mie[3 * u + 1] = csca / area;
        a.mie[3 * u + 2] = S.ssca > 0.0 ? 2.0 * S.sg / S.ssca : 0.0;
    }
}

// Effective medium of each cell, eqs. (13)-(20): one wave per cell.  Lanes
// stride over the cell's entries; an entry with a Gaussian spread is taken
// by the whole wave, its 101 diameters across the lanes (the weight
// normalisation is a wave sum).  Partial sums are reduced across the wave.
__global__ void emt_cells(OpticsArgs a)
{
    const int lane = threadIdx.x & 63;
    const int c = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (c >= a.n_cells) return;   // whole waves
    const int64_t b = a.offsets[c], e = a.offsets[c + 1];
    double mus = 0.0, mua = 0.0, gs = 0.0, F = 0.0;
    for (int64_t j = b + lane; j < e; j += 64) {
        const double f = a.f[j];
        F += f;
        if (a.sd && a.sd[j] > 0.0) continue;   // below
        const double* q = a.mie + 3 * (size_t)j * a.units;
        const double r = a.r[j];
        const double ws = 1.5 * q[1] * f / (2.0 * r);
        mus += ws;
        mua += 1.5 * (q[0] - q[1]) * f / (2.0 * r);
        gs += ws * q[2];
    }
    if (a.sd) {
        for (int64_t j = b; j < e; ++j) {
            const double sd = a.sd[j];
            if (!(sd > 0.0)) continue;
            // Gaussian weights of the 101 diameters, renormalised over the positive ones
            const double d0 = 2.0 * a.r[j], f = a.f[j];
            const double* q = a.mie + 3 * (size_t)j * a.units;
            double wsum = 0.0;
            for (int k = lane; k < kSpreadSizes; k += 64) {
                const double d = spread_diameter(d0, sd, k);
                if (!(d > 0.0)) continue;
                const double z = (d - d0) / sd;
                wsum += exp(-0.5 * z * z);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o);
            for (int k = lane; k < kSpreadSizes; k += 64) {
                const double d = spread_diameter(d0, sd, k);
                if (!(d > 0.0)) continue;
                const double z = (d - d0) / sd;
                const double fk = f * (exp(-0.5 * z * z) / wsum), rk = 0.5 * d;
                const double* qk = q + 3 * k;
                const double ws = 1.5 * qk[1] * fk / (2.0 * rk);
                mus += ws;
                mua += 1.5 * (qk[0] - qk[1]) * fk / (2.0 * rk);
                gs += ws * qk[2];
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mus += __shfl_xor(mus, o);
        mua += __shfl_xor(mua, o);
        gs += __shfl_xor(gs, o);
        F += __shfl_xor(F, o);
    }
    if (lane != 0) return;
    double g = mus > 0.0 ? gs / mus : 0.0;
    if (mus < 0.0) mus = 0.0;
    if (mua < 0.0) mua = 0.0;
    if (F > 0.08) {
        const double C = 1.0 + 1.5 * F - 0.75 * F * F;
        mus *= C;
        mua *= C;
    }
    mua += 4.0 * 3.141592653589793 * a.k_m[c] * (1.0 - F) / a.lam[c];
    if (a.out_mu_s) a.out_mu_s[c] = (float)mus;
    if (a.out_mu_a) a.out_mu_a[c] = (float)mua;
    if (a.out_g) a.out_g[c] = (float)g;
    if (a.out_f64) {
        a.out_f64[3 * (size_t)c + 0] = mus;
        a.out_f64[3 * (size_t)c + 1] = mua;
        a.out_f64[3 * (size_t)c + 2] = g;
    }
}

__global__ void lognormal_check(LognormalArgs a)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= a.n_designs) return;
    const int s = a.species[d], h = a.matrix[d], k = a.rmed[d];
    const double f = a.f[d];
    if (s < 0 || s >= a.n_species) optics_report(a.err, d, kLnErrSpecies);
    else if (h < 0 || h >= a.n_matrix) optics_report(a.err, d, kLnErrMatrix);
    else if (k < 0 || k >= a.n_rmed) optics_report(a.err, d, kLnErrRmed);
    else if (!(f >= 0.0 && f <= 1.0)) optics_report(a.err, d, kLnErrFraction);
}

// one thread per (species, matrix, wavelength, median radius)
__global__ void lognormal_table(LognormalArgs a)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t cells = (size_t)a.n_species * a.n_matrix * a.n_lambda;
    if (t >= cells * a.n_rmed) return;
    const int k = (int)(t % a.n_rmed);
    const size_t c = t / a.n_rmed;
    double ts = 0.0, ta = 0.0, tg = 0.0;
    for (int b = 0; b < a.n_bins; ++b) {
        const int j = k + b;
        const double* q = a.mie + 3 * (c * a.n_radii + j);
        const double r = a.radii[j], w = a.w[b];
        const double ws = 1.5 * q[1] * w / (2.0 * r);
        ts += ws;
        ta += 1.5 * (q[0] - q[1]) * w / (2.0 * r);
        tg += ws * q[2];
    }
    a.table[3 * t + 0] = ts;
    a.table[3 * t + 1] = ta;
    a.table[3 * t + 2] = tg;
}

// one thread per (design, wavelength) cell
__global__ void lognormal_cells(LognormalArgs a)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)a.n_designs * a.n_lambda) return;
    const int d = (int)(t / a.n_lambda), l = (int)(t % a.n_lambda);
    const int s = a.species[d], h = a.matrix[d], k = a.rmed[d];
    const double F = a.f[d];
    const double* T = a.table + 3 * ((((size_t)s * a.n_matrix + h) * a.n_lambda + l) * a.n_rmed + k);
    double mus = F * T[0], mua = F * T[1];
    const double gs = F * T[2];
    const double g = mus > 0.0 ? gs / mus : 0.0;
    if (mus < 0.0) mus = 0.0;
    if (mua < 0.0) mua = 0.0;
    if (F > 0.08) {
        const double C = 1.0 + 1.5 * F - 0.75 * F * F;
        mus *= C;
        mua *= C;
    }
    mua += 4.0 * 3.141592653589793 * a.k_m * (1.0 - F) / a.lam[l];
    if (a.out_mu_s) a.out_mu_s[t] = (float)mus;
    if (a.out_mu_a) a.out_mu_a[t] = (float)mua;
    if (a.out_g) a.out_g[t] = (float)g;
}

hipError_t launch_lognormal_check(const LognormalArgs& a, hipStream_t st)
{
    if (a.n_designs <= 0) return hipSuccess;
    hipLaunchKernelGGL(lognormal_check, dim3((a.n_designs + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lognormal_table(const LognormalArgs& a, hipStream_t st)
{
    const size_t n = (size_t)a.n_species * a.n_matrix * a.n_lambda * a.n_rmed;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(lognormal_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lognormal_cells(const LognormalArgs& a, hipStream_t st)
{
    const size_t n = (size_t)a.n_designs * a.n_lambda;
    if (n == 0) return hipSuccess;
    if ((n + 255) / 256 > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lognormal_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_optics_scan(const OpticsArgs& a, hipStream_t st)
{
    if (a.n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(optics_scan, dim3((unsigned)(((size_t)a.n_cells * 64 + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mie(const OpticsArgs& a, int grid, int block, hipStream_t st)
{
    if (a.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(mie_entries, dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

size_t mie_order_bytes(int64_t n_units)
{
    return (size_t)n_units * (sizeof(unsigned int) + sizeof(unsigned short)) + 256;
}

hipError_t launch_mie_order(const OpticsArgs& a, int64_t n_units, void* buf, hipStream_t st)
{
    if (n_units <= 0) return hipSuccess;
    const int64_t per_block = order_range(n_units);
    const int64_t blocks = (n_units + per_block - 1) / per_block;
    unsigned int* order = reinterpret_cast<unsigned int*>(buf);
    unsigned short* cls = reinterpret_cast<unsigned short*>(order + n_units);
    hipLaunchKernelGGL(order_units, dim3((unsigned)blocks), dim3(256), 0, st, a, n_units, per_block, cls, order);
    return hipGetLastError();
}

hipError_t launch_emt(const OpticsArgs& a, hipStream_t st)
{
    if (a.n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(emt_cells, dim3((unsigned)(((size_t)a.n_cells * 64 + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace fos
