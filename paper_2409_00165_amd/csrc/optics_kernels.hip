// optics_kernels.hip -- effective scattering properties of particle-laden
// layers on the GPU (Methodology, Scattering properties): Lorenz-Mie
// efficiencies of every (particle size, wavelength) entry in an absorbing
// host, eqs. (1)-(5), (10)-(12), (15), then the effective medium of every
// layer cell, eqs. (13)-(20).  Double precision throughout.
//
//   optics_scan : per cell -- validate, record the owning cell of each
//                 particle entry, and the largest Mie series length.
//   mie_entries : grid-stride over particle entries; per entry the
//                 logarithmic derivative D_n(m x) by downward recurrence (kept
//                 in a strided global scratch), psi_n(x) and xi_n(x) by upward
//                 recurrence, a_n and b_n in the Bohren-Huffman form, and the
//                 three series of eqs. (11), (12), (15).
//   emt_cells   : per cell -- eqs. (13)-(16), the clamp, the dependent-
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
// Smith's division
__device__ __forceinline__ cd operator/(cd a, cd b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return cd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    const double r = b.re / b.im, d = b.re * r + b.im;
    return cd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ cd recip(cd b) { return mk(1.0, 0.0) / b; }
__device__ __forceinline__ cd csin_(cd z) { return cd{sin(z.re) * cosh(z.im), cos(z.re) * sinh(z.im)}; }
__device__ __forceinline__ cd ccos_(cd z) { return cd{cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)}; }

__device__ __forceinline__ int series_length(double ay) { return (int)ceil(2.0 + ay + 4.3 * cbrt(ay)); }

__device__ __forceinline__ void optics_report(unsigned long long* err, int cell, int code)
{
    atomicMin(err, ((unsigned long long)(uint32_t)cell << 8) | (unsigned long long)code);
}

__global__ void optics_scan(OpticsArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cells) return;
    const double lam = a.lam[c], nm = a.n_m[c], km = a.k_m[c];
    const int64_t b = a.offsets[c], e = a.offsets[c + 1];
    bool bad = false;
    if (!(lam > 0.0) || !isfinite(lam)) { optics_report(a.err, c, kOptErrLambda); bad = true; }
    if (!(nm > 0.0) || !isfinite(nm)) { optics_report(a.err, c, kOptErrNm); bad = true; }
    if (!(km >= 0.0) || !isfinite(km)) { optics_report(a.err, c, kOptErrKm); bad = true; }
    if (b < 0 || e < b || e > a.n_entries) { optics_report(a.err, c, kOptErrOffsets); return; }
    if (bad) return;
    int nmax = 0;
    const double two_pi = 2.0 * 3.141592653589793;
    for (int64_t j = b; j < e; ++j) {
        const double np_ = a.n_p[j], kp = a.k_p[j], r = a.r[j], f = a.f[j];
        if (!(np_ > 0.0) || !isfinite(np_)) { optics_report(a.err, c, kOptErrNp); return; }
        if (!(kp >= 0.0) || !isfinite(kp)) { optics_report(a.err, c, kOptErrKp); return; }
        if (!(r > 0.0) || !isfinite(r)) { optics_report(a.err, c, kOptErrRadius); return; }
        if (!(f >= 0.0) || !isfinite(f)) { optics_report(a.err, c, kOptErrFraction); return; }
        a.cell_of[j] = c;
        const double ay = two_pi * r * sqrt(np_ * np_ + kp * kp) / lam;   // |y| of eq. (1)
        const int nn = series_length(ay) + 1;
        if (nn > nmax) nmax = nn;
    }
    if (nmax > 0) atomicMax(a.nmax, (unsigned int)nmax);
}

__global__ void mie_entries(OpticsArgs a)
{
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nthreads = (size_t)gridDim.x * blockDim.x;
    const double pi = 3.141592653589793;
    for (size_t j = tid; j < (size_t)a.n_entries; j += nthreads) {
        const int c = a.cell_of[j];
        const double lam = a.lam[c], r = a.r[j];
        const cd Nm = mk(a.n_m[c], a.k_m[c]);
        const cd Np = mk(a.n_p[j], a.k_p[j]);
        const double k0r = 2.0 * pi * r / lam;
        const cd x = k0r * Nm;
        const cd m = Np / Nm;
        const cd y = m * x;
        // |y| by the same expression as optics_scan, so the series length
        // never exceeds the scratch the host sized from it
        const double ay = 2.0 * pi * r * sqrt(a.n_p[j] * a.n_p[j] + a.k_p[j] * a.k_p[j]) / lam;
        int nn = series_length(ay) + 1;              // eq. (15) needs a_{nmax+1}
        if (nn > a.nn_cap) nn = a.nn_cap;
        const int nmax = nn - 1;
        // D_n(y), n = 1..nn, downward from far above; stored strided
        cd* D = reinterpret_cast<cd*>(a.scratch) + tid;   // D[n * nthreads]
        int nstart = nn;
        if (ceil(ay) > nstart) nstart = (int)ceil(ay);
        nstart += 16;
        const cd iy = recip(y);
        cd d = mk(0.0, 0.0);
        for (int n = nstart; n > nn; --n) {
            const cd ny = (double)n * iy;
            d = ny - recip(d + ny);
        }
        D[(size_t)nn * nthreads] = d;
        for (int n = nn; n >= 2; --n) {
            const cd ny = (double)n * iy;
            d = ny - recip(d + ny);
            D[(size_t)(n - 1) * nthreads] = d;
        }
        // upward psi_n(x), xi_n(x) = x h_n^(1)(x)
        const cd ix = recip(x);
        const cd sx = csin_(x), cx = ccos_(x);
        cd psi_m1 = cx, psi_0 = sx;
        cd xi_m1 = mk(cx.re - sx.im, cx.im + sx.re);   // cos x + i sin x
        cd xi_0 = mk(sx.re + cx.im, sx.im - cx.re);    // sin x - i cos x
        const cd iNm2 = recip(Nm * Nm);
        const cd im = recip(m);
        double sext = 0.0, ssca = 0.0, sg = 0.0;
        cd a_prev = mk(0.0, 0.0), b_prev = mk(0.0, 0.0);
        bool done = false;
        for (int n = 1; n <= nn && !done; ++n) {
            const double fn = (double)n;
            const cd psi_n = (2.0 * fn - 1.0) * ix * psi_0 - psi_m1;
            const cd xi_n = (2.0 * fn - 1.0) * ix * xi_0 - xi_m1;
            cd an, bn;
            if (!isfinite(xi_n.re) || !isfinite(xi_n.im) || abs2(xi_n) > 1e300) {
                // psi_n/xi_n -> 0 far above |x|: remaining coefficients vanish
                an = mk(0.0, 0.0); bn = mk(0.0, 0.0);
                done = true;
            } else {
                const cd Dn = D[(size_t)n * nthreads];
                const cd nx = fn * ix;
                const cd ta = Dn * im + nx;
                const cd tb = m * Dn + nx;
                an = (ta * psi_n - psi_0) / (ta * xi_n - xi_0);
                bn = (tb * psi_n - psi_0) / (tb * xi_n - xi_0);
            }
            if (n >= 2) {   // cross term of eq. (15) for the pair (n-1, n)
                const double f1 = fn - 1.0;
                sg += f1 * (f1 + 2.0) / (f1 + 1.0) * ((a_prev * conj_(an)).re + (b_prev * conj_(bn)).re);
            }
            if (n <= nmax) {
                sext += (2.0 * fn + 1.0) * ((an + bn) * iNm2).re;
                ssca += (2.0 * fn + 1.0) * (abs2(an) + abs2(bn));
                sg += (2.0 * fn + 1.0) / (fn * (fn + 1.0)) * (an * conj_(bn)).re;
            }
            a_prev = an; b_prev = bn;
            psi_m1 = psi_0; psi_0 = psi_n;
            xi_m1 = xi_0; xi_0 = xi_n;
        }
        // eqs. (10)-(12)
        const double alpha = 4.0 * pi * r * a.k_m[c] / lam;
        double gam;
        if (fabs(alpha) < 1e-3)
            gam = 1.0 + alpha * (2.0 / 3.0 + alpha * (0.25 + alpha * (1.0 / 15.0 + alpha / 72.0)));
        else
            gam = 2.0 * (1.0 + (alpha - 1.0) * exp(alpha)) / (alpha * alpha);
        const double area = pi * r * r;
        const double cext = lam * lam / (2.0 * pi) * sext;
        const double csca = lam * lam * exp(-alpha) / (2.0 * pi * gam * abs2(Nm)) * ssca;
        a.mie[3 * j + 0] = cext / area;
        a.mie[3 * j + 1] = csca / area;
        a.mie[3 * j + 2] = ssca > 0.0 ? 2.0 * sg / ssca : 0.0;
    }
}

__global__ void emt_cells(OpticsArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cells) return;
    const int64_t b = a.offsets[c], e = a.offsets[c + 1];
    double mus = 0.0, mua = 0.0, gs = 0.0, F = 0.0;
    for (int64_t j = b; j < e; ++j) {
        const double qe = a.mie[3 * j], qs = a.mie[3 * j + 1], gi = a.mie[3 * j + 2];
        const double f = a.f[j], r = a.r[j];
        const double ws = 1.5 * qs * f / (2.0 * r);
        mus += ws;
        mua += 1.5 * (qe - qs) * f / (2.0 * r);
        gs += ws * gi;
        F += f;
    }
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
    hipLaunchKernelGGL(optics_scan, dim3((a.n_cells + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mie(const OpticsArgs& a, int grid, int block, hipStream_t st)
{
    if (a.n_entries <= 0) return hipSuccess;
    hipLaunchKernelGGL(mie_entries, dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_emt(const OpticsArgs& a, hipStream_t st)
{
    if (a.n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(emt_cells, dim3((a.n_cells + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace fos
