"""Pins of the oracle's asymmetry parameter and effective-medium assembly
that do not reduce to zero on both sides (Methodology, Scattering
properties, eqs. (11)-(20)).

* eq. (15): g of a single sphere against the mean cosine of its phase
  function, |S1|^2 + |S2|^2 integrated over the scattering angle by
  Gauss-Legendre quadrature, with a_n, b_n from a direct SciPy Bessel
  evaluation and the angular functions pi_n, tau_n from derivatives of
  Legendre polynomials (numpy); the same integral gives Q_sca (eq. (12) in a
  real host), so both the series and its prefactors are pinned away from the
  Rayleigh limit;
* eq. (16): g of a mixture is weighted by each population's scattering
  coefficient -- an index-matched second population (which scatters
  nothing) leaves g unchanged for any volume fraction, and two scattering
  populations give the mu_s-weighted mean of their own g;
* eq. (20): particles with the host's own complex index (no contrast, so
  q_ext = q_sca = 0) leave mu_a = 4 pi k_m (1 - sum f) / lambda exactly,
  unscaled by the dependent-scattering factor even above the threshold;
* eqs. (17)-(19): the factor C = 1 + 1.5 F - 0.75 F^2 of the two benchmark
  slabs' total volume fractions, 1.1425 at F = 0.10 and 1.182325 at
  F = 0.13, recovered from the oracle's own single-population optics.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy.special import spherical_jn, spherical_yn

from paper_2409_00165_amd import workloads as W


def _ab_scipy(x, m, nmax):
    """Lorenz-Mie a_n, b_n (n = 1..nmax) of a sphere of relative index m at
    size parameter x, from Riccati-Bessel functions psi = z j_n(z) and
    xi = z h_n^(1)(z) evaluated by SciPy (eqs. (2)-(5) with the host index
    folded into x)."""
    n = np.arange(1, nmax + 1)
    y = m * x
    psi = lambda z: z * spherical_jn(n, z)
    dpsi = lambda z: spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)
    h = lambda z: spherical_jn(n, z) + 1j * spherical_yn(n, z)
    dh = lambda z: spherical_jn(n, z, derivative=True) + 1j * spherical_yn(n, z, derivative=True)
    xi = lambda z: z * h(z)
    dxi = lambda z: h(z) + z * dh(z)
    a = (m * psi(y) * dpsi(x) - psi(x) * dpsi(y)) / (m * psi(y) * dxi(x) - xi(x) * dpsi(y))
    b = (psi(y) * dpsi(x) - m * psi(x) * dpsi(y)) / (psi(y) * dxi(x) - m * xi(x) * dpsi(y))
    return a, b


def _phase_function_moments(a, b, n_nodes):
    """Integral over mu = cos(theta) in [-1, 1] of |S1|^2 + |S2|^2 and of mu
    times it.  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n), S2 likewise with
    pi and tau swapped; pi_n(mu) = P_n'(mu), tau_n(mu) = mu P_n'(mu) -
    (1 - mu^2) P_n''(mu).  Gauss-Legendre with n_nodes nodes is exact for the
    polynomial integrand once n_nodes > nmax + 1."""
    mu, w = npleg.leggauss(n_nodes)
    S1 = np.zeros_like(mu, dtype=complex)
    S2 = np.zeros_like(mu, dtype=complex)
    for k in range(1, len(a) + 1):
        P = npleg.Legendre.basis(k)
        d1, d2 = P.deriv(1)(mu), P.deriv(2)(mu)
        pi_k = d1
        tau_k = mu * d1 - (1.0 - mu * mu) * d2
        c = (2.0 * k + 1.0) / (k * (k + 1.0))
        S1 += c * (a[k - 1] * pi_k + b[k - 1] * tau_k)
        S2 += c * (a[k - 1] * tau_k + b[k - 1] * pi_k)
    I = np.abs(S1) ** 2 + np.abs(S2) ** 2
    return float(np.sum(w * I)), float(np.sum(w * mu * I))


@pytest.mark.parametrize("x", [0.5, 3.0, 10.0])
@pytest.mark.parametrize("m", [1.5 + 0.0j, 1.5 + 0.1j, 2.4 + 0.01j, 1.1 + 0.0j])
def test_asymmetry_equals_phase_function_mean_cosine(orc, x, m):
    # host 1.33 (real), lam 0.55 um: r from x = 2 pi r n_m / lam
    n_m, lam = 1.33, 0.55
    r = x * lam / (2.0 * math.pi * n_m)
    n_p = m * n_m
    qe, qs, g, nmax = orc.mie_sphere(lam, n_m, 0.0, n_p.real, n_p.imag, r)
    nterm = int(nmax) + 12                  # past the series' own cut-off
    a, b = _ab_scipy(complex(x), complex(m), nterm)
    i0, i1 = _phase_function_moments(a, b, nterm + 8)
    assert g == pytest.approx(i1 / i0, rel=1e-8, abs=1e-12)
    # the same integral is the scattering efficiency: Q_sca = (1/x^2) int I dmu
    assert qs == pytest.approx(i0 / (x * x), rel=1e-8)
    # and a forward-peaked phase function gives g > 0 away from Rayleigh
    if x >= 3.0:
        assert g > 0.1


def test_asymmetry_of_strongly_absorbing_sphere(orc):
    # a metal-like sphere backscatters: g from the series equals the phase
    # function's mean cosine, including its sign
    n_m, lam, x, m = 1.0, 0.5, 1.2, 0.3 + 3.0j
    r = x * lam / (2.0 * math.pi * n_m)
    _, qs, g, nmax = orc.mie_sphere(lam, n_m, 0.0, m.real, m.imag, r)
    a, b = _ab_scipy(complex(x), m, int(nmax) + 12)
    i0, i1 = _phase_function_moments(a, b, int(nmax) + 20)
    assert g == pytest.approx(i1 / i0, rel=1e-8, abs=1e-12)
    assert qs == pytest.approx(i0 / (x * x), rel=1e-8)


@pytest.mark.parametrize("f2", [1e-3, 0.05, 0.3])
def test_index_matched_population_does_not_weight_g(orc, f2):
    # population 2 has the matrix index: it scatters and absorbs nothing, so
    # by eq. (16) (weights q_sca f / r) the mixture's g is population 1's,
    # whatever its volume fraction; a volume-fraction weighting would give
    # g1 f1 / (f1 + f2)
    lam, n_m = 0.7, 1.5
    one = orc.layer_optics(lam, n_m, 0.0, [2.6], [1e-3], [0.3], [0.05])
    mix = orc.layer_optics(lam, n_m, 0.0, [2.6, n_m], [1e-3, 0.0], [0.3, 0.2], [0.05, f2])
    assert one[2] > 0.2
    assert mix[2] == pytest.approx(one[2], rel=1e-12)
    F = 0.05 + f2
    C = 1 + 1.5 * F - 0.75 * F * F if F > 0.08 else 1.0
    assert mix[0] == pytest.approx(C * one[0], rel=1e-12)


def test_mixture_g_is_scattering_weighted_mean(orc):
    # two scattering populations with very different g (small and large
    # spheres), total volume fraction below the threshold and a clear matrix:
    # mu_s adds and g is the mu_s-weighted mean of the populations' own g
    lam, n_m = 0.6, 1.4
    p1 = orc.layer_optics(lam, n_m, 0.0, [2.5], [1e-3], [0.04], [0.03])
    p2 = orc.layer_optics(lam, n_m, 0.0, [2.5], [1e-3], [1.5], [0.04])
    mix = orc.layer_optics(lam, n_m, 0.0, [2.5, 2.5], [1e-3, 1e-3], [0.04, 1.5], [0.03, 0.04])
    assert abs(p1[2] - p2[2]) > 0.3          # the populations differ in g
    assert mix[0] == pytest.approx(p1[0] + p2[0], rel=1e-12)
    assert mix[1] == pytest.approx(p1[1] + p2[1], rel=1e-12)
    assert mix[2] == pytest.approx((p1[0] * p1[2] + p2[0] * p2[2]) / (p1[0] + p2[0]), rel=1e-12)


@pytest.mark.parametrize("F", [0.05, 0.2, 0.5])
def test_matrix_absorption_with_contrast_free_particles(orc, F):
    # particles of the host's own complex index have no Mie coefficients
    # (m = 1), so mu_s = 0 and mu_a is the matrix term of eq. (20) alone:
    # 4 pi k_m (1 - F) / lambda -- scaled by the volume the matrix fills and
    # not by the dependent-scattering factor, even for F above 0.08
    lam, n_m, k_m = 0.9, 1.45, 1e-3
    mus, mua, g = orc.layer_optics(lam, n_m, k_m, [n_m, n_m], [k_m, k_m], [0.15, 0.6], [0.4 * F, 0.6 * F])
    assert abs(mus) < 1e-12 * mua
    assert mua == pytest.approx(4.0 * math.pi * k_m * (1.0 - F) / lam, rel=1e-10)


def _species_entries(species, f_total, lam):
    r, w = W.lognormal_bins(0.25, 0.3, 20)
    n, k = W.SPECIES[species](np.array([lam]))
    return [n[0]] * len(r), [k[0]] * len(r), list(r), list(f_total * w)


@pytest.mark.parametrize("lam", [0.45, 1.0, 4.0])
def test_dependent_scattering_factor_single_slab(orc, lam):
    # single 50 um slab: species A, r = 0.2 um, f = 0.10 > 0.08 -> C = 1.1425;
    # at f = 0.05 no factor applies, and the particle terms are linear in f
    hi = orc.layer_optics(lam, 1.5, 0.0, [2.5 + 0.1 / lam**2], [1e-3], [0.2], [0.10])
    lo = orc.layer_optics(lam, 1.5, 0.0, [2.5 + 0.1 / lam**2], [1e-3], [0.2], [0.05])
    assert hi[0] / (2.0 * lo[0]) == pytest.approx(1.1425, rel=1e-12)
    assert hi[1] / (2.0 * lo[1]) == pytest.approx(1.1425, rel=1e-12)
    assert hi[2] == pytest.approx(lo[2], rel=1e-12)


@pytest.mark.parametrize("lam", [0.5, 2.0, 9.0])
def test_dependent_scattering_factor_two_species_slab(orc, lam):
    # the 500 um slab: species A at 0.08 and B at 0.05 (total 0.13 -> C =
    # 1.182325), each population alone at or below the threshold (0.08 is
    # not above it, so no factor); the matrix term is checked separately, so
    # k_m = 0 here
    a = _species_entries("A", 0.08, lam)
    b = _species_entries("B", 0.05, lam)
    oa = orc.layer_optics(lam, 1.5, 0.0, *a)
    ob = orc.layer_optics(lam, 1.5, 0.0, *b)
    mix = orc.layer_optics(lam, 1.5, 0.0, *(x + y for x, y in zip(a, b)))
    assert mix[0] / (oa[0] + ob[0]) == pytest.approx(1.182325, rel=1e-12)
    assert mix[1] / (oa[1] + ob[1]) == pytest.approx(1.182325, rel=1e-12)
