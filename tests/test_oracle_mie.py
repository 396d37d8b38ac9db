"""Pins of the oracle's Mie theory and effective-medium assembly
(Methodology, Scattering properties, eqs. (1)-(20)).

* a_n, b_n against a direct evaluation of eqs. (2)-(5) with SciPy's
  spherical Bessel functions (complex arguments, moderate size);
* Rayleigh limit: Q_sca -> 8/3 x^4 |K|^2, Q_abs -> 4 x Im K, g -> 0;
* large-sphere limit: Q_ext -> 2 with the x^(-2/3) edge correction;
* lossless sphere in a lossless host: Q_ext = Q_sca;  m -> 1: Q -> 0;
* absorbing host: gamma -> 1 as k_m -> 0 (eq. (10)) and continuity of the
  cross sections in k_m;
* effective medium: the matrix-only absorption 4 pi k / lambda, invariance
  under splitting a population, geometric-optics extinction 3 f / (2 r) for
  large spheres, and a log-normal of vanishing width reducing to one size.
"""
import math

import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

from paper_2409_00165_amd import workloads as W


def _direct_ab(x, m, nmax):
    """Eqs. (2)-(5) with psi = z j_n, xi = z h_n^(1) from SciPy."""
    n = np.arange(1, nmax + 1)
    y = m * x

    def psi(z):
        return z * spherical_jn(n, z)

    def dpsi(z):
        return spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)

    def xi(z):
        return z * (spherical_jn(n, z) + 1j * spherical_yn(n, z))

    def dxi(z):
        h = spherical_jn(n, z) + 1j * spherical_yn(n, z)
        dh = spherical_jn(n, z, derivative=True) + 1j * spherical_yn(n, z, derivative=True)
        return h + z * dh

    nm = 1.0          # host index folded into x
    npart = m
    A_y, A_x, B_x = dpsi(y) / psi(y), dpsi(x) / psi(x), dxi(x) / xi(x)
    pre = psi(x) / xi(x)
    a = pre * (nm * A_y - npart * A_x) / (nm * A_y - npart * B_x)
    b = pre * (npart * A_y - nm * A_x) / (npart * A_y - nm * B_x)
    return a, b


@pytest.mark.parametrize("x,m", [(0.3, 1.5 + 0.01j), (3.0, 1.5 + 0.01j), (10.0, 2.5 + 0.1j),
                                 (5.0 + 0.01j, 1.7 + 0.002j), (25.0, 1.33 + 1e-4j),
                                 (8.0, 0.8 + 2.0j), (10 * math.pi, 1.5 + 0.1j),
                                 (4 * math.pi, 1.5 + 0.0j)])
def test_coefficients_match_direct_bessel_evaluation(orc, x, m):
    nmax = orc.mie_nmax(abs(m * x)) + 1
    a, b = orc.mie_coeffs(complex(x), complex(m), nmax)
    ad, bd = _direct_ab(complex(x), complex(m), nmax)
    assert np.max(np.abs(a - ad)) < 1e-10
    assert np.max(np.abs(b - bd)) < 1e-10


@pytest.mark.parametrize("m", [1.5 + 0.1j, 2.5 + 0.001j, 1.33 + 0.0j])
def test_rayleigh_limit(orc, m):
    x = 1e-3
    # lam = 2 pi, host index 1  =>  x = r
    qe, qs, g, _ = orc.mie_sphere(2 * math.pi, 1.0, 0.0, m.real, m.imag, x)
    K = (m * m - 1) / (m * m + 2)
    assert qs / (8.0 / 3.0 * x**4 * abs(K) ** 2) == pytest.approx(1.0, abs=1e-5)
    if m.imag > 0:
        assert (qe - qs) / (4 * x * K.imag) == pytest.approx(1.0, abs=1e-5)
    assert abs(g) < 1e-5


@pytest.mark.parametrize("x", [1000.0, 800 * math.pi, 4000.0, 20000.0])
def test_large_sphere_extinction_paradox(orc, x):
    # absorbing sphere: Q_ext = 2 + c x^(-2/3) + ..., c ~ 2 (edge term)
    qe, qs, g, _ = orc.mie_sphere(2 * math.pi, 1.0, 0.0, 1.5, 0.1, x)
    corr = (qe - 2.0) * x ** (2.0 / 3.0)
    assert 1.5 < corr < 2.5
    qe_r, qs_r, _, _ = orc.mie_sphere(2 * math.pi, 1.0, 0.0, 1.5, 0.0, x)
    assert abs(qe_r - 2.0) < 3.0 * x ** (-2.0 / 3.0)


@pytest.mark.parametrize("x,m", [(0.5, 1.5), (4.0, 2.0), (30.0, 1.33)])
def test_lossless_sphere_extinction_equals_scattering(orc, x, m):
    qe, qs, g, _ = orc.mie_sphere(2 * math.pi, 1.0, 0.0, m, 0.0, x)
    assert abs(qe - qs) <= 1e-12 * qe


def test_index_match_gives_no_scattering(orc):
    qe, qs, g, _ = orc.mie_sphere(0.5, 1.5, 0.0, 1.5, 0.0, 0.3)
    assert abs(qe) < 1e-14 and abs(qs) < 1e-14
    # Rayleigh-Gans regime: Q_sca grows as (m - 1)^2 near m = 1
    q1 = orc.mie_sphere(0.5, 1.5, 0.0, 1.5 * (1 + 1e-4), 0.0, 0.3)[1]
    q2 = orc.mie_sphere(0.5, 1.5, 0.0, 1.5 * (1 + 2e-4), 0.0, 0.3)[1]
    assert q2 / q1 == pytest.approx(4.0, rel=1e-3)


def test_absorbing_host_geometric_term(orc):
    assert orc.gamma_term(0.0) == 1.0
    # eq. (10) series vs closed form at the switch-over and beyond
    for a in (1e-3 * 0.999, 1e-3 * 1.001, 0.01, 0.5, 3.0):
        closed = 2 * (1 + (a - 1) * math.exp(a)) / a**2
        assert orc.gamma_term(a) == pytest.approx(closed, rel=1e-9)
    # continuity of the cross sections as k_m -> 0
    q0 = orc.mie_sphere(0.6, 1.5, 0.0, 2.5, 1e-3, 0.3)
    q1 = orc.mie_sphere(0.6, 1.5, 1e-9, 2.5, 1e-3, 0.3)
    assert q1[0] == pytest.approx(q0[0], rel=1e-7)
    assert q1[1] == pytest.approx(q0[1], rel=1e-7)
    assert q1[2] == pytest.approx(q0[2], rel=1e-7)


def test_effective_medium_matrix_only(orc):
    mus, mua, g = orc.layer_optics(0.5, 1.5, 1e-4, [], [], [], [])
    assert mus == 0.0 and g == 0.0
    assert mua == pytest.approx(4 * math.pi * 1e-4 / 0.5, rel=1e-14)


def test_effective_medium_population_split_invariance(orc):
    one = orc.layer_optics(0.7, 1.5, 1e-4, [2.6], [1e-3], [0.2], [0.06])
    two = orc.layer_optics(0.7, 1.5, 1e-4, [2.6, 2.6], [1e-3, 1e-3], [0.2, 0.2], [0.03, 0.03])
    assert np.allclose(one, two, rtol=1e-13)
    # crossing the 8 % threshold scales the particle terms by C (eq. 17)
    lo = orc.layer_optics(0.7, 1.5, 0.0, [2.6], [1e-3], [0.2], [0.08])
    hi = orc.layer_optics(0.7, 1.5, 0.0, [2.6, 2.6], [1e-3, 1e-3], [0.2, 0.2], [0.08, 1e-12])
    F = 0.08 + 1e-12
    assert hi[0] / lo[0] == pytest.approx(1 + 1.5 * F - 0.75 * F * F, rel=1e-9)


def test_effective_medium_geometric_optics_limit(orc):
    # large opaque spheres: mu_ext -> 2 * (projected area per volume) = 3 f/(2 r)
    f, r = 0.01, 200.0
    mus, mua, g = orc.layer_optics(0.5, 1.0, 0.0, [1.5], [0.1], [r], [f])
    assert (mus + mua) == pytest.approx(3 * f / (2 * r), rel=0.01)


def test_lognormal_narrow_width_reduces_to_one_size(orc):
    r1, w1 = W.lognormal_bins(0.25, 1e-6, 20)
    a = orc.layer_optics(0.6, 1.5, 1e-4, [2.7] * 20, [1e-3] * 20, r1, 0.05 * w1)
    b = orc.layer_optics(0.6, 1.5, 1e-4, [2.7], [1e-3], [0.25], [0.05])
    assert np.allclose(a, b, rtol=1e-5)
    assert w1.sum() == pytest.approx(1.0, abs=1e-14)


def test_workload_optics_shapes_and_ranges(orc):
    wl = W.single_slab_23()
    mus, mua, g = orc.workload_optics(wl, n_threads=4)
    assert mus.shape == (23, 1)
    assert (mus > 0).all() and (mua > 0).all() and ((g > -1) & (g < 1)).all()
