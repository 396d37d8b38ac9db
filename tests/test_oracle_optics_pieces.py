"""Pins of the oracle's Fresnel reflectance and Henyey-Greenstein sampler."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("n1,n2", [(1.0, 1.5), (1.5, 1.0), (1.33, 2.4), (1.0, 1.0)])
def test_fresnel_normal_incidence(orc, n1, n2):
    assert orc.fresnel(1.0, n1, n2) == pytest.approx(((n1 - n2) / (n1 + n2)) ** 2, abs=1e-15)


@pytest.mark.parametrize("ni,n,k", [(1.0, 3.5, 0.01), (1.5, 0.2, 3.0), (1.2, 1.4, 0.5)])
def test_fresnel_complex_normal_incidence(orc, ni, n, k):
    N = n + 1j * k
    assert orc.fresnel(1.0, ni, n, k) == pytest.approx(abs((ni - N) / (ni + N)) ** 2, rel=1e-13)


def test_fresnel_matches_snell_angle_form(orc):
    # r_s = -sin(ti-tt)/sin(ti+tt), r_p = tan(ti-tt)/tan(ti+tt)
    for ni, nt in [(1.0, 1.5), (1.5, 1.0), (1.45, 2.3)]:
        for ci in np.linspace(0.05, 0.999, 23):
            ti = math.acos(ci)
            st = ni / nt * math.sin(ti)
            if st >= 1:
                assert orc.fresnel(ci, ni, nt) == 1.0
                continue
            tt = math.asin(st)
            R = 0.5 * ((math.sin(ti - tt) / math.sin(ti + tt)) ** 2
                       + (math.tan(ti - tt) / math.tan(ti + tt)) ** 2)
            assert orc.fresnel(ci, ni, nt) == pytest.approx(R, rel=1e-11, abs=1e-14)


def test_fresnel_brewster_and_grazing(orc):
    n1, n2 = 1.0, 1.5
    tb = math.atan(n2 / n1)  # p-polarised reflectance vanishes
    ci = math.cos(tb)
    tt = math.asin(n1 / n2 * math.sin(tb))
    rs2 = (math.sin(tb - tt) / math.sin(tb + tt)) ** 2
    assert orc.fresnel(ci, n1, n2) == pytest.approx(0.5 * rs2, rel=1e-12)
    assert orc.fresnel(0.0, n1, n2) == pytest.approx(1.0, abs=1e-15)


def test_fresnel_total_internal_reflection_and_reciprocity(orc):
    n1, n2 = 1.5, 1.0
    c_crit = math.sqrt(1 - (n2 / n1) ** 2)
    assert orc.fresnel(c_crit * 0.999, n1, n2) == 1.0
    # Stokes reciprocity: R(theta_i, a->b) = R(theta_t, b->a)
    for ci in (0.2, 0.5, 0.9):
        st = 1.0 / 1.5 * math.sqrt(1 - ci * ci)
        ct = math.sqrt(1 - st * st)
        assert orc.fresnel(ci, 1.0, 1.5) == pytest.approx(orc.fresnel(ct, 1.5, 1.0), rel=1e-12)


def _hg_moments(orc, g, n=200000):
    u = (np.arange(n) + 0.5) / n   # midpoint rule over the inverse CDF
    c = np.array([orc.hg_cos(g, x) for x in u])
    return c.mean(), (0.5 * (3 * c * c - 1)).mean(), c


@pytest.mark.parametrize("g", [0.0, 1e-4, 0.3, 0.9, -0.5])
def test_hg_legendre_moments(orc, g):
    # HG phase function has Legendre moments g^l: E[cos] = g, E[P2] = g^2
    m1, m2, _ = _hg_moments(orc, g)
    assert m1 == pytest.approx(g, abs=2e-5)
    assert m2 == pytest.approx(g * g, abs=2e-5)


def test_hg_cdf_closed_form(orc):
    # P(cos < 0) = (1-g)/(2g) ((1+g)/sqrt(1+g^2) - 1)
    for g in (0.2, 0.6, 0.85):
        _, _, c = _hg_moments(orc, g, 100000)
        pb = (1 - g) / (2 * g) * ((1 + g) / math.sqrt(1 + g * g) - 1)
        assert (c < 0).mean() == pytest.approx(pb, abs=2e-5)


def test_hg_degenerate(orc):
    assert orc.hg_cos(1.0, 0.0) == 1.0 and orc.hg_cos(1.0, 0.7) == 1.0
    assert orc.hg_cos(-1.0, 0.3) == -1.0
    assert orc.hg_cos(0.0, 0.25) == -0.5
