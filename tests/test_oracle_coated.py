"""Pins of the oracle's coated-sphere Mie coefficients (supplementary eqs.
(S1)-(S9)) and of the 101-size Gaussian diameter spread (Scattering
properties section): reductions to the homogeneous sphere, the coated-sphere
Rayleigh limit, lossless extinction, and the size-spread bookkeeping."""
import math

import numpy as np
import pytest


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.mark.parametrize("lam,nm,km,ns,ks,r", [
    (0.5, 1.5, 0.0, 2.0, 0.01, 0.2),
    (0.8, 1.33, 1e-3, 1.45, 0.2, 0.6),
    (2.0, 1.0, 0.0, 3.5, 0.0, 1.0),
])
def test_core_of_shell_material_is_a_homogeneous_sphere(orc, lam, nm, km, ns, ks, r):
    ref = orc.mie_sphere(lam, nm, km, ns, ks, r)
    got = orc.mie_coated(lam, nm, km, ns, ks, 0.55 * r, ns, ks, r)
    for k in range(3):
        assert _rel(got[k], ref[k]) < 1e-11, (got, ref)


@pytest.mark.parametrize("lam,nm,km,nc,kc,ns,ks,r", [
    (0.5, 1.5, 0.0, 1.0, 0.0, 2.0, 0.01, 0.2),
    (0.6, 1.0, 0.0, 3.0, 0.5, 1.45, 0.0, 0.4),
])
def test_vanishing_core_leaves_the_shell_sphere(orc, lam, nm, km, nc, kc, ns, ks, r):
    # core volume 1e-12 of the particle: its effect is far below 1e-9
    ref = orc.mie_sphere(lam, nm, km, ns, ks, r)
    got = orc.mie_coated(lam, nm, km, nc, kc, 1e-4 * r, ns, ks, r)
    for k in range(3):
        assert _rel(got[k], ref[k]) < 1e-9, (got, ref)


@pytest.mark.parametrize("lam,nm,km,nc,kc,ns,ks,rc", [
    (0.5, 1.5, 0.0, 2.0, 0.01, 1.0, 0.0, 0.2),
    (1.2, 1.33, 1e-4, 2.5, 0.3, 1.45, 0.1, 0.5),
])
def test_vanishing_shell_leaves_the_core_sphere(orc, lam, nm, km, nc, kc, ns, ks, rc):
    ref = orc.mie_sphere(lam, nm, km, nc, kc, rc)
    got = orc.mie_coated(lam, nm, km, nc, kc, rc, ns, ks, rc * (1 + 1e-10))
    for k in range(3):
        assert _rel(got[k], ref[k]) < 1e-7, (got, ref)


@pytest.mark.parametrize("m1,m2,q", [(1.0 + 0j, 1.5 + 0.1j, 0.5), (2.0 + 0.5j, 1.3 + 0j, 0.8),
                                     (1.5 + 0j, 1.5 + 0j, 0.3)])
def test_coated_rayleigh_limit(orc, m1, m2, q):
    """Small coated sphere: Q_sca -> 8/3 y^4 |P|^2 and Q_abs -> 4 y Im P with
    the coated-sphere polarizability (per unit volume times 3 / (4 pi))
    P = [(e2 - 1)(e1 + 2 e2) + f (e1 - e2)(1 + 2 e2)] /
        [(e2 + 2)(e1 + 2 e2) + 2 f (e2 - 1)(e1 - e2)],  e = m^2, f = q^3."""
    lam, r = 1.0, 1e-4
    y = 2 * math.pi * r / lam
    e1, e2, f = m1 ** 2, m2 ** 2, q ** 3
    P = ((e2 - 1) * (e1 + 2 * e2) + f * (e1 - e2) * (1 + 2 * e2)) / \
        ((e2 + 2) * (e1 + 2 * e2) + 2 * f * (e2 - 1) * (e1 - e2))
    qext, qsca, g, _ = orc.mie_coated(lam, 1.0, 0.0, m1.real, m1.imag, q * r, m2.real, m2.imag, r)
    assert _rel(qsca, 8.0 / 3.0 * y ** 4 * abs(P) ** 2) < 1e-4
    if P.imag > 0:
        assert _rel(qext - qsca, 4 * y * P.imag) < 1e-4
    assert abs(g) < 1e-3


@pytest.mark.parametrize("nc,ns,q,lam", [(1.0, 1.45, 0.7, 0.5), (2.6, 1.5, 0.4, 0.9)])
def test_lossless_coated_sphere_extinguishes_by_scattering(orc, nc, ns, q, lam):
    qext, qsca, _, _ = orc.mie_coated(lam, 1.0, 0.0, nc, 0.0, q * 0.5, ns, 0.0, 0.5)
    assert abs(qext - qsca) <= 1e-10 * qext


def test_coated_coefficients_literal_against_spherical_bessels(orc):
    """The recurrences behind the literal form against scipy's spherical
    Bessel functions (moderate complex arguments)."""
    from scipy.special import spherical_jn, spherical_yn
    x, y = 2.0, 3.1
    m1, m2 = 1.2 + 0.05j, 1.7 + 0.02j
    nmax = 12
    a, b = orc.mie_coated_coeffs(x, y, m1, m2, nmax)
    psi = lambda n, z: z * spherical_jn(n, z)
    chi = lambda n, z: z * spherical_yn(n, z)
    dpsi = lambda n, z: spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)
    dchi = lambda n, z: spherical_yn(n, z) + z * spherical_yn(n, z, derivative=True)
    for n in range(1, nmax + 1):
        An = (m2 * psi(n, m2 * x) * dpsi(n, m1 * x) - m1 * dpsi(n, m2 * x) * psi(n, m1 * x)) / \
             (m2 * chi(n, m2 * x) * dpsi(n, m1 * x) - m1 * dchi(n, m2 * x) * psi(n, m1 * x))
        ua = dpsi(n, m2 * y) - An * dchi(n, m2 * y)
        va = psi(n, m2 * y) - An * chi(n, m2 * y)
        xi = psi(n, y) + 1j * chi(n, y)
        dxi = dpsi(n, y) + 1j * dchi(n, y)
        an = (psi(n, y) * ua - m2 * dpsi(n, y) * va) / (xi * ua - m2 * dxi * va)
        assert abs(a[n - 1] - an) <= 1e-10 * max(abs(an), 1e-30) + 1e-15, n


def test_gaussian_sizes_bookkeeping(orc):
    r, w = orc.gaussian_sizes(0.4, 0.05)
    assert len(r) == 101
    assert abs(w.sum() - 1.0) < 1e-14
    d = 2 * r
    assert abs(d[0] - (0.4 - 0.15)) < 1e-14 and abs(d[-1] - (0.4 + 0.15)) < 1e-14
    assert abs((w * d).sum() - 0.4) < 1e-14                     # symmetric about D
    sd = math.sqrt((w * (d - 0.4) ** 2).sum())
    assert 0.95 * 0.05 < sd < 0.05                              # truncated at 3 sigma
    r0, w0 = orc.gaussian_sizes(0.4, 0.0)
    assert len(r0) == 1 and r0[0] == 0.2 and w0[0] == 1.0
    rn, wn = orc.gaussian_sizes(0.1, 0.05)                      # diameters <= 0 left out
    assert len(rn) == 84 and rn.min() > 0 and abs(wn.sum() - 1) < 1e-14


def test_layer_optics_ex_reduces_to_layer_optics(orc):
    args = (0.7, 1.5, 1e-4, [2.5, 1.45], [1e-3, 0.01], [0.2, 0.35], [0.05, 0.1])
    ref = orc.layer_optics(*args)
    assert orc.layer_optics_ex(*args) == ref
    assert orc.layer_optics_ex(*args, sd=[0.0, 0.0], r_core=[0.0, 0.0], n_core=[1, 1], k_core=[0, 0]) == ref


def test_narrow_gaussian_spread_is_one_size(orc):
    args = (0.7, 1.5, 0.0, [2.5], [1e-3], [0.2], [0.05])
    ref = orc.layer_optics(*args)
    got = orc.layer_optics_ex(*args, sd=[1e-7])
    for a, b in zip(got, ref):
        assert _rel(a, b) < 1e-8
