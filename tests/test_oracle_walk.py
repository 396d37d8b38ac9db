"""Pins of the oracle photon walk (Methodology, Photon transport).

The walk has no closed form in general; it is pinned by
  * exact invariants: photon-count conservation, A = 0 in lossless media,
    T = 1 through index-matched clear layers;
  * the incoherent Beer-Lambert + Fresnel solution of non-scattering stacks
    (multinomial z-tests and chi^2), including an absorbing substrate;
  * g = 1 behaving exactly like no scattering;
  * the thin-slab single-scattering limit R / tau_s -> P_back(g);
  * an independent deterministic adding-doubling solution of the slab
    radiative transfer equation with scattering and Fresnel boundaries.
"""
import math

import numpy as np
import pytest

from rte_adding import _fresnel_unpolarised, slab_rat
from stats import chi2_multinomial, z_bound

TH = 4


def _one(orc, mus, mua, g, n, t, **kw):
    L = len(mus)
    photons = kw.pop("photons", 200_000)
    seed = kw.pop("seed", 11)
    nu, nl, kl, mu0 = kw.pop("n_upper", 1.0), kw.pop("n_lower", 1.0), kw.pop("k_lower", 0.0), kw.pop("mu0", 1.0)
    o = orc.walk_batch([L], [mus], [mua], [g], [n], [t], [nu], [nl], [kl], [mu0], [photons],
                       seed=seed, n_threads=TH, **kw)[0]
    return o, photons


def _adding_stack(n_list, t_list, mua_list, n_upper, n_lower, k_lower, mu0):
    """Incoherent adding of interface and layer elements of a non-scattering
    stack: element = (Rf, Tf, Rb, Tb).  Returns (R_spec, R_diff, A, T)."""
    # direction cosine in each layer from Snell's law
    s = n_upper * math.sqrt(1 - mu0 * mu0)
    cos = [math.sqrt(1 - (s / n) ** 2) for n in n_list]

    def iface(n1, c1, n2, c2, k2=0.0):
        Rf = float(_fresnel_unpolarised(np.array([c1]), n1, n2, k2)[0])
        Rb = float(_fresnel_unpolarised(np.array([c2]), n2, n1)[0]) if k2 == 0.0 else 0.0
        return (Rf, 1 - Rf, Rb, 1 - Rb)

    def add(A, B):
        d = 1 - A[2] * B[0]
        return (A[0] + A[1] * B[0] * A[3] / d, A[1] * B[1] / d,
                B[2] + B[3] * A[2] * B[1] / d, B[3] * A[3] / d)

    top = iface(n_upper, mu0, n_list[0], cos[0])
    tot = top
    for i, (n, t, mua) in enumerate(zip(n_list, t_list, mua_list)):
        tau = math.exp(-mua * t / cos[i])
        tot = add(tot, (0.0, tau, 0.0, tau))
        if i + 1 < len(n_list):
            tot = add(tot, iface(n, cos[i], n_list[i + 1], cos[i + 1]))
    # bottom: into the lower half-space (absorbing substrates never return light)
    if k_lower == 0.0:
        c_lo = math.sqrt(max(0.0, 1 - (s / n_lower) ** 2))
        tot = add(tot, iface(n_list[-1], cos[-1], n_lower, c_lo))
    else:
        Rf = float(_fresnel_unpolarised(np.array([cos[-1]]), n_list[-1], n_lower, k_lower)[0])
        tot = add(tot, (Rf, 1 - Rf, 0.0, 0.0))
    R, T = tot[0], tot[1]
    return top[0], R - top[0], 1 - R - T, T


def _check_multinomial(o, N, probs):
    counts = np.array([o[0], o[1], o[2], o[3]], dtype=np.float64)
    assert o[4] == 0
    assert counts.sum() == N
    for c, p in zip(counts, probs):
        assert abs(c / N - p) <= z_bound(p, N) + 1e-12, (counts / N, probs)
    chi2, dof = chi2_multinomial(counts, probs)
    assert chi2 < dof + 6 * math.sqrt(2 * max(dof, 1)) + 10


@pytest.mark.parametrize("case", [
    dict(n=[1.5], t=[50.0], mua=[0.01]),
    dict(n=[1.5], t=[20.0], mua=[0.05], mu0=0.6),
    dict(n=[1.3], t=[30.0], mua=[0.02], n_upper=1.0, n_lower=1.8),
    dict(n=[1.5], t=[40.0], mua=[0.005], n_lower=3.5, k_lower=0.01),
    dict(n=[1.4, 1.7, 1.5], t=[10.0, 25.0, 5.0], mua=[0.01, 0.0, 0.04], n_lower=3.5, k_lower=0.01,
         mu0=0.8),
])
def test_non_scattering_stack_closed_form(orc, case):
    n, t, mua = case["n"], case["t"], case["mua"]
    L = len(n)
    kw = {k: case[k] for k in ("n_upper", "n_lower", "k_lower", "mu0") if k in case}
    o, N = _one(orc, [0.0] * L, mua, [0.0] * L, n, t, **kw)
    probs = _adding_stack(n, t, mua, kw.get("n_upper", 1.0), kw.get("n_lower", 1.0),
                          kw.get("k_lower", 0.0), kw.get("mu0", 1.0))
    _check_multinomial(o, N, probs)


def test_forward_scattering_g1_equals_no_scattering(orc):
    n, t, mua = [1.5], [50.0], [0.01]
    probs = _adding_stack(n, t, mua, 1.0, 1.0, 0.0, 1.0)
    o, N = _one(orc, [0.7], mua, [1.0], n, t)
    _check_multinomial(o, N, probs)


def test_index_matched_clear_layers_transmit_everything(orc):
    o, N = _one(orc, [0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0], [10.0, 3.0], mu0=0.3,
                photons=5000)
    assert o[3] == N and o[:3].sum() == 0 and o[4] == 0


@pytest.mark.parametrize("mus,g,n_lower,k_lower", [(0.5, 0.8, 1.0, 0.0), (2.0, 0.0, 1.33, 0.0),
                                                    (1.0, 0.5, 2.0, 0.0)])
def test_lossless_conservation_and_zero_absorption(orc, mus, g, n_lower, k_lower):
    o, N = _one(orc, [mus], [0.0], [g], [1.5], [20.0], n_lower=n_lower, k_lower=k_lower,
                photons=20000)
    assert o[2] == 0
    assert o[0] + o[1] + o[3] + o[4] == N
    assert o[4] == 0


def test_conservation_with_absorption_and_cap(orc):
    o, N = _one(orc, [3.0, 1.0], [0.02, 0.1], [0.6, 0.2], [1.5, 1.3], [10.0, 10.0], photons=20000,
                max_steps=50)
    assert o[:5].sum() == N
    assert o[4] > 0                     # some photons reach the cap ...
    assert o[5] <= 50 * N               # ... and no photon takes more steps


@pytest.mark.parametrize("g", [0.0, 0.5, 0.85])
def test_thin_slab_single_scattering_limit(orc, g):
    # tau_s = 5e-3, index matched, lossless: R / tau_s -> P(cos < 0) of HG
    tau = 5e-3
    N = 2_000_000
    o, _ = _one(orc, [tau / 10.0], [0.0], [g], [1.0], [10.0], photons=N)
    pb = 0.5 if g == 0 else (1 - g) / (2 * g) * ((1 + g) / math.sqrt(1 + g * g) - 1)
    R = (o[0] + o[1]) / N
    expect = tau * pb
    assert abs(R - expect) <= z_bound(expect, N) + 0.03 * expect


@pytest.mark.parametrize("tau,omega,g,n,mu0,n_lower,k_lower", [
    (1.0, 0.9, 0.5, 1.0, 1.0, 1.0, 0.0),
    (2.0, 0.95, 0.7, 1.5, 1.0, 1.0, 0.0),
    (0.5, 0.8, -0.3, 1.4, 1.0, 1.0, 0.0),
    (4.0, 0.99, 0.3, 1.5, 0.7, 1.0, 0.0),
    (3.0, 0.97, 0.6, 1.5, 1.0, 3.5, 0.01),
])
def test_scattering_slab_against_adding_doubling(orc, tau, omega, g, n, mu0, n_lower, k_lower):
    t = 1.0
    o, N = _one(orc, [omega * tau / t], [(1 - omega) * tau / t], [g], [n], [t], mu0=mu0,
                n_lower=n_lower, k_lower=k_lower, photons=400_000, seed=5)
    probs = slab_rat(tau, omega, g, n_slab=n, mu0=mu0, n_lower=n_lower, k_lower=k_lower, nodes=48)
    for c, p in zip(o[:4], probs):
        assert abs(c / N - p) <= z_bound(p, N) + 2e-5, (o[:4] / N, probs)


def test_photon_ranges_compose(orc):
    # walking [0, N) equals walking [0, a) plus [a, N) with the same seed
    kw = dict(n_upper=1.0, n_lower=1.2, k_lower=0.0, mu0=0.9, seed=3)
    full = orc.walk([1.0], [0.1], [0.4], [1.5], [5.0], photons=3000, **kw)
    a = orc.walk([1.0], [0.1], [0.4], [1.5], [5.0], photons=1000, **kw)
    b = orc.walk([1.0], [0.1], [0.4], [1.5], [5.0], photons=2000, photon_begin=1000, **kw)
    assert (full == a + b).all()
