"""Pins of the oracle's weighted-packet walk (MCML form with Russian
roulette): closed forms of non-scattering stacks, exact lossless bookkeeping,
an independent adding-doubling RTE solution, and agreement in expectation
with the analog walk.  Tolerances use the estimator's own variance (from the
per-photon sums of squares) at 4 standard errors."""
import math

import numpy as np
import pytest

from rte_adding import slab_rat
from test_oracle_walk import _adding_stack


def _w(orc, mus, mua, g, n, t, n_upper=1.0, n_lower=1.0, k_lower=0.0, mu0=1.0, photons=200_000, seed=11):
    L = len(n)
    o, st = orc.walk_weighted_batch([L], [mus], [mua], [g], [n], [t], [n_upper], [n_lower], [k_lower], [mu0],
                                    [photons], seed=seed)
    return o[0], st[0], photons


def _estimates(o, N):
    """(R_spec, R_diff, A, T) means and the standard errors of R_diff, A, T."""
    mean = o[:4] / N
    var = np.array([o[4] / N - mean[1] ** 2, o[5] / N - mean[2] ** 2, o[6] / N - mean[3] ** 2])
    return mean, np.sqrt(np.maximum(var, 0.0) / N)


@pytest.mark.parametrize("case", [
    dict(n=[1.5], t=[50.0], mua=[0.01]),
    dict(n=[1.3], t=[30.0], mua=[0.02], n_lower=1.8, mu0=0.7),
    dict(n=[1.4, 1.7, 1.5], t=[10.0, 25.0, 5.0], mua=[0.01, 0.0, 0.04], n_lower=3.5, k_lower=0.01, mu0=0.8),
])
def test_weighted_non_scattering_stack_closed_form(orc, case):
    # without scattering a packet deposits its whole weight at its first
    # interaction, so the weighted walk is the analog one: same closed form
    n, t, mua = case["n"], case["t"], case["mua"]
    L = len(n)
    kw = {k: case[k] for k in ("n_lower", "k_lower", "mu0") if k in case}
    o, st, N = _w(orc, [0.0] * L, mua, [0.0] * L, n, t, **kw)
    probs = _adding_stack(n, t, mua, 1.0, kw.get("n_lower", 1.0), kw.get("k_lower", 0.0), kw.get("mu0", 1.0))
    mean, se = _estimates(o, N)
    assert abs(mean[0] - probs[0]) < 1e-12           # specular part is deterministic
    for k in range(3):
        assert abs(mean[k + 1] - probs[k + 1]) <= 4 * se[k] + 1e-12, (mean, probs)
    assert o[7] == 0 and st[1] == 0                    # no roulette, no cap


@pytest.mark.parametrize("mus,g,n_lower", [(0.5, 0.8, 1.0), (2.0, 0.0, 1.33), (1.0, -0.4, 2.0)])
def test_weighted_lossless_conserves_every_packet(orc, mus, g, n_lower):
    o, st, N = _w(orc, [mus], [0.0], [g], [1.5], [20.0], n_lower=n_lower, photons=20_000)
    assert o[2] == 0.0 and o[5] == 0.0                 # nothing deposited
    assert o[7] == 0                                   # weights never drop, no roulette
    assert abs(o[0] + o[1] + o[3] - N) < 1e-9 * N      # every packet leaves whole


@pytest.mark.parametrize("tau,omega,g,n,mu0,n_lower,k_lower", [
    (1.0, 0.9, 0.5, 1.0, 1.0, 1.0, 0.0),
    (2.0, 0.95, 0.7, 1.5, 1.0, 1.0, 0.0),
    (4.0, 0.99, 0.3, 1.5, 0.7, 1.0, 0.0),
    (3.0, 0.6, 0.6, 1.5, 1.0, 3.5, 0.01),
])
def test_weighted_against_adding_doubling(orc, tau, omega, g, n, mu0, n_lower, k_lower):
    o, st, N = _w(orc, [omega * tau], [(1 - omega) * tau], [g], [n], [1.0], mu0=mu0, n_lower=n_lower,
                  k_lower=k_lower, photons=300_000, seed=5)
    probs = slab_rat(tau, omega, g, n_slab=n, mu0=mu0, n_lower=n_lower, k_lower=k_lower, nodes=48)
    mean, se = _estimates(o, N)
    assert abs(mean[0] - probs[0]) < 1e-12
    for k in range(3):
        assert abs(mean[k + 1] - probs[k + 1]) <= 4 * se[k] + 2e-5, (mean, probs)


@pytest.mark.parametrize("mus,mua,g,t", [(1.0, 0.1, 0.5, 10.0), (20.0, 0.02, 0.9, 5.0), (0.3, 0.3, 0.0, 8.0)])
def test_weighted_agrees_with_analog_in_expectation(orc, mus, mua, g, t):
    N = 200_000
    o, st, _ = _w(orc, [mus], [mua], [g], [1.5], [t], photons=N, seed=21)
    a = orc.walk_batch([1], [[mus]], [[mua]], [[g]], [[1.5]], [[t]], [1.0], [1.0], [0.0], [1.0], [N], seed=22)[0]
    mean, se = _estimates(o, N)
    pa = np.array([a[0] + a[1], a[2], a[3]], dtype=np.float64) / N
    pw = np.array([mean[0] + mean[1], mean[2], mean[3]])
    se_a = np.sqrt(pa * (1 - pa) / N)
    for k in range(3):
        assert abs(pw[k] - pa[k]) <= 4 * math.hypot(se[k], se_a[k]) + 1e-12, (pw, pa)
    # every photon either leaves or is stopped by roulette; the total weight
    # balances in expectation (roulette adds or removes weight at random)
    assert abs(o[:4].sum() / N - 1.0) < 4 * max(se.max(), 1e-4)
