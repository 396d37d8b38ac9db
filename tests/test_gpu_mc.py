"""GPU parity tests of the HIP photon walk against the FP64 CPU oracle.

All calls go through the C ABI (paper_2409_00165_amd.fos -> libfos_mc.so).
Statistical bar (per wavelength and channel R, A, T): the GPU and oracle
proportions agree within 4 pooled binomial standard errors,
4 sqrt(p(1-p)(1/N1 + 1/N2)) -- at 1e6 photons each this is <= 2.9e-3.
Integer work (generator words, conservation, determinism) is bit-exact.
"""
import math

import numpy as np
import pytest

from gpu_helpers import (arrays_from_problem, channels, load_golden, make_arrays, run_gpu,
                         run_oracle)
from rte_adding import slab_rat
from stats import pooled_bound, z_bound
from test_oracle_walk import _adding_stack

pytestmark = pytest.mark.gpu

GPU_SEED = 0x6A11_0002


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2409_00165_amd import fos
    c = fos.Context(0)
    yield c.handle
    c.close()


def _pooled_check(g_counts, n_g, o_counts, n_o, label, k=4.0, alpha=1e-3):
    """Two independent samples of every (item, channel) proportion agree
    within k pooled binomial standard errors.  Under exact agreement each
    channel exceeds k with probability P(|z| > k) (6.3e-5 at k = 4), so a
    comparison of m channels sees about m * 6.3e-5 such channels by chance:
    0.1 on a 500-wavelength spectrum, about 1 on 6400 items.  The test
    therefore allows as many channels beyond k as a Poisson count of that
    mean reaches with probability 1 - alpha, and none beyond the
    family-wise bound k_fw (every channel inside it with probability 1 -
    alpha); the aggregate chi^2 over all channels bounds the rest."""
    from scipy.stats import norm, poisson
    g_counts = np.asarray(g_counts, np.float64); o_counts = np.asarray(o_counts, np.float64)
    n_g = np.asarray(n_g, np.float64)[:, None]; n_o = np.asarray(n_o, np.float64)[:, None]
    d = np.abs(g_counts / n_g - o_counts / n_o)
    se = pooled_bound(g_counts, n_g, o_counts, n_o, k=1.0)
    both_zero = (g_counts == 0) & (o_counts == 0)
    live = (se > 0) & ~both_zero
    z = np.where(live, d / np.where(live, se, 1.0), 0.0)
    m = int(live.sum())
    k_fw = max(k, float(norm.isf(alpha / (2 * max(m, 1)))))
    beyond = int((z > k).sum())
    allowed = int(poisson.ppf(1.0 - alpha, m * 2 * norm.sf(k)))
    worst = np.unravel_index(np.argmax(z), z.shape)
    chi2, dof = float((z[live] ** 2).sum()), m
    print(f"{label}: max |dp| = {d.max():.3e}, max z = {z.max():.2f} at {worst}; {beyond} of {m} channels "
          f"beyond {k:g} SE (allowed {allowed}), family-wise bound {k_fw:.2f}; chi2 = {chi2:.1f} over {dof}",
          flush=True)
    assert ((z <= k_fw) | ~live).all(), f"{label}: channel beyond {k_fw:.2f} pooled SE at {worst}"
    assert beyond <= allowed, f"{label}: {beyond} channels beyond {k:g} pooled SE (allowed {allowed})"
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def test_philox_words_bit_exact(ctx, torch, orc):
    from paper_2409_00165_amd import fos
    rng = np.random.default_rng(5)
    n = 4096
    photon = rng.integers(0, 2**63, n, dtype=np.int64)
    photon[:8] = [0, 1, 2**32 - 1, 2**32, 2**40 + 7, 2**63 - 1, 12345, 99]
    step = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    stream = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    seed = 0xDEADBEEF_12345678
    dp = torch.from_numpy(photon).cuda()
    ds = torch.from_numpy(step.view(np.int32)).cuda()
    dstr = torch.from_numpy(stream.view(np.int32)).cuda()
    out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    fos.fos_philox_words(ctx, dp, ds, dstr, seed, out)
    torch.cuda.synchronize()
    words = out.cpu().numpy().view(np.uint32).reshape(n, 4)
    for j in range(0, n, 17):
        p = int(photon[j])
        ref = orc.philox([p & 0xFFFFFFFF, p >> 32, int(step[j]), int(stream[j])],
                         [seed & 0xFFFFFFFF, seed >> 32])
        assert list(words[j]) == ref, j


def test_fresnel_device_matches_oracle(ctx, torch, orc):
    from paper_2409_00165_amd import fos
    cases = []
    for ni, nt, kt in [(1.0, 1.5, 0.0), (1.5, 1.0, 0.0), (1.5, 1.33, 0.0), (1.3, 1.7, 0.0),
                       (1.5, 3.5, 0.01), (1.5, 0.2, 3.0), (1.45, 1.45, 0.0), (1.6, 2.4, 0.5)]:
        for c in np.linspace(0.0, 1.0, 201):
            cases.append((c, ni, nt, kt))
    a = np.array(cases, np.float32)
    cols = [torch.from_numpy(np.ascontiguousarray(a[:, i])).cuda() for i in range(4)]
    out = torch.zeros(len(a), dtype=torch.float32, device="cuda")
    fos.fos_eval_fresnel(ctx, *cols, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = np.array([orc.fresnel(float(c), float(ni), float(nt), float(kt)) for c, ni, nt, kt in a])
    err = np.abs(got - ref)
    print("fresnel max abs err", err.max(), flush=True)
    assert err.max() < 3e-6
    # total internal reflection clear of the critical angle: exactly 1 on the
    # device too (its TIR branch); within a few FP32 ulp of the critical
    # cosine the float ratio m = ni/nt may put the device on the other side,
    # where R is continuous and tends to 1, and at grazing incidence (c = 0)
    # R = 1 comes out of the approximate reciprocal and square root (~1 ulp)
    c, ni, nt, kt = (a[:, i].astype(np.float64) for i in range(4))
    s2t = (ni / nt) ** 2 * (1.0 - c * c)
    tir = (kt == 0) & (c > 0) & (s2t >= 1.0 + 1e-5)
    assert tir.sum() > 50 and (ref[tir] == 1.0).all()
    assert (got[tir] == 1.0).all()
    graze = (c == 0) | (np.abs(s2t - 1.0) < 1e-5)
    assert (got[ref == 1.0] >= 1.0 - 3e-6).all() and (np.abs(got[graze] - ref[graze]) < 3e-6).all()


def test_hg_device_matches_oracle(ctx, torch, orc):
    from paper_2409_00165_amd import fos
    gs = [0.0, 1e-4, 0.3, 0.9, -0.5, 0.99, -0.99, 0.999, 1.0, -1.0]
    us = (np.arange(2048) / 2048.0).astype(np.float32)
    G = np.repeat(np.array(gs, np.float32), len(us))
    U = np.tile(us, len(gs))
    out = torch.zeros(len(G), dtype=torch.float32, device="cuda")
    fos.fos_eval_hg(ctx, torch.from_numpy(G).cuda(), torch.from_numpy(U).cuda(), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = np.array([orc.hg_cos(float(g), float(u)) for g, u in zip(G, U)])
    err = np.abs(got - ref)
    print("hg max abs err per g", [float(err[i * 2048:(i + 1) * 2048].max()) for i in range(len(gs))],
          flush=True)
    assert err.max() < 2e-6
    # Legendre moments of the device sampler over a fine midpoint grid
    for g in (0.0, 1e-4, 0.3, 0.9, -0.5):
        u = ((np.arange(1 << 16) + 0.5) / (1 << 16)).astype(np.float32)
        o = torch.zeros(len(u), dtype=torch.float32, device="cuda")
        fos.fos_eval_hg(ctx, torch.full((len(u),), g, dtype=torch.float32, device="cuda"),
                        torch.from_numpy(u).cuda(), o)
        torch.cuda.synchronize()
        c = o.cpu().numpy().astype(np.float64)
        assert abs(c.mean() - g) < 1e-4
        assert abs((0.5 * (3 * c * c - 1)).mean() - g * g) < 1e-4


# ---------------------------------------------------------------------------
# boundary behaviour
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("field,value,layer", [
    ("mu_s", -1.0, 1), ("mu_a", float("nan"), 0), ("g", 1.5, 0), ("n_layer", 0.9, 1),
    ("thickness", 0.0, 0), ("n_upper", 0.5, None), ("mu0", 0.0, None), ("k_lower", -0.1, None),
    ("n_layers", 3, None),
])
def test_invalid_problem_is_rejected_without_side_effects(ctx, torch, field, value, layer):
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = make_arrays([[1.0, 2.0]] * 4, 0.01, 0.5, 1.5, 10.0, photons=100)
    if layer is None:
        a[field][2] = value
    else:
        a[field][2, layer] = value
    prob = device_problem(a)
    tal = torch.full((4 * 6,), 77, dtype=torch.int64, device="cuda")
    with pytest.raises(fos.FosError) as ei:
        fos.fos_mc_run(ctx, prob, 1, tal)
    assert ei.value.status == 1
    msg = str(ei.value)
    assert "item 2" in msg and field in msg, msg
    torch.cuda.synchronize()
    assert (tal.cpu().numpy() == 77).all()


def test_bad_launch_and_unprepared(ctx, torch):
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = make_arrays([[1.0]], 0.0, 0.0, 1.5, 10.0, photons=10)
    prob = device_problem(a)
    tal = torch.zeros(6, dtype=torch.int64, device="cuda")
    for bad in ({"block_size": 96}, {"refill_min": 65}, {"blocks_per_cu": 100}, {"max_steps": 1 << 33}):
        with pytest.raises(fos.FosError) as ei:
            fos.fos_mc_run(ctx, prob, 1, tal, launch=bad)
        assert ei.value.status == 1


def test_empty_batch_and_zero_photon_items(ctx, torch):
    a = make_arrays([[1.0], [1.0], [0.5]], 0.1, 0.3, 1.5, 10.0, photons=[0, 2000, 0])
    t = run_gpu(ctx, a, 3)
    assert (t[0] == 0).all() and (t[2] == 0).all()
    assert t[1, :5].sum() == 2000
    e = make_arrays(np.zeros((0, 1)), 0.0, 0.0, 1.5, 1.0)
    assert run_gpu(ctx, e, 3).shape == (0, 6)


def test_invariants_conservation_lossless_clear(ctx, torch):
    # item 0: lossless scattering -> A = 0;  item 1: index-matched clear
    # layers -> T = N;  item 2: absorbing multi-layer;  item 3: conductor below
    a = make_arrays([[0.5, 2.0, 0.0], [0.0, 0.0, 0.0], [3.0, 1.0, 0.2], [1.0, 0.0, 0.5]],
                    [[0, 0, 0], [0, 0, 0], [0.02, 0.1, 0.0], [0.01, 0.0, 0.1]],
                    [[0.8, 0.0, 0.5], [0, 0, 0], [0.6, 0.2, -0.3], [0.3, 0.0, 0.9]],
                    [[1.5, 1.3, 1.7], [1.0, 1.0, 1.0], [1.5, 1.3, 1.4], [1.4, 1.4, 1.6]],
                    [[20.0, 5.0, 1.0], [10.0, 3.0, 1.0], [10.0, 10.0, 4.0], [3.0, 7.0, 2.0]],
                    n_lower=[1.0, 1.0, 1.33, 0.2], k_lower=[0, 0, 0, 3.0], mu0=[1.0, 0.3, 0.8, 0.6],
                    photons=50_000)
    t = run_gpu(ctx, a, 9)
    assert (t[:, :5].sum(1) == 50_000).all()
    assert t[0, 2] == 0 and t[0, 4] == 0
    assert t[1, 3] == 50_000
    assert (t[:, 4] == 0).all()


def test_step_cap(ctx, torch, orc):
    a = make_arrays([[3.0, 1.0]], [[0.02, 0.1]], [[0.6, 0.2]], [[1.5, 1.3]], [[10.0, 10.0]],
                    photons=20000)
    t = run_gpu(ctx, a, 4, launch={"max_steps": 50})[0]
    assert t[:5].sum() == 20000 and t[4] > 0 and t[5] <= 50 * 20000
    o = run_oracle(orc, a, 5, max_steps=50)[0]
    _pooled_check(np.array([[t[0] + t[1], t[2], t[3], t[4]]]), [20000],
                  np.array([[o[0] + o[1], o[2], o[3], o[4]]]), [20000], "capped")


# ---------------------------------------------------------------------------
# closed forms and the deterministic RTE solution
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    dict(n=[1.5], t=[50.0], mua=[0.01]),
    dict(n=[1.5], t=[20.0], mua=[0.05], mu0=0.6),
    dict(n=[1.3], t=[30.0], mua=[0.02], n_upper=1.0, n_lower=1.8),
    dict(n=[1.5], t=[40.0], mua=[0.005], n_lower=3.5, k_lower=0.01),
    dict(n=[1.4, 1.7, 1.5], t=[10.0, 25.0, 5.0], mua=[0.01, 0.0, 0.04], n_lower=3.5, k_lower=0.01, mu0=0.8),
])
def test_non_scattering_closed_form_gpu(ctx, torch, case):
    n, t, mua = case["n"], case["t"], case["mua"]
    L = len(n)
    kw = {k: case[k] for k in ("n_upper", "n_lower", "k_lower", "mu0") if k in case}
    N = 1_000_000
    a = make_arrays([[0.0] * L], [mua], [[0.0] * L], [n], [t], photons=N, **kw)
    tal = run_gpu(ctx, a, 21)[0]
    probs = _adding_stack(n, t, mua, kw.get("n_upper", 1.0), kw.get("n_lower", 1.0), kw.get("k_lower", 0.0),
                          kw.get("mu0", 1.0))
    assert tal[:4].sum() == N and tal[4] == 0
    for c, p in zip(tal[:4], probs):
        assert abs(c / N - p) <= z_bound(p, N) + 1e-6, (tal[:4] / N, probs)


@pytest.mark.parametrize("tau,omega,g,n,mu0,n_lower,k_lower", [
    (1.0, 0.9, 0.5, 1.0, 1.0, 1.0, 0.0),
    (2.0, 0.95, 0.7, 1.5, 1.0, 1.0, 0.0),
    (0.5, 0.8, -0.3, 1.4, 1.0, 1.0, 0.0),
    (4.0, 0.99, 0.3, 1.5, 0.7, 1.0, 0.0),
    (3.0, 0.97, 0.6, 1.5, 1.0, 3.5, 0.01),
    (10.0, 0.999, 0.8, 1.5, 1.0, 1.0, 0.0),
])
def test_scattering_slab_against_adding_doubling_gpu(ctx, torch, tau, omega, g, n, mu0, n_lower, k_lower):
    N = 2_000_000
    a = make_arrays([[omega * tau]], [[(1 - omega) * tau]], [[g]], [[n]], [[1.0]], mu0=mu0,
                    n_lower=n_lower, k_lower=k_lower, photons=N)
    tal = run_gpu(ctx, a, 22)[0]
    probs = slab_rat(tau, omega, g, n_slab=n, mu0=mu0, n_lower=n_lower, k_lower=k_lower, nodes=48)
    print("gpu", tal[:4] / N, "adding-doubling", np.round(probs, 6), flush=True)
    for c, p in zip(tal[:4], probs):
        assert abs(c / N - p) <= z_bound(p, N) + 5e-5


# ---------------------------------------------------------------------------
# parity with the oracle on the workloads
# ---------------------------------------------------------------------------

def test_parity_single_slab_23(ctx, torch, orc):
    G = load_golden("single_slab_23")
    a = arrays_from_problem(G["problem"])
    o = np.asarray(G["tallies"], np.int64)
    t = run_gpu(ctx, a, GPU_SEED)
    N = a["photons"]
    assert (t[:, :5].sum(1) == N).all()
    _pooled_check(channels(t), N, channels(o), N, "single_slab_23")
    # the same seed on both sides walks the same photons: the outcome counts
    # then differ only through photons whose paths FP32 and FP64 round apart
    t_same = run_gpu(ctx, a, G["oracle_seed"])
    frac = np.abs(channels(t_same) - channels(o)).max(1) / N
    print("same-seed max |dcount|/N per item:", frac.max(), flush=True)
    assert frac.max() <= 5e-3


def test_parity_two_species_500_full_size(ctx, torch):
    """500 wavelengths x 1e6 photons (the benchmark workload and launch)."""
    G = load_golden("two_species_500")
    a = arrays_from_problem(G["problem"])
    o = np.asarray(G["tallies"], np.int64)
    t = run_gpu(ctx, a, GPU_SEED)
    N = a["photons"]
    assert (t[:, :5].sum(1) == N).all() and (t[:, 4] == 0).all()
    _pooled_check(channels(t), N, channels(o), N, "two_species_500")
    steps_g, steps_o = t[:, 5].sum(), o[:, 5].sum()
    print("mean steps/photon gpu", steps_g / N.sum(), "oracle", steps_o / N.sum(), flush=True)
    assert abs(steps_g / steps_o - 1) < 2e-3


def test_parity_stacks_3layer(ctx, torch):
    G = load_golden("stacks_3layer")
    a = arrays_from_problem(G["problem"])
    o = np.asarray(G["tallies"], np.int64)
    t = run_gpu(ctx, a, GPU_SEED)
    N = a["photons"]
    assert (t[:, :5].sum(1) == N).all()
    _pooled_check(channels(t), N, channels(o), N, "stacks_3layer")


# ---------------------------------------------------------------------------
# determinism and graph capture
# ---------------------------------------------------------------------------

def _det_problem():
    rng = np.random.default_rng(3)
    I = 37
    a = make_arrays(rng.uniform(0, 3, (I, 3)), rng.uniform(0, 0.2, (I, 3)), rng.uniform(-0.5, 0.95, (I, 3)),
                    rng.uniform(1.0, 1.8, (I, 3)), rng.uniform(0.5, 20, (I, 3)),
                    n_upper=1.0, n_lower=rng.uniform(1, 3.5, I), k_lower=np.where(rng.uniform(size=I) < 0.5, 0.0, 0.02),
                    mu0=rng.uniform(0.2, 1.0, I), photons=rng.integers(0, 30000, I),
                    n_layers=rng.integers(1, 4, I))
    return a


def test_bit_identical_across_launch_configs(ctx, torch):
    a = _det_problem()
    ref = run_gpu(ctx, a, 1234)
    for launch in ({"block_size": 64, "refill_min": 1, "chunk": 1, "blocks_per_cu": 1},
                   {"block_size": 1024, "refill_min": 64, "chunk": 37, "blocks_per_cu": 2},
                   {"block_size": 256, "refill_min": 8, "chunk": 1 << 20, "blocks_per_cu": 8},
                   {"block_size": 512, "refill_min": 32, "chunk": 4096, "blocks_per_cu": 4},
                   {"tail_lanes": -1}, {"tail_lanes": 1}, {"tail_lanes": 64},
                   {"block_size": 64, "refill_min": 3, "chunk": 5, "blocks_per_cu": 1, "tail_lanes": 40}):
        t = run_gpu(ctx, a, 1234, launch=launch)
        assert (t == ref).all(), launch
    assert (run_gpu(ctx, a, 1234) == ref).all()
    assert not (run_gpu(ctx, a, 1235) == ref).all()


def _heavy_tail_problem(layers):
    """Thick, weakly absorbing slabs (walks of 1e4..1e6 steps, many beyond a
    cap of 5e4) mixed with thin ones, so that the end of a launch is a few
    long walks in otherwise idle waves."""
    rng = np.random.default_rng(41)
    I = 48
    tau = np.where(np.arange(I) % 3 == 0, rng.uniform(300, 1500, I), rng.uniform(0.1, 20, I))
    t = np.full((I, layers), 100.0 / layers)
    return make_arrays(np.repeat(tau[:, None] / 100.0, layers, 1), np.full((I, layers), 1e-7),
                       rng.uniform(-0.2, 0.9, (I, layers)), rng.uniform(1.0, 1.6, (I, layers)), t,
                       n_lower=rng.uniform(1, 2, I), k_lower=np.where(np.arange(I) % 4 == 0, 0.01, 0.0),
                       mu0=rng.uniform(0.5, 1.0, I), photons=rng.integers(200, 3000, I))


@pytest.mark.parametrize("layers", [1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_tail_draws_prepared_across_lanes_are_bit_identical(ctx, torch, layers, weighted):
    """At the end of a launch, a wave with no photons left to claim and few in
    flight computes their next draws on all its lanes ahead of time (any
    tail_lanes threshold, or never): the tallies are the same bits, including
    the photons stopped by the step cap."""
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _heavy_tail_problem(layers)
    prob = device_problem(a)
    nt = fos.N_TALLY_W if weighted else fos.N_TALLY
    run = fos.fos_mc_run_weighted if weighted else fos.fos_mc_run
    outs = []
    for tail in (-1, 1, 4, 8, 16, 33, 64):
        tal = torch.full((prob.n_items * nt,), -1, dtype=torch.int64, device="cuda")
        run(ctx, prob, 777, tal, launch={"tail_lanes": tail, "max_steps": 50_000, "chunk": 64})
        torch.cuda.synchronize()
        outs.append(tal.cpu().numpy().reshape(prob.n_items, nt))
    for o in outs[1:]:
        assert (o == outs[0]).all()
    t = outs[0]
    capped = t[:, 8] if weighted else t[:, 4]
    steps = t[:, 9] if weighted else t[:, 5]
    print("capped photons", int(capped.sum()), "max mean steps per photon", float((steps / a["photons"]).max()),
          flush=True)
    assert capped.sum() > 0 and (steps / a["photons"]).max() > 1e3


def _heavy_tail_bulk(layers):
    """The heavy-tailed items with 30 times the photons (2.3e6), so that
    every wave of the default grid is busy when the queue runs out."""
    a = dict(_heavy_tail_problem(layers))
    a["photons"] = a["photons"] * 30
    return a


@pytest.mark.parametrize("layers", [1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_regrouped_drain_is_bit_identical(ctx, torch, layers, weighted):
    """Waves left with few photons once the queue is empty hand them to
    other waves through the hand-off list (regroup_lanes), with and without
    prepared draws and on other grids: every photon continues with the same
    draws, so the tallies are the same bits as the plain walk's, capped
    photons included.  Photons were handed off, and none was lost."""
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _heavy_tail_bulk(layers)
    prob = device_problem(a)
    nt = fos.N_TALLY_W if weighted else fos.N_TALLY
    run = fos.fos_mc_run_weighted if weighted else fos.fos_mc_run
    base = {"max_steps": 50_000, "chunk": 64}
    configs = [{"tail_lanes": -1, "regroup_lanes": -1}, {"tail_lanes": -1, "regroup_lanes": 4},
               {"tail_lanes": -1, "regroup_lanes": 16}, {"tail_lanes": 16, "regroup_lanes": 16},
               {"tail_lanes": 16, "regroup_lanes": 32, "blocks_per_cu": 16},
               {"tail_lanes": 8, "regroup_lanes": 8, "block_size": 128}]
    outs, handed = [], []
    for cfg in configs:
        print("regroup case", layers, weighted, cfg, flush=True)
        tal = torch.full((prob.n_items * nt,), -1, dtype=torch.int64, device="cuda")
        run(ctx, prob, 4242, tal, launch={**base, **cfg})
        torch.cuda.synchronize()
        outs.append(tal.cpu().numpy().reshape(prob.n_items, nt))
        h, lost = fos.fos_mc_handoff_counts(ctx)
        assert lost == 0, cfg
        handed.append(h if cfg["regroup_lanes"] > 0 else 0)
    print("photons handed off per config", handed, flush=True)
    for o, cfg in zip(outs[1:], configs[1:]):
        assert (o == outs[0]).all(), cfg
    assert min(handed[1:]) > 0
    t = outs[0]
    if not weighted:
        assert (t[:, :5].sum(1) == a["photons"]).all()
    assert (t[:, 8] if weighted else t[:, 4]).sum() > 0


def test_regrouped_walk_full_size_bit_identical(ctx, torch):
    """The benchmark slab (500 wavelengths x 1e6 photons) in the tail build
    with regrouping gives the plain walk's tallies bit for bit."""
    from paper_2409_00165_amd import fos
    G = load_golden("two_species_500")
    a = arrays_from_problem(G["problem"])
    plain = run_gpu(ctx, a, 91)
    grouped = run_gpu(ctx, a, 91, launch={"tail_lanes": 16, "regroup_lanes": 16})
    h, lost = fos.fos_mc_handoff_counts(ctx)
    print("photons handed off", h, flush=True)
    assert lost == 0 and h > 0
    assert np.array_equal(plain, grouped)


def test_regrouped_graph_replays_match_eager(ctx, torch):
    """A captured regrouping walk (its hand-off list reset by a kernel inside
    the graph) replays to the eager tallies, with eager work between."""
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _heavy_tail_bulk(1)
    prob = device_problem(a)
    I = prob.n_items
    L = {"tail_lanes": 16, "regroup_lanes": 16, "max_steps": 50_000, "chunk": 64}
    eager = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_run(ctx, prob, 5, eager, launch=L)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    out = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_graph_capture(ctx, out, launch=L)
    for rep in range(3):
        out.fill_(-5)
        junk = torch.randn(1000, device="cuda").sum()
        fos.fos_mc_graph_launch(ctx, 5)
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == ref).all(), rep
        assert fos.fos_mc_handoff_counts(ctx)[1] == 0
        del junk


def test_regroup_lanes_are_validated(ctx, torch):
    from paper_2409_00165_amd import fos
    a = _det_problem()
    for bad in (-2, 33):
        with pytest.raises(fos.FosError, match="regroup_lanes"):
            run_gpu(ctx, a, 1, launch={"regroup_lanes": bad})


def test_per_problem_chunk_keeps_results(torch):
    """A fresh context sizes the claim chunk per problem when no chunk is
    given (small batches get smaller chunks); an explicit launch chunk and a
    chunk fixed with fos_mc_set_launch are used as given.  The tallies are
    the same bits in every case."""
    from paper_2409_00165_amd import fos
    a = _det_problem()
    with fos.Context(0) as c:
        auto = run_gpu(c.handle, a, 99)
        assert fos.fos_mc_get_launch(c.handle).chunk == 2048
        for chunk in (2048, 256, 3):
            assert (run_gpu(c.handle, a, 99, launch={"chunk": chunk}) == auto).all(), chunk
        fos.fos_mc_set_launch(c.handle, {"chunk": 512})
        assert fos.fos_mc_get_launch(c.handle).chunk == 512
        assert (run_gpu(c.handle, a, 99) == auto).all()


def test_single_layer_build_matches_general_build(ctx, torch):
    """Problems whose items all have one layer run a build of the walk without
    the layer-change code.  The same items padded to three layer slots (still
    one layer each) run the general build; both forms of the walk must give
    the same tallies bit for bit."""
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    rng = np.random.default_rng(12)
    I = 24
    cols = [rng.uniform(0.05, 20, I), rng.uniform(1e-3, 0.5, I), rng.uniform(-0.5, 0.95, I),
            rng.uniform(1.0, 1.8, I), rng.uniform(1.0, 30.0, I)]
    kw = dict(n_lower=np.where(rng.uniform(size=I) < 0.5, 1.0, 3.5),
              k_lower=np.where(rng.uniform(size=I) < 0.5, 0.0, 0.02), mu0=rng.uniform(0.3, 1.0, I),
              photons=rng.integers(1000, 20000, I))
    one = make_arrays(*[c[:, None] for c in cols], **kw)
    three = make_arrays(*[np.repeat(c[:, None], 3, axis=1) for c in cols], n_layers=1, **kw)
    assert one["mu_s"].shape[1] == 1 and three["mu_s"].shape[1] == 3
    assert np.array_equal(run_gpu(ctx, one, 77), run_gpu(ctx, three, 77))
    w = []
    for a in (one, three):
        prob = device_problem(a)
        tal = torch.zeros(I * fos.N_TALLY_W, dtype=torch.int64, device="cuda")
        fos.fos_mc_run_weighted(ctx, prob, 78, tal)
        torch.cuda.synchronize()
        w.append(tal.cpu().numpy())
    assert np.array_equal(w[0], w[1])


def test_graph_capture_replays_match_eager(ctx, torch):
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _det_problem()
    prob = device_problem(a)
    I = prob.n_items
    eager = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_run(ctx, prob, 77, eager)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    out = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_prepare(ctx, prob)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            fos.fos_mc_execute(ctx, 77, out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-5)
        junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert (out.cpu().numpy() == ref).all(), rep
        del junk


def test_max_layers_eight(ctx, torch, orc):
    L = 8
    rng = np.random.default_rng(8)
    a = make_arrays(rng.uniform(0, 2, (3, L)), rng.uniform(0, 0.05, (3, L)), rng.uniform(0, 0.9, (3, L)),
                    rng.uniform(1.0, 1.7, (3, L)), rng.uniform(1, 5, (3, L)), n_lower=1.5, photons=200_000,
                    n_layers=[8, 5, 1])
    t = run_gpu(ctx, a, 31)
    o = run_oracle(orc, a, 32)
    N = a["photons"]
    _pooled_check(channels(t), N, channels(o), N, "eight_layers")
