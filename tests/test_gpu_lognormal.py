"""Log-normal populations on a shared radius grid (fos_optics_lognormal):
against the FP64 oracle's per-entry effective medium, against the GPU's own
per-entry path (fos_optics_run) on the same designs, the per-item arrays of a
paint problem, and validation."""
import numpy as np
import pytest

from paper_2409_00165_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2409_00165_amd import fos
    c = fos.Context(0)
    yield c.handle
    c.close()


def _lognormal(ctx, torch, sweep):
    from paper_2409_00165_amd import surrogate_pipeline as SP
    prob = SP.paint_problem(ctx, sweep)
    torch.cuda.synchronize()
    T = prob.tensors
    return prob, np.stack([T[k].cpu().numpy().astype(np.float64) for k in ("mu_s", "mu_a", "g")], 1)


def _errors(ref, got):
    """mu_s, mu_a relative to the cell's extinction; g absolute where the cell
    scatters."""
    ext = np.maximum(ref[:, 0] + ref[:, 1], 1e-300)
    e_s = np.abs(got[:, 0] - ref[:, 0]) / ext
    e_a = np.abs(got[:, 1] - ref[:, 1]) / ext
    e_g = np.where(ref[:, 0] > 1e-9 * ext, np.abs(got[:, 2] - ref[:, 2]), 0.0)
    return e_s.max(), e_a.max(), e_g.max()


def test_lognormal_matches_oracle(ctx, torch, orc):
    sweep = W.paint_sweep(40, n_lambda=60, seed=5)
    _, got = _lognormal(ctx, torch, sweep)
    mus, mua, g = orc.workload_optics(sweep.workload())
    ref = np.stack([mus[:, 0], mua[:, 0], g[:, 0]], 1)
    e = _errors(ref, got)
    print("lognormal grid vs oracle (float outputs):", e, flush=True)
    assert e[0] < 1e-6 and e[1] < 1e-6 and e[2] < 1e-6


def test_lognormal_full_sweep_sampled(ctx, torch, orc):
    """The paint sweep at full size in one call (10^6 designs x 200
    wavelengths = 2e8 cells): 64 designs drawn at random, all their
    wavelengths, against the oracle's per-entry effective medium."""
    from paper_2409_00165_amd import surrogate_pipeline as SP
    L = 200
    sweep = W.paint_sweep(1_000_000, n_lambda=L)
    prob = SP.paint_problem(ctx, sweep)
    assert prob.n_items == 1_000_000 * L
    designs = np.sort(np.random.default_rng(21).choice(1_000_000, size=64, replace=False))
    rows = torch.from_numpy((designs[:, None] * L + np.arange(L)[None, :]).ravel()).cuda()
    got = np.stack([prob.tensors[k][rows].cpu().numpy().astype(np.float64) for k in ("mu_s", "mu_a", "g")], 1)
    del prob
    torch.cuda.empty_cache()
    mus, mua, g = orc.workload_optics(sweep.workload(designs))
    ref = np.stack([mus[:, 0], mua[:, 0], g[:, 0]], 1)
    e = _errors(ref, got)
    print("full sweep, 64 sampled designs vs oracle (float outputs):", e, flush=True)
    assert e[0] < 1e-6 and e[1] < 1e-6 and e[2] < 1e-6


def test_lognormal_equals_per_entry_path(ctx, torch):
    from paper_2409_00165_amd import surrogate_pipeline as SP
    sweep = W.paint_sweep(300, n_lambda=100, seed=6)
    _, got = _lognormal(ctx, torch, sweep)
    per = SP.optics_problem(ctx, sweep.workload())
    torch.cuda.synchronize()
    ref = np.stack([per.tensors[k].cpu().numpy().astype(np.float64) for k in ("mu_s", "mu_a", "g")], 1)
    e = _errors(ref, got)
    print("lognormal grid vs per-entry GPU path:", e, flush=True)
    assert e[0] < 1e-6 and e[1] < 1e-6 and e[2] < 1e-6


def test_paint_problem_items(ctx, torch):
    sweep = W.paint_sweep(25, n_lambda=30, seed=7, photons=12345)
    prob, _ = _lognormal(ctx, torch, sweep)
    T = {k: v.cpu().numpy() for k, v in prob.tensors.items() if k != "photons"}
    L = 30
    assert prob.n_items == 25 * L and prob.max_layers == 1
    assert (T["n_layers"] == 1).all()
    assert np.array_equal(T["n_layer"], np.repeat(W.PAINT_NM[sweep.matrix].astype(np.float32), L))
    assert np.array_equal(T["thickness"], np.repeat(sweep.thickness.astype(np.float32), L))
    assert (T["n_upper"] == 1).all() and (T["n_lower"] == 1).all() and (T["k_lower"] == 0).all()
    assert (T["mu0"] == 1).all()
    assert (prob.tensors["photons"].view(torch.int64).cpu().numpy() == 12345).all()


@pytest.mark.parametrize("field,value,word", [("species", 2, "species"), ("matrix", -1, "matrix"),
                                              ("rmed", 34, "median"), ("f", 1.5, "f ")])
def test_lognormal_rejects_bad_designs(ctx, torch, field, value, word):
    from paper_2409_00165_amd import fos
    sweep = W.paint_sweep(8, n_lambda=10, seed=8)
    arrays = {"species": sweep.species.copy(), "matrix": sweep.matrix.copy(), "rmed": sweep.rmed.copy(),
              "f": sweep.f.copy()}
    arrays[field][3] = value
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    lp = fos.LognormalProblem(**sweep.lognormal_tables(), species=dev(arrays["species"], np.int32),
                              matrix=dev(arrays["matrix"], np.int32), rmed=dev(arrays["rmed"], np.int32),
                              f=dev(arrays["f"], np.float64))
    out = [torch.full((80,), 7.0, device="cuda") for _ in range(3)]
    with pytest.raises(fos.FosError) as ei:
        fos.fos_optics_lognormal(ctx, lp, *out)
    assert "design 3" in str(ei.value) and word in str(ei.value)
    torch.cuda.synchronize()
    assert all(bool((o == 7.0).all()) for o in out)
