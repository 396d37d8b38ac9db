"""Batched uneven items, launch tuning and graph-captured sweeps (GPU)."""
import numpy as np
import pytest

from gpu_helpers import arrays_from_problem, channels, load_golden, make_arrays, run_gpu
from test_gpu_mc import GPU_SEED, _det_problem, _pooled_check

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


def _device_problem_with_gpu_optics(ctx, torch, wl):
    """Workload -> GPU optics -> device transport problem (the product path)."""
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    req = W.optics_request(wl)
    op = fos.OpticsProblem.from_request(req)
    C = op.n_cells
    mus, mua, g = (torch.zeros(C, dtype=torch.float32, device="cuda") for _ in range(3))
    fos.fos_optics_run(ctx, op, mus, mua, g)
    geo = W.item_geometry(wl)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    ph = t(geo["photons"], np.int64)
    if hasattr(torch, "uint64"):
        ph = ph.view(torch.uint64)
    return fos.MCProblem(t(geo["n_layers"], np.int32), mus, mua, g, t(geo["n_layer"], np.float32).reshape(-1),
                         t(geo["thickness"], np.float32).reshape(-1), t(geo["n_upper"], np.float32),
                         t(geo["n_lower"], np.float32), t(geo["k_lower"], np.float32), t(geo["mu0"], np.float32), ph)


def test_autotune_picks_a_valid_launch_and_keeps_results(ctx, torch):
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _det_problem()
    prob = device_problem(a)
    ref = run_gpu(ctx, a, 99)
    fos.fos_mc_prepare(ctx, prob)
    best, ms = fos.fos_mc_autotune(ctx, seed=5, sample_photons=200_000)
    print("autotune:", best, f"{ms:.3f} ms", flush=True)
    assert best["block_size"] % 64 == 0 and 1 <= best["refill_min"] <= 64 and ms > 0
    assert best["tail_lanes"] in (-1, 16)
    assert fos.fos_mc_get_launch(ctx).as_dict() == best
    assert (run_gpu(ctx, a, 99) == ref).all()


def test_autotune_cache_serves_the_class_it_was_tuned_on(torch, tmp_path):
    """The tuned launch is written to the cache under the problem's class; a
    second context with the same cache takes it for a problem of that class
    without trial launches (the recorded time comes back), and a problem of
    another class is tuned afresh and added."""
    import json
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    path = str(tmp_path / "launches.json")
    a = _det_problem()
    with fos.Context(0) as c1:
        fos.fos_mc_autotune_cache(c1.handle, path)
        fos.fos_mc_prepare(c1.handle, device_problem(a))
        best, ms = fos.fos_mc_autotune(c1.handle, seed=5, sample_photons=100_000)
    cache = json.load(open(path))
    assert len(cache) == 1
    (key, entry), = cache.items()
    assert key.startswith("gfx950") and "|L3|" in key
    assert {k: entry[k] for k in best if k in entry} == {k: v for k, v in best.items() if k in entry}
    with fos.Context(0) as c2:
        fos.fos_mc_autotune_cache(c2.handle, path)
        fos.fos_mc_prepare(c2.handle, device_problem(a))
        best2, ms2 = fos.fos_mc_autotune(c2.handle, seed=9, sample_photons=100_000)
        assert best2 == best and abs(ms2 - entry["ms"]) < 1e-3
        assert (run_gpu(c2.handle, a, 99) == run_gpu(c2.handle, a, 99, launch=best)).all()
        b = make_arrays(np.full((20, 1), 2.0), 0.05, 0.7, 1.5, 10.0, photons=50_000)
        fos.fos_mc_prepare(c2.handle, device_problem(b))
        fos.fos_mc_autotune(c2.handle, seed=9, sample_photons=100_000)
    assert len(json.load(open(path))) == 2


def test_graph_sweep_replays_any_seed(ctx, torch):
    from paper_2409_00165_amd import fos
    from gpu_helpers import device_problem
    a = _det_problem()
    prob = device_problem(a)
    I = prob.n_items
    refs = {s: run_gpu(ctx, a, s) for s in (11, 12)}
    fos.fos_mc_prepare(ctx, prob)
    out = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_graph_capture(ctx, out)
    for s in (11, 12, 11):
        out.fill_(-1)
        fos.fos_mc_graph_launch(ctx, s)
        torch.cuda.synchronize()
        assert (out.cpu().numpy().reshape(I, 6) == refs[s]).all(), s
    fos.fos_mc_prepare(ctx, prob)            # re-preparing invalidates the graph
    with pytest.raises(fos.FosError) as ei:
        fos.fos_mc_graph_launch(ctx, 11)
    assert ei.value.status == 6


def test_batched_three_layer_designs_full_budgets(ctx, torch):
    """The batched benchmark sweep at its full size, in the launch the
    benchmark times: 4096 three-layer designs x 100 wavelengths with photon
    budgets log-uniform in [1e4, 1e6] (8.9e10 photons), GPU optics, autotuned
    launch, one graph-captured persistent walk.  The 64 designs of the oracle
    golden (stratified over the budgets, at their own budgets) are checked
    item by item; every item conserves its photons."""
    from paper_2409_00165_amd import fos
    from paper_2409_00165_amd import workloads as W
    wl = W.stacks_3layer(n_designs=4096)
    prob = _device_problem_with_gpu_optics(ctx, torch, wl)
    I = prob.n_items
    fos.fos_mc_prepare(ctx, prob)
    best, ms = fos.fos_mc_autotune(ctx, seed=7)
    print("autotuned launch", best, f"{ms:.2f} ms on the sample", flush=True)
    tal = torch.zeros(I * 6, dtype=torch.int64, device="cuda")
    fos.fos_mc_graph_capture(ctx, tal)
    fos.fos_mc_graph_launch(ctx, GPU_SEED)
    torch.cuda.synchronize()
    t = tal.cpu().numpy().reshape(I, 6)
    N = W.item_geometry(wl)["photons"].astype(np.int64)
    assert (t[:, :5].sum(1) == N).all() and (t[:, 4] == 0).all()
    G = load_golden("stacks_3layer")
    designs = np.asarray(G["designs"], np.int64)
    L = len(wl.wavelengths)
    rows = (designs[:, None] * L + np.arange(L)[None, :]).ravel()
    o = np.asarray(G["tallies"], np.int64)
    No = np.asarray(G["problem"]["photons"], np.int64)
    assert (No == N[rows]).all()
    _pooled_check(channels(t[rows]), N[rows], channels(o), No, "stacks_3layer 4096 designs")
    print("photon-steps:", int(t[:, 5].sum()), "mean per photon", t[:, 5].sum() / N.sum(), flush=True)
