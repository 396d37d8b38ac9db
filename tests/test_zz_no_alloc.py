"""The allocation-free walk (fos_mc_run_noalloc) against fos_mc_run through
the C ABI: the same tallies bit for bit, on two calls in a row (the second
with a smaller problem, so the scratch holds the first call's larger table),
for single- and multi-layer problems; a problem larger than the scratch is
rejected before any work, leaving the tallies untouched; and the context's
own prepared problem is not disturbed."""
import numpy as np
import pytest

from gpu_helpers import device_problem, make_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _problem(I, layers, seed):
    rng = np.random.default_rng(seed)
    return make_arrays(rng.uniform(0, 5, (I, layers)), rng.uniform(0, 0.3, (I, layers)),
                       rng.uniform(-0.5, 0.95, (I, layers)), rng.uniform(1.0, 1.8, (I, layers)),
                       rng.uniform(0.5, 20, (I, layers)), n_upper=1.0, n_lower=rng.uniform(1, 3.5, I),
                       k_lower=np.where(rng.uniform(size=I) < 0.5, 0.0, 0.02), mu0=rng.uniform(0.2, 1.0, I),
                       photons=rng.integers(0, 20000, I), n_layers=rng.integers(1, layers + 1, I))


def _run(fn, ctx, a, seed, torch, launch=None):
    from paper_2409_00165_amd import fos
    prob = device_problem(a)
    tal = torch.full((prob.n_items * fos.N_TALLY,), -1, dtype=torch.int64, device="cuda")
    fn(ctx, prob, seed, tal, launch=launch)
    torch.cuda.synchronize()
    return tal.cpu().numpy().reshape(prob.n_items, fos.N_TALLY)


@pytest.mark.parametrize("layers", [1, 3])
def test_noalloc_matches_run_on_two_calls(torch, layers):
    from paper_2409_00165_amd import fos
    with fos.Context(0) as c:
        h = c.handle
        for I, seed in ((3000, 11), (257, 12)):          # the second call is smaller
            a = _problem(I, layers, seed)
            ref = _run(fos.fos_mc_run, h, a, seed, torch)
            got = _run(fos.fos_mc_run_noalloc, h, a, seed, torch)
            assert (got == ref).all(), (I, layers)
            assert (got[:, :5].sum(1) == a["photons"]).all()
        # an explicit launch gives the same bits too
        got = _run(fos.fos_mc_run_noalloc, h, a, 12, torch, launch={"block_size": 128, "chunk": 100})
        assert (got == ref).all()


def test_noalloc_rejects_a_problem_beyond_its_scratch_without_side_effects(torch):
    from paper_2409_00165_amd import fos
    with fos.Context(0) as c:
        h = c.handle
        small = _problem(64, 2, 3)
        ref = _run(fos.fos_mc_run, h, small, 5, torch)      # the context's prepared problem
        big = make_arrays(np.full((40_000, 8), 0.5), 0.01, 0.5, 1.4, 10.0, photons=10)
        prob = device_problem(big)
        tal = torch.full((prob.n_items * fos.N_TALLY,), -1, dtype=torch.int64, device="cuda")
        with pytest.raises(fos.FosError) as ei:
            fos.fos_mc_run_noalloc(h, prob, 1, tal)
        assert ei.value.status == 1 and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((tal == -1).all())
        # the context still holds its own prepared problem
        assert fos.fos_mc_prepared_items(h) == 64
        out = torch.zeros(64 * fos.N_TALLY, dtype=torch.int64, device="cuda")
        fos.fos_mc_execute(h, 5, out)
        torch.cuda.synchronize()
        assert (out.cpu().numpy().reshape(64, fos.N_TALLY) == ref).all()


def test_noalloc_validates_like_prepare(torch):
    from paper_2409_00165_amd import fos
    with fos.Context(0) as c:
        a = _problem(100, 2, 8)
        a["g"][37, 0] = 1.5
        prob = device_problem(a)
        tal = torch.full((100 * fos.N_TALLY,), -1, dtype=torch.int64, device="cuda")
        with pytest.raises(fos.FosError) as ei:
            fos.fos_mc_run_noalloc(c.handle, prob, 1, tal)
        assert "item 37" in str(ei.value) and "g" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((tal == -1).all())


def test_noalloc_rejects_regrouping(torch):
    """Regrouping needs the context's hand-off list, so the allocation-free
    walk refuses it before any work."""
    from paper_2409_00165_amd import fos
    a = _problem(300, 1, 3)
    with fos.Context(0) as c:
        prob = device_problem(a)
        tal = torch.full((prob.n_items * fos.N_TALLY,), -7, dtype=torch.int64, device="cuda")
        with pytest.raises(fos.FosError, match="regroup"):
            fos.fos_mc_run_noalloc(c.handle, prob, 1, tal, launch={"regroup_lanes": 8})
        torch.cuda.synchronize()
        assert bool((tal == -7).all())
