"""Parity of the output stage (fos_output_prepare / fos_output_run, eq. (21),
band emittance and colour) with the FP64 oracle (oracle/output.py).

Tolerances follow from the device arithmetic: the weights are FP64 values
rounded to FP32, and each output is an FP32 sum over the grid, taken per lane
over ceil(L / 64) strided terms and then across the wave in 6 butterfly
steps.  For nonnegative terms x_l w_l summing to S that bounds the error by
(ceil(L/64) + 6 + 2) u S with u = 2^-24 (products, weight rounding and
additions); the tests allow 4x that.  CIELAB and sRGB carry the XYZ error
through their steepest slopes: CIELAB's f(t) rises at most 841/108 per unit
of t, the sRGB encoding at most 12.92."""
import math

import numpy as np
import pytest

from paper_2409_00165_amd import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2409_00165_amd import fos
    c = fos.Context(0)
    yield c
    c.close()


def _solar_standin():
    return W.solar_standin()


def _illuminant_standin():
    return W.blackbody_samples(0.30, 0.90, 0.005, 6504.0)


def _rat(D, L, seed):
    rng = np.random.default_rng(seed)
    return rng.dirichlet(np.ones(3), size=(D, L)).astype(np.float32)


def _f64(sp):
    return None if sp is None else (sp[0].astype(np.float64), sp[1].astype(np.float64))


def _run(ctx, torch, lam, rat, solar=None, illuminant=None, band=None, colour=True):
    from paper_2409_00165_amd import fos
    h = ctx.handle
    D, L = rat.shape[0], rat.shape[1]
    avail = fos.fos_output_prepare(h, lam, solar, illuminant, band)
    tot = torch.full((D * 4,), -7.0, device="cuda")
    col = torch.full((D * 9,), -7.0, device="cuda") if colour else None
    fos.fos_output_run(h, D, L, torch.from_numpy(np.ascontiguousarray(rat).ravel()).cuda(), tot, col)
    torch.cuda.synchronize()
    return (avail, tot.view(D, 4).cpu().numpy().astype(np.float64),
            None if col is None else col.view(D, 9).cpu().numpy().astype(np.float64))


def _tolerances(L, white, M):
    """Per-column tolerances of totals [4] and colour [9] (see module docstring)."""
    n = math.ceil(L / 64) + 8
    t_sum = 4.0 * n * U
    t_xyz = t_sum * np.asarray(white, np.float64)
    t_tot = np.full(4, t_sum)
    slope = 841.0 / 108.0
    dfx, dfy, dfz = (slope * (t_xyz[i] / white[i] + 2 * U) for i in range(3))
    t_lab = np.array([116.0 * dfy, 500.0 * (dfx + dfy), 200.0 * (dfy + dfz)]) + 2e-4
    lin = np.abs(M) @ (t_xyz + 4 * U * np.asarray(white))
    t_rgb = 12.92 * lin + 2e-6
    return t_tot, np.concatenate([t_xyz, t_lab, t_rgb])


def _compare(got, ref, tol, what):
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), f"{what}: NaN pattern differs"
    err = np.where(nan_r, 0.0, np.abs(got - np.where(nan_r, 0.0, ref)))
    bad = err > tol
    assert not bad.any(), f"{what}: max excess {np.max(err - tol):.3g}, worst column {np.argmax((err - tol).max(0))}"


def _colour_params(white):
    from oracle import output as O
    return O.SRGB_FROM_XYZ @ O.bradford_adaptation(white, O.D65_WHITE)


@pytest.mark.parametrize("case", ["paper_grid", "log_grid_equal_energy"])
def test_output_stage_matches_oracle(ctx, torch, case):
    from oracle import output as O
    from paper_2409_00165_amd import fos
    if case == "paper_grid":
        # the paper's example grid (0.25 - 2.5 um every 0.005 um): solar and colour, no band
        lam = np.round(np.arange(0.25, 2.5 + 1e-9, 0.005), 6).astype(np.float32)
        solar, illum, band, D = _solar_standin(), _illuminant_standin(), (8.0, 13.0, 300.0), 37
        want = fos.OUTPUT_SOLAR | fos.OUTPUT_COLOUR
    else:
        lam = W.grid_log(0.25, 16.0, 200).astype(np.float32)
        solar, illum, band, D = _solar_standin(), None, (8.0, 13.0, 300.0), 1001
        want = fos.OUTPUT_SOLAR | fos.OUTPUT_BAND | fos.OUTPUT_COLOUR
    rat = _rat(D, lam.size, seed=5)
    print(f"output stage {case}: {D} designs x {lam.size} wavelengths", flush=True)
    avail, tot, col = _run(ctx, torch, lam, rat, solar, illum, band)
    assert avail == want
    rt, rc = O.output_stage(lam.astype(np.float64), rat.astype(np.float64), _f64(solar), _f64(illum), band)
    white = O.tristimulus(lam.astype(np.float64), np.ones((1, lam.size)), _f64(illum))[1]
    t_tot, t_col = _tolerances(lam.size, white, _colour_params(white))
    _compare(tot, rt, t_tot[None, :], "totals")
    _compare(col, rc, t_col[None, :], "colour")


def test_output_weights_match_oracle(ctx, torch):
    """The prepared quadrature rows equal the oracle's stage applied to one-hot
    spectra (a spectrum 1 at one wavelength and 0 elsewhere picks out that
    wavelength's weight), within the FP32 rounding of each weight; the white
    point and colour matrix match too."""
    from oracle import output as O
    from paper_2409_00165_amd import fos
    lam = W.grid_log(0.25, 16.0, 157).astype(np.float32)
    solar, illum, band = _solar_standin(), _illuminant_standin(), (8.0, 13.0, 300.0)
    h = ctx.handle
    avail = fos.fos_output_prepare(h, lam, solar, illum, band)
    assert avail == fos.OUTPUT_SOLAR | fos.OUTPUT_BAND | fos.OUTPUT_COLOUR
    w = torch.zeros(5 * lam.size, device="cuda")
    p = torch.zeros(12, device="cuda")
    assert fos.fos_output_weights(h, lam.size, w, p) == avail
    torch.cuda.synchronize()
    w = w.view(5, lam.size).cpu().numpy().astype(np.float64)
    p = p.cpu().numpy().astype(np.float64)
    L = lam.size
    eye = np.eye(L)
    rat = np.zeros((L, L, 3))
    rat[:, :, 0] = eye
    rat[:, :, 1] = eye
    l64 = lam.astype(np.float64)
    tot, col = O.output_stage(l64, rat, _f64(solar), _f64(illum), band)
    ref = np.stack([tot[:, 0], tot[:, 3], col[:, 0], col[:, 1], col[:, 2]])
    assert np.all(np.abs(w - ref) <= 2 * U * np.abs(ref) + 1e-30)
    assert np.allclose(w.sum(1)[[0, 1, 3]], 1.0, atol=L * U)
    white = O.tristimulus(l64, np.ones((1, L)), _f64(illum))[1]
    assert np.allclose(p[:3], white, rtol=2 * U, atol=0)
    M = _colour_params(white)
    assert np.allclose(p[3:].reshape(3, 3), M, rtol=4 * U, atol=4 * U)


def test_output_availability_follows_the_grid(ctx, torch):
    from oracle import output as O
    from paper_2409_00165_amd import fos
    solar = _solar_standin()
    rat = _rat(9, 300, seed=8)
    # starts above 0.28 um: no solar totals; no band points; visible covered
    lam = np.linspace(0.30, 2.5, 300).astype(np.float32)
    avail, tot, col = _run(ctx, torch, lam, rat, solar, None, (8.0, 13.0, 300.0))
    assert avail == fos.OUTPUT_COLOUR
    assert np.isnan(tot).all() and np.isfinite(col).all()
    rt, rc = O.output_stage(lam.astype(np.float64), rat.astype(np.float64), _f64(solar), None, (8.0, 13.0, 300.0))
    assert np.isnan(rt).all()
    # an infrared-only grid: band only
    lam = np.linspace(5.0, 16.0, 300).astype(np.float32)
    avail, tot, col = _run(ctx, torch, lam, rat, solar, None, (8.0, 13.0, 300.0))
    assert avail == fos.OUTPUT_BAND
    assert np.isnan(tot[:, :3]).all() and np.isfinite(tot[:, 3]).all() and np.isnan(col).all()
    rt, _ = O.output_stage(lam.astype(np.float64), rat.astype(np.float64), _f64(solar), None, (8.0, 13.0, 300.0))
    assert np.allclose(tot[:, 3], rt[:, 3], atol=1e-5)
    # a single wavelength: nothing to integrate
    avail, tot, col = _run(ctx, torch, np.array([0.55], np.float32), rat[:, :1], solar, None, (8.0, 13.0, 300.0))
    assert avail == 0 and np.isnan(tot).all() and np.isnan(col).all()
    # a solar spectrum with no power on the grid: NaN totals although the grid covers the range
    dark = (np.array([5.0, 6.0], np.float32), np.array([1.0, 1.0], np.float32))
    lam = np.linspace(0.28, 2.5, 300).astype(np.float32)
    avail, tot, _ = _run(ctx, torch, lam, rat, dark, None, None, colour=False)
    assert avail & fos.OUTPUT_SOLAR and np.isnan(tot[:, :3]).all()


def test_output_stage_validation(torch):
    from paper_2409_00165_amd import fos
    c = fos.Context(0)
    h = c.handle
    tot = torch.zeros(4, device="cuda")
    one = torch.full((3,), 1.0 / 3.0, device="cuda")
    with pytest.raises(fos.FosError, match="NOT_PREPARED"):
        fos.fos_output_run(h, 1, 1, one, tot)
    lam = np.linspace(0.3, 2.5, 10).astype(np.float32)
    bad_grids = [lam[::-1].copy(), np.where(np.arange(10) == 4, np.nan, lam).astype(np.float32),
                 (lam - 1.0).astype(np.float32), np.repeat(lam[:5], 2)]
    for g in bad_grids:
        with pytest.raises(fos.FosError, match="INVALID_ARG"):
            fos.fos_output_prepare(h, g)
    bad_spectra = [(np.array([0.5], np.float32), np.array([1.0], np.float32)),
                   (np.array([0.5, 0.4], np.float32), np.array([1.0, 1.0], np.float32)),
                   (np.array([0.4, 0.5], np.float32), np.array([1.0, -1.0], np.float32)),
                   (np.array([0.4, 0.5], np.float32), np.array([1.0, np.inf], np.float32))]
    for sp in bad_spectra:
        with pytest.raises(fos.FosError, match="INVALID_ARG"):
            fos.fos_output_prepare(h, lam, solar=sp)
        with pytest.raises(fos.FosError, match="INVALID_ARG"):
            fos.fos_output_prepare(h, lam, illuminant=sp)
    with pytest.raises(fos.FosError, match="INVALID_ARG"):
        fos.fos_output_prepare(h, lam, band=(13.0, 8.0, 300.0))
    with pytest.raises(fos.FosError, match="INVALID_ARG"):
        fos.fos_output_prepare(h, lam, band=(8.0, 13.0, float("nan")))
    # a failed preparation leaves the stage unprepared
    fos.fos_output_prepare(h, lam)
    with pytest.raises(fos.FosError, match="INVALID_ARG"):
        fos.fos_output_prepare(h, lam[::-1].copy())
    with pytest.raises(fos.FosError, match="NOT_PREPARED"):
        fos.fos_output_run(h, 1, 10, torch.zeros(30, device="cuda"), tot)
    # the spectra must be laid out on the prepared grid
    fos.fos_output_prepare(h, lam)
    with pytest.raises(fos.FosError, match="INVALID_ARG"):
        fos.fos_output_run(h, 1, 9, torch.zeros(27, device="cuda"), tot)
    # zero designs is a no-op; a band of non-positive temperature is simply left out
    assert fos.fos_output_prepare(h, lam, band=(8.0, 13.0, 0.0)) == fos.OUTPUT_COLOUR
    fos.fos_output_run(h, 0, 10, torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"))
    c.close()


def test_output_prepare_twice_reuses_the_context(ctx, torch):
    """Grids of every register width the run kernel is built for (up to 64,
    128, 256, 512 and 1024 wavelengths per wave, and the wide form beyond),
    one after another on the same context, with design counts that leave
    ragged and odd chunks of 32: each run sees its own preparation."""
    from oracle import output as O
    solar = _solar_standin()
    for L, D in ((640, 21), (203, 66), (1500, 7), (100, 1), (64, 95), (1024, 33), (451, 64)):
        lam = W.grid_log(0.25, 16.0, L).astype(np.float32)
        rat = _rat(D, L, seed=L)
        _, tot, col = _run(ctx, torch, lam, rat, solar, None, (8.0, 13.0, 300.0))
        rt, rc = O.output_stage(lam.astype(np.float64), rat.astype(np.float64), _f64(solar), None,
                                (8.0, 13.0, 300.0))
        white = O.tristimulus(lam.astype(np.float64), np.ones((1, L)), None)[1]
        t_tot, t_col = _tolerances(L, white, _colour_params(white))
        _compare(tot, rt, t_tot[None, :], f"totals L={L}")
        _compare(col, rc, t_col[None, :], f"colour L={L}")


def test_output_stage_full_size_sampled(ctx, torch):
    """10^6 designs x 200 wavelengths (the design sweep's size), in the launch
    the benchmark times; 2,000 sampled designs plus the first and last checked
    against the oracle."""
    from oracle import output as O
    from paper_2409_00165_amd import fos
    D, L = 1_000_000, 200
    lam = W.grid_log(0.25, 16.0, L).astype(np.float32)
    solar, band = _solar_standin(), (8.0, 13.0, 300.0)
    print(f"output stage full size: {D} x {L}", flush=True)
    rat = W.synthetic_rat_device(torch, D, L, seed=2409)
    h = ctx.handle
    fos.fos_output_prepare(h, lam, solar, None, band)
    tot = torch.empty(D * 4, device="cuda")
    col = torch.empty(D * 9, device="cuda")
    fos.fos_output_run(h, D, L, rat, tot, col)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    pick = np.unique(np.concatenate([[0, D - 1], rng.integers(0, D, 2000)]))
    idx = torch.from_numpy(pick).cuda()
    sub = rat.view(D, L, 3).index_select(0, idx).cpu().numpy().astype(np.float64)
    got_t = tot.view(D, 4).index_select(0, idx).cpu().numpy().astype(np.float64)
    got_c = col.view(D, 9).index_select(0, idx).cpu().numpy().astype(np.float64)
    rt, rc = O.output_stage(lam.astype(np.float64), sub, _f64(solar), None, band)
    white = O.tristimulus(lam.astype(np.float64), np.ones((1, L)), None)[1]
    t_tot, t_col = _tolerances(L, white, _colour_params(white))
    _compare(got_t, rt, t_tot[None, :], "totals")
    _compare(got_c, rc, t_col[None, :], "colour")
