"""Pins of the output-stage oracle (oracle/output.py) against what the
mathematics and published colorimetry fix: trapezoid exactness, the eq. (21)
invariants, Wien's and Stefan-Boltzmann's laws, the CIE 1931 equal-energy
white and photopic peak, CIE illuminant A and the Planckian locus of Kim et
al. (an independent published fit), CIELAB's white and mid grey, and the
published sRGB primaries and D65 white."""
import numpy as np
import pytest

from oracle import output as O
from paper_2409_00165_amd import workloads as W

VIS = np.arange(360.0, 831.0, 1.0) / 1000.0      # 1 nm grid over the CIE tables' range, um


def _chromaticity(XYZ):
    XYZ = np.asarray(XYZ, np.float64)
    return XYZ[..., 0] / XYZ.sum(-1), XYZ[..., 1] / XYZ.sum(-1)


def test_trapezoid_is_exact_on_linear_integrands():
    lam = W.grid_log(0.25, 16.0, 57)
    f = 0.3 + 1.7 * lam
    exact = 0.3 * (lam[-1] - lam[0]) + 0.85 * (lam[-1] ** 2 - lam[0] ** 2)
    assert O.trapezoid(lam, f) == pytest.approx(exact, rel=1e-13)


def test_solar_totals_flat_spectrum_and_conservation():
    lam = W.grid_log(0.25, 4.0, 301)
    sol_um = np.linspace(0.28, 4.0, 187)
    sol = (sol_um, O.planck(sol_um, 5778.0))
    rng = np.random.default_rng(3)
    rat = rng.dirichlet(np.ones(3), size=(5, lam.size))
    rat[0, :, :] = (0.25, 0.6, 0.15)                 # flat spectrum: the totals are its values
    tot = O.solar_totals(lam, rat, sol)
    assert np.allclose(tot[0], (0.25, 0.6, 0.15), atol=1e-14)
    assert np.allclose(tot.sum(1), 1.0, atol=1e-13)  # R + A + T = 1 at every wavelength


def test_solar_totals_weight_by_interval_width():
    """G = 1 and R(lambda) = lambda on a non-uniform grid: R_s is the mean
    wavelength (l0 + l1) / 2 exactly -- an unweighted sum over grid points
    would not give it."""
    lam = W.grid_log(0.25, 2.5, 211)
    rat = np.zeros((1, lam.size, 3))
    rat[0, :, 0] = lam
    tot = O.solar_totals(lam, rat, (np.array([0.1, 3.0]), np.array([1.0, 1.0])))
    assert tot[0, 0] == pytest.approx(0.5 * (0.25 + 2.5), rel=1e-13)


def test_solar_spectrum_is_zero_outside_its_samples():
    """A spectrum given on 1 - 2 um only: R(lambda) = lambda on a uniform
    grid averages to 1.5 (the linear ramps at the two ends weigh 1.0 and 2.0
    alike); holding the end values beyond the samples would give 1.375."""
    lam = np.linspace(0.25, 2.5, 451)
    rat = np.zeros((1, lam.size, 3))
    rat[0, :, 0] = lam
    tot = O.solar_totals(lam, rat, (np.array([1.0, 2.0]), np.array([1.0, 1.0])))
    assert tot[0, 0] == pytest.approx(1.5, rel=1e-12)


def test_solar_totals_need_the_solar_range_and_a_spectrum():
    sol = (np.array([0.2, 4.0]), np.array([1.0, 1.0]))
    rat = np.full((2, 100, 3), 1.0 / 3.0)
    assert np.all(np.isfinite(O.solar_totals(np.linspace(0.28, 2.5, 100), rat, sol)))
    assert np.all(np.isnan(O.solar_totals(np.linspace(0.30, 2.5, 100), rat, sol)))
    assert np.all(np.isnan(O.solar_totals(np.linspace(0.28, 2.49, 100), rat, sol)))
    assert np.all(np.isnan(O.solar_totals(np.linspace(0.28, 2.5, 100), rat, None)))
    # the decision is taken on single-precision grid values: float32(0.28) > 0.28 still covers
    lam32 = np.linspace(0.28, 2.5, 100).astype(np.float32)
    assert float(lam32[0]) > 0.28 and np.all(np.isfinite(O.solar_totals(lam32, rat, sol)))


def test_planck_obeys_wien_and_stefan_boltzmann():
    for T in (300.0, 5778.0):
        lam = np.linspace(0.5 * 2897.77 / T, 2.0 * 2897.77 / T, 200001)
        peak = lam[np.argmax(O.planck(lam, T))]
        assert peak * T == pytest.approx(2897.77, rel=2e-5)          # Wien: lambda_max T = b
    lam = W.grid_log(0.5, 5000.0, 400001)
    ratio = O.trapezoid(lam, O.planck(lam, 600.0)) / O.trapezoid(lam, O.planck(lam, 300.0))
    assert ratio == pytest.approx(16.0, rel=1e-4)                      # total power ~ T^4


def test_band_emittance():
    lam = W.grid_log(0.25, 16.0, 200)
    A = np.full((3, lam.size), 0.93)
    assert np.allclose(O.band_emittance(lam, A, 8.0, 13.0, 300.0), 0.93, atol=1e-14)
    # only points inside the band count
    A2 = np.where((lam >= 8.0) & (lam <= 13.0), 0.5, 1.0)[None, :]
    assert O.band_emittance(lam, A2, 8.0, 13.0, 300.0)[0] == pytest.approx(0.5, abs=1e-14)
    assert np.isnan(O.band_emittance(lam, A, 8.0, 8.05, 300.0)).all()   # no two points in the band
    assert np.isnan(O.band_emittance(lam, A, 8.0, 13.0, 0.0)).all()


def test_colour_matching_fit_equal_energy_white_and_photopic_peak():
    cmf = O.cmf_cie1931(VIS)
    XYZ = np.array([O.trapezoid(VIS, cmf[c]) for c in range(3)])
    x, y = _chromaticity(XYZ)
    assert abs(x - 1.0 / 3.0) < 1e-3 and abs(y - 1.0 / 3.0) < 1e-3     # illuminant E is (1/3, 1/3)
    assert O.cmf_cie1931(np.array([0.555]))[1, 0] == pytest.approx(1.0, abs=5e-3)  # V(555 nm) = 1


def test_colour_matching_fit_against_illuminant_a_and_the_planckian_locus():
    # CIE illuminant A: Planck's law with c2 = 1.435e-2 m K at 2848 K; (x, y) = (0.44757, 0.40745)
    S_A = 1.0 / (VIS**5 * np.expm1(1.435e4 / (VIS * 2848.0)))
    cmf = O.cmf_cie1931(VIS)
    XYZ = np.array([O.trapezoid(VIS, S_A * cmf[c]) for c in range(3)])
    x, y = _chromaticity(XYZ)
    assert abs(x - 0.44757) < 2.5e-3 and abs(y - 0.40745) < 2.5e-3
    # Kim et al. (2002): cubic fit of the Planckian locus, 4000 - 25000 K
    for T in (4000.0, 5000.0, 6500.0, 10000.0, 20000.0):
        S = O.planck(VIS, T)
        XYZ = np.array([O.trapezoid(VIS, S * cmf[c]) for c in range(3)])
        x, y = _chromaticity(XYZ)
        xk = -3.0258469e9 / T**3 + 2.1070379e6 / T**2 + 0.2226347e3 / T + 0.240390
        yk = 3.0817580 * xk**3 - 5.87338670 * xk**2 + 3.75112997 * xk - 0.37001483
        assert abs(x - xk) < 1.5e-3 and abs(y - yk) < 1.5e-3, (T, x, y, xk, yk)


def test_tristimulus_normalisation_and_range():
    lam = np.linspace(0.25, 2.5, 451)
    S = (np.array([0.3, 1.0]), np.array([0.2, 1.4]))
    XYZ, white = O.tristimulus(lam, np.ones((2, lam.size)), S)
    assert np.allclose(XYZ, white[None, :], atol=1e-14) and white[1] == pytest.approx(1.0, abs=1e-14)
    grey, _ = O.tristimulus(lam, np.full((1, lam.size), 0.4), S)
    assert np.allclose(grey[0], 0.4 * white, atol=1e-14)
    XYZ, white = O.tristimulus(np.linspace(0.40, 2.5, 100), np.ones((1, 100)))
    assert np.isnan(XYZ).all() and np.isnan(white).all()          # the visible range is not covered


def test_cielab_white_grey_and_breakpoint():
    white = np.array([0.9642, 1.0, 0.8251])
    lab = O.cielab(white[None, :], white)[0]
    assert np.allclose(lab, (100.0, 0.0, 0.0), atol=1e-12)
    grey = O.cielab(0.18419 * white[None, :], white)[0]
    assert grey[0] == pytest.approx(50.0, abs=1e-2)                 # L* = 50 is 18.42 % luminance
    assert abs(grey[1]) < 1e-12 and abs(grey[2]) < 1e-12
    e = O._LAB_EPS
    lo, hi = O._lab_f(np.array([e * (1 - 1e-12), e * (1 + 1e-12)]))
    assert abs(hi - lo) < 1e-9                                       # the two branches meet
    dark = O.cielab(1e-3 * white[None, :], white)[0]
    assert dark[0] == pytest.approx(1e-3 * 24389.0 / 27.0, rel=1e-9)  # L* = kappa Y below the breakpoint


def test_cielab_of_the_srgb_primaries():
    """Published L*a*b* (D65) of the sRGB red, green and blue primaries."""
    prim = np.array([[0.4124, 0.2126, 0.0193], [0.3576, 0.7152, 0.1192], [0.1805, 0.0722, 0.9505]])
    ref = np.array([[53.24, 80.09, 67.20], [87.73, -86.18, 83.18], [32.30, 79.19, -107.86]])
    assert np.allclose(O.cielab(prim, O.D65_WHITE), ref, atol=0.1)


def test_srgb_matrix_against_published_primaries_and_white():
    # XYZ of the sRGB red, green and blue primaries (IEC 61966-2-1 forward matrix, columns)
    prim = np.array([[0.4124, 0.3576, 0.1805],
                     [0.2126, 0.7152, 0.0722],
                     [0.0193, 0.1192, 0.9505]])
    assert np.allclose(O.SRGB_FROM_XYZ @ prim, np.eye(3), atol=1e-3)
    assert np.allclose(O.SRGB_FROM_XYZ @ O.D65_WHITE, 1.0, atol=1e-3)


def test_srgb_transfer_function():
    b = 0.0031308
    assert abs(12.92 * b - (1.055 * b ** (1 / 2.4) - 0.055)) < 1e-6    # continuous at the breakpoint
    assert O.srgb_encode(np.array([0.0, 1.0])) == pytest.approx([0.0, 1.0], abs=1e-12)
    v = np.linspace(0, 1, 1001)
    assert np.all(np.diff(O.srgb_encode(v)) > 0)


def test_bradford_normalisation_and_adaptation():
    assert np.allclose(O.BRADFORD @ np.ones(3), 1.0, atol=2e-4)     # equal energy -> equal cone responses
    src = np.array([1.0985, 1.0, 0.3558])                            # an incandescent white
    M = O.bradford_adaptation(src, O.D65_WHITE)
    assert np.allclose(M @ src, O.D65_WHITE, atol=1e-12)
    assert np.allclose(O.bradford_adaptation(O.D65_WHITE, O.D65_WHITE), np.eye(3), atol=1e-12)


@pytest.mark.parametrize("illuminant", [None, "planck2856", "planck6504"])
def test_perfect_white_is_srgb_white_and_black_is_black(illuminant):
    lam = W.grid_log(0.3, 2.5, 300)
    ill = None
    if illuminant is not None:
        T = float(illuminant[6:])
        um = np.linspace(0.3, 2.5, 500)
        ill = (um, O.planck(um, T))
    rat = np.zeros((2, lam.size, 3))
    rat[0, :, 0] = 1.0
    tot, col = O.output_stage(lam, rat, illuminant=ill)
    assert np.allclose(col[0, 3:6], (100.0, 0.0, 0.0), atol=1e-10)
    assert np.allclose(col[0, 6:9], 1.0, atol=1e-3)
    assert np.allclose(col[1], 0.0, atol=1e-12)
    assert np.isnan(tot).all()                                       # no solar spectrum, no band


def test_output_stage_assembles_the_pieces():
    lam = W.grid_log(0.25, 16.0, 200)
    rng = np.random.default_rng(11)
    rat = rng.dirichlet(np.ones(3), size=(4, lam.size))
    sol = (np.linspace(0.28, 4.0, 300), O.planck(np.linspace(0.28, 4.0, 300), 5778.0))
    tot, col = O.output_stage(lam, rat, solar=sol, band=(8.0, 13.0, 300.0))
    assert np.allclose(tot[:, :3], O.solar_totals(lam, rat, sol))
    assert np.allclose(tot[:, 3], O.band_emittance(lam, rat[:, :, 1], 8.0, 13.0, 300.0))
    XYZ, white = O.tristimulus(lam, rat[:, :, 0])
    assert np.allclose(col[:, :3], XYZ) and np.allclose(col[:, 3:6], O.cielab(XYZ, white))
    assert np.all((col[:, 6:] >= 0) & (col[:, 6:] <= 1))
