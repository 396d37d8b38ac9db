"""FP64 oracle of the output stage -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this module.  It shares nothing with the HIP kernels.

What a finished spectrum turns into (paper, Output section and Results):
  * eq. (21): the solar-weighted totals R_s, A_s, T_s -- the integral over
    the simulated range of the spectral value times the solar irradiation G,
    over the integral of G.  They are computed only when a solar spectrum is
    given and the simulated range covers at least 0.28 - 2.5 um;
  * the emittance in a band (the sky window of the Introduction), by
    Kirchhoff's law the absorptance weighted by a blackbody spectrum;
  * the colour of the reflectance spectrum (the painted bilayer of Results;
    the paper does not say how it is computed).  Reading taken here: CIE 1931
    tristimulus values under an illuminant (equal energy unless one is
    given), the colour-matching functions from the multi-lobe analytic fit of
    Wyman, Sloan and Shirley (JCGT 2(2), 2013), CIELAB relative to the
    illuminant's white (CIE 15), and sRGB (IEC 61966-2-1) after a Bradford
    adaptation from the illuminant's white to D65.
Every spectrum given as samples is linear between them and zero outside
them (the paper interpolates input files linearly onto the simulated grid,
Input section).  Integrals are trapezoid sums over the simulated grid.

Parity status: pinned -- trapezoid exactness on linear integrands, the
eq. (21) invariants (a flat spectrum, R + A + T = 1), Planck's law against
Wien's displacement law and the Stefan-Boltzmann T^4 ratio, the colour
matching fit against the equal-energy white point, the photopic peak
ybar(555 nm) = 1, CIE illuminant A and the Planckian locus of Kim et al.,
CIELAB against its white and its 18.4 % grey, the sRGB matrix against the
published sRGB primaries and the D65 white, the transfer function's
continuity at its breakpoint, and the Bradford matrix against its
equal-energy normalisation (tests/test_oracle_output.py).
"""
from __future__ import annotations

import numpy as np

SOLAR_RANGE_UM = (0.28, 2.5)      # eq. (21) needs the simulated range to cover this
VISIBLE_RANGE_UM = (0.38, 0.78)   # the colour needs the simulated range to cover this
PLANCK_C2_UM_K = 14387.769        # second radiation constant hc/k, um K


def _f32(v):
    return np.float32(v)


def _covers(lam, lo, hi):
    """Whether the grid spans [lo, hi].  The grid reaches the device in
    single precision, so this decision (and band membership below) is taken
    on single-precision values on both sides."""
    return len(lam) >= 2 and _f32(lam[0]) <= _f32(lo) and _f32(lam[-1]) >= _f32(hi)

# ---------------------------------------------------------------------------
# spectra on the grid
# ---------------------------------------------------------------------------


def spectrum_on_grid(um, value, lam):
    """Samples (um, value) read at the grid wavelengths: linear between
    samples, zero outside [um[0], um[-1]]."""
    um = np.asarray(um, np.float64)
    value = np.asarray(value, np.float64)
    lam = np.asarray(lam, np.float64)
    out = np.interp(lam, um, value)
    out[(lam < um[0]) | (lam > um[-1])] = 0.0
    return out


def trapezoid(lam, f):
    """Integral of f over the grid by the trapezoid rule: the sum over
    intervals [a, b] of (b - a) (f(a) + f(b)) / 2.  f: [..., L]."""
    lam = np.asarray(lam, np.float64)
    f = np.asarray(f, np.float64)
    h = lam[1:] - lam[:-1]
    return np.sum(0.5 * h * (f[..., 1:] + f[..., :-1]), axis=-1)


def planck(lam_um, temperature_k):
    """Planck's law up to a constant factor: lambda^-5 / (exp(c2 / (lambda T)) - 1)."""
    lam = np.asarray(lam_um, np.float64)
    return 1.0 / (lam**5 * np.expm1(PLANCK_C2_UM_K / (lam * temperature_k)))


# ---------------------------------------------------------------------------
# eq. (21) and the band emittance
# ---------------------------------------------------------------------------


def solar_totals(lam, rat, solar):
    """Eq. (21) for R, A and T: [D, 3].  rat: [D, L, 3]; solar: (um, G)
    samples or None.  NaN when no spectrum is given or the grid does not
    cover 0.28 - 2.5 um."""
    lam = np.asarray(lam, np.float64)
    rat = np.asarray(rat, np.float64)
    D = rat.shape[0]
    if solar is None or not _covers(lam, *SOLAR_RANGE_UM):
        return np.full((D, 3), np.nan)
    G = spectrum_on_grid(solar[0], solar[1], lam)
    den = trapezoid(lam, G)
    return np.stack([trapezoid(lam, rat[:, :, c] * G) / den for c in range(3)], axis=1)


def band_emittance(lam, absorptance, lo_um, hi_um, temperature_k):
    """Blackbody-weighted absorptance over the grid points inside
    [lo_um, hi_um] (the trapezoid rule on that part of the grid): [D].
    NaN when fewer than two grid points fall in the band."""
    lam = np.asarray(lam, np.float64)
    A = np.asarray(absorptance, np.float64)
    lam32 = lam.astype(np.float32)
    inside = (lam32 >= _f32(lo_um)) & (lam32 <= _f32(hi_um))
    if temperature_k <= 0 or inside.sum() < 2:
        return np.full(A.shape[0], np.nan)
    sub = lam[inside]
    B = planck(sub, temperature_k)
    return trapezoid(sub, A[:, inside] * B) / trapezoid(sub, B)


# ---------------------------------------------------------------------------
# colour
# ---------------------------------------------------------------------------

# Multi-lobe fit of the CIE 1931 2-degree colour-matching functions (Wyman,
# Sloan, Shirley 2013): each is a sum of weight * g(lambda; mu, s1, s2), where
# g is a Gaussian of width s1 below its centre mu and s2 above it (nm).
_CMF_LOBES = {
    "x": ((1.056, 599.8, 37.9, 31.0), (0.362, 442.0, 16.0, 26.7), (-0.065, 501.1, 20.4, 26.2)),
    "y": ((0.821, 568.8, 46.9, 40.5), (0.286, 530.9, 16.3, 31.1)),
    "z": ((1.217, 437.0, 11.8, 36.0), (0.681, 459.0, 26.0, 13.8)),
}


def _lobe(lam_nm, mu, s1, s2):
    t = (lam_nm - mu) / np.where(lam_nm < mu, s1, s2)
    return np.exp(-0.5 * t * t)


def cmf_cie1931(lam_um):
    """(xbar, ybar, zbar) at the wavelengths lam_um: [3, L]."""
    lam_nm = 1000.0 * np.asarray(lam_um, np.float64)
    return np.stack([sum(w * _lobe(lam_nm, mu, s1, s2) for (w, mu, s1, s2) in _CMF_LOBES[c]) for c in "xyz"])


def tristimulus(lam, reflectance, illuminant=None):
    """CIE XYZ of each reflectance spectrum under the illuminant (samples
    (um, S), or None for equal energy), scaled so that a perfect reflector
    has Y = 1: X = int R S xbar / int S ybar, and so on.  Returns (XYZ [D, 3],
    white [3]); NaN when the grid does not cover 0.38 - 0.78 um."""
    lam = np.asarray(lam, np.float64)
    R = np.asarray(reflectance, np.float64)
    D = R.shape[0]
    if not _covers(lam, *VISIBLE_RANGE_UM):
        return np.full((D, 3), np.nan), np.full(3, np.nan)
    S = np.ones_like(lam) if illuminant is None else spectrum_on_grid(illuminant[0], illuminant[1], lam)
    cmf = cmf_cie1931(lam)
    norm = trapezoid(lam, S * cmf[1])
    XYZ = np.stack([trapezoid(lam, R * S * cmf[c]) / norm for c in range(3)], axis=1)
    white = np.array([trapezoid(lam, S * cmf[c]) / norm for c in range(3)])
    return XYZ, white


_LAB_EPS = (6.0 / 29.0) ** 3


def _lab_f(t):
    t = np.asarray(t, np.float64)
    return np.where(t > _LAB_EPS, np.cbrt(t), t / (3.0 * (6.0 / 29.0) ** 2) + 4.0 / 29.0)


def cielab(XYZ, white):
    """CIE 1976 L*a*b* of XYZ relative to the white (Xn, Yn, Zn): [D, 3]."""
    XYZ = np.asarray(XYZ, np.float64)
    fx, fy, fz = (_lab_f(XYZ[:, c] / white[c]) for c in range(3))
    return np.stack([116.0 * fy - 16.0, 500.0 * (fx - fy), 200.0 * (fy - fz)], axis=1)


# Bradford cone-response matrix (Lam 1985, as used by the ICC and CIECAM97s).
BRADFORD = np.array([[0.8951, 0.2664, -0.1614],
                     [-0.7502, 1.7135, 0.0367],
                     [0.0389, -0.0685, 1.0296]])
# IEC 61966-2-1: linear sRGB from CIE XYZ, and the D65 white (x, y) = (0.3127, 0.3290).
SRGB_FROM_XYZ = np.array([[3.2406, -1.5372, -0.4986],
                          [-0.9689, 1.8758, 0.0415],
                          [0.0557, -0.2040, 1.0570]])
D65_WHITE = np.array([0.3127 / 0.3290, 1.0, (1.0 - 0.3127 - 0.3290) / 0.3290])


def bradford_adaptation(src_white, dst_white):
    """3 x 3 matrix taking XYZ seen under src_white to XYZ under dst_white:
    cone responses scaled by the ratio of the two whites' responses."""
    src = BRADFORD @ np.asarray(src_white, np.float64)
    dst = BRADFORD @ np.asarray(dst_white, np.float64)
    return np.linalg.inv(BRADFORD) @ np.diag(dst / src) @ BRADFORD


def srgb_encode(v):
    """The sRGB transfer function on linear values in [0, 1]."""
    v = np.asarray(v, np.float64)
    return np.where(v <= 0.0031308, 12.92 * v, 1.055 * np.power(np.maximum(v, 0.0031308), 1.0 / 2.4) - 0.055)


def srgb(XYZ, white):
    """Encoded sRGB in [0, 1] of XYZ seen under `white`: adapted to D65,
    linear sRGB clipped to [0, 1] (colours outside the gamut), then encoded."""
    M = SRGB_FROM_XYZ @ bradford_adaptation(white, D65_WHITE)
    lin = np.asarray(XYZ, np.float64) @ M.T
    return srgb_encode(np.clip(lin, 0.0, 1.0))


# ---------------------------------------------------------------------------
# the whole stage
# ---------------------------------------------------------------------------


def output_stage(lam, rat, solar=None, illuminant=None, band=None):
    """totals [D, 4] = (R_s, A_s, T_s, band emittance) and colour [D, 9] =
    (X, Y, Z, L*, a*, b*, sRGB r, g, b) of D spectra rat [D, L, 3] on the
    grid lam [L] (um).  band = (lo_um, hi_um, temperature_k) or None."""
    rat = np.asarray(rat, np.float64)
    D = rat.shape[0]
    totals = np.empty((D, 4))
    totals[:, :3] = solar_totals(lam, rat, solar)
    totals[:, 3] = np.nan if band is None else band_emittance(lam, rat[:, :, 1], *band)
    XYZ, white = tristimulus(lam, rat[:, :, 0], illuminant)
    colour = np.empty((D, 9))
    colour[:, :3] = XYZ
    if np.all(np.isfinite(white)):
        colour[:, 3:6] = cielab(XYZ, white)
        colour[:, 6:9] = srgb(XYZ, white)
    else:
        colour[:, 3:] = np.nan
    return totals, colour
