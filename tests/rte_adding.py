"""Deterministic slab radiative-transfer solver used as an independent pin.

The paper lists the adding-doubling method among deterministic solvers of
the radiative transfer equation (Introduction, refs. [26], [27]).  This is a
small flux-matrix adding-doubling code for one homogeneous plane-parallel
layer with a Henyey-Greenstein phase function, written only for tests: it
shares nothing with the Monte Carlo oracle or the GPU walk, so agreement
between them checks the walk's free-path sampling, albedo split, HG
sampling, direction update and Fresnel boundaries at once.

Formulation
-----------
Directions are discretised by Gauss-Legendre nodes mu_i in (0, 1] per
hemisphere (the interval is split at the critical cosine when the slab is
optically denser than its surroundings, so the boundary reflectance is smooth
on each piece), plus one extra node carrying the refracted incident beam
(weight zero: nothing scatters into it).  Matrices act on *photon fluxes per
direction node*: column = incoming node, row = outgoing node, so operators
compose by matrix products.

A thin layer of optical thickness d (single-scatter generator) has
    T_ij = delta_ij exp(-d/mu_j) + omega (d/mu_j) P(+mu_j -> +mu_i)
    R_ij =                          omega (d/mu_j) P(+mu_j -> -mu_i)
with P the azimuth-averaged HG redistribution
    h(mu, mu') = sum_l (2l+1) g^l P_l(mu) P_l(mu'),
    P(mu' -> mu_i) = h(mu_i, mu') w_i / 2  (renormalised to sum to one).
Doubling a symmetric layer:  E = (I - R R)^-1,  T' = T E T,  R' = R + T R E T.
Fresnel interfaces act diagonally (specular reflection keeps |mu|).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss, legval


def _fresnel_unpolarised(ci, ni, nt, kt=0.0):
    """Unpolarised Fresnel reflectance via Snell angles (sine/tangent form
    for real media, the impedance form for a complex transmitting medium)."""
    ci = np.asarray(ci, dtype=np.float64)
    if kt == 0.0:
        if nt == ni:
            return np.zeros_like(ci)
        si = np.sqrt(np.clip(1 - ci**2, 0, None))
        st = ni / nt * si
        out = np.ones_like(ci)
        ok = st < 1.0
        ti = np.arccos(np.clip(ci[ok], -1, 1))
        tt = np.arcsin(st[ok])
        with np.errstate(divide="ignore", invalid="ignore"):
            rs = -np.sin(ti - tt) / np.sin(ti + tt)
            rp = np.tan(ti - tt) / np.tan(ti + tt)
            r = 0.5 * (rs**2 + rp**2)
        # normal incidence: ((ni-nt)/(ni+nt))^2
        r = np.where(ti == 0.0, ((ni - nt) / (ni + nt)) ** 2, r)
        out[ok] = r
        return out
    N = nt + 1j * kt
    si2 = 1 - ci**2
    ct = np.sqrt(1 - (ni / N) ** 2 * si2 + 0j)
    ct = np.where(np.imag(N * ct) < 0, -ct, ct)
    rs = (ni * ci - N * ct) / (ni * ci + N * ct)
    rp = (N * ci - ni * ct) / (N * ci + ni * ct)
    return 0.5 * (np.abs(rs) ** 2 + np.abs(rp) ** 2)


def _nodes(n_per_piece, breaks):
    x, w = leggauss(n_per_piece)
    mus, ws = [], []
    for a, b in zip(breaks[:-1], breaks[1:]):
        mus.append(0.5 * (b - a) * x + 0.5 * (b + a))
        ws.append(0.5 * (b - a) * w)
    return np.concatenate(mus), np.concatenate(ws)


def _redistribution(mu, g, lmax):
    """h(+mu_i, +mu_j) and h(-mu_i, +mu_j) on node sets."""
    l = np.arange(lmax + 1)
    coef = (2 * l + 1) * g**l
    P = np.array([legval(mu, np.eye(lmax + 1)[k]) for k in range(lmax + 1)])  # [l, n]
    sign = (-1.0) ** l
    h_same = (P * coef[:, None]).T @ P
    h_flip = ((P * (coef * sign)[:, None]).T) @ P
    return h_same, h_flip


def slab_rat(tau, omega, g, n_slab=1.0, n_upper=1.0, n_lower=1.0, k_lower=0.0, mu0=1.0,
             nodes=48, lmax=None):
    """(R_specular, R_diffuse, A, T) of a homogeneous slab of optical
    thickness tau, single-scattering albedo omega and HG asymmetry g, index
    n_slab between a real upper medium and a (possibly complex) lower one,
    lit from above at incidence cosine mu0."""
    # incident beam after the top interface
    r_spec = float(_fresnel_unpolarised(np.array([mu0]), n_upper, n_slab)[0])
    st = n_upper / n_slab * np.sqrt(1 - mu0**2)
    mu_in = np.sqrt(1 - st**2)
    # quadrature split at critical cosines of the two faces
    breaks = [0.0, 1.0]
    for n_out in (n_upper, n_lower):
        if n_slab > n_out:
            breaks.append(np.sqrt(1 - (n_out / n_slab) ** 2))
    breaks = sorted(set(breaks))
    mu_q, w_q = _nodes(nodes, breaks)
    mu = np.concatenate([[mu_in], mu_q])
    w = np.concatenate([[0.0], w_q])
    M = len(mu)
    if lmax is None:
        lmax = 2 * nodes - 1 if g == 0 else int(min(4 * nodes, max(8, np.log(1e-16) / np.log(abs(g)))))
    h_same, h_flip = _redistribution(mu, g, lmax)
    Pd = h_same * w[:, None] / 2.0   # [i, j]: from +mu_j into +mu_i
    Pu = h_flip * w[:, None] / 2.0   # from +mu_j into -mu_i
    tot = Pd.sum(0) + Pu.sum(0)
    Pd /= tot
    Pu /= tot
    # thin layer and doubling
    K = int(np.ceil(np.log2(max(tau, 1e-30) / 1e-8))) if tau > 0 else 0
    K = max(K, 0)
    d = tau / 2.0**K
    T = np.diag(np.exp(-d / mu)) + omega * Pd * (d / mu)[None, :]
    R = omega * Pu * (d / mu)[None, :]
    I = np.eye(M)
    for _ in range(K):
        E = np.linalg.inv(I - R @ R)
        T, R = T @ E @ T, R + T @ R @ E @ T
    # boundaries (diagonal internal reflectances)
    Bt = np.diag(_fresnel_unpolarised(mu, n_slab, n_upper))
    Bb = np.diag(_fresnel_unpolarised(mu, n_slab, n_lower, k_lower))
    s = np.zeros(M)
    s[0] = 1.0 - r_spec
    # x = s + Bt (R x + T y),  y = Bb (T x + R y)
    A = np.block([[I - Bt @ R, -Bt @ T], [-Bb @ T, I - Bb @ R]])
    sol = np.linalg.solve(A, np.concatenate([s, np.zeros(M)]))
    x, y = sol[:M], sol[M:]
    up = R @ x + T @ y
    down = T @ x + R @ y
    r_diff = float(((I - Bt) @ up).sum())
    trans = float(((I - Bb) @ down).sum())
    absorbed = 1.0 - r_spec - r_diff - trans
    return r_spec, r_diff, absorbed, trans
