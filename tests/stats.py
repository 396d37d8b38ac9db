"""Binomial statistics shared by the Monte Carlo tests."""
import numpy as np


def z_bound(p, n, k=4.0, floor=0.0):
    """k standard errors of a proportion p estimated from n photons."""
    p = np.clip(np.asarray(p, dtype=np.float64), 0.0, 1.0)
    return k * np.sqrt(p * (1 - p) / n) + floor


def pooled_bound(c1, n1, c2, n2, k=4.0):
    """Two-sample pooled bound k * sqrt(pbar(1-pbar)(1/n1 + 1/n2))."""
    c1 = np.asarray(c1, dtype=np.float64); c2 = np.asarray(c2, dtype=np.float64)
    n1 = np.asarray(n1, dtype=np.float64); n2 = np.asarray(n2, dtype=np.float64)
    pbar = (c1 + c2) / (n1 + n2)
    return k * np.sqrt(pbar * (1 - pbar) * (1.0 / n1 + 1.0 / n2))


def chi2_multinomial(counts, probs):
    """Pearson chi^2 of observed counts against expected probabilities,
    over the cells with non-zero expectation; returns (chi2, dof)."""
    counts = np.asarray(counts, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    n = counts.sum()
    m = probs > 0
    e = n * probs[m]
    chi2 = float(((counts[m] - e) ** 2 / e).sum())
    return chi2, int(m.sum()) - 1
