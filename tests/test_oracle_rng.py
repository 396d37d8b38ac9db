"""Pins of the oracle's Philox4x32-10 and its uniform mapping."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(orc, ctr, key, expect):
    assert orc.philox(ctr, key) == expect


def test_uniform_mapping_range_and_counter_layout(orc):
    # counter = (photon lo, photon hi, step, stream), key = (seed lo, seed hi);
    # U = (word >> 8) * 2^-24
    photon, step, stream, seed = (1 << 33) + 5, 17, 9, 0x1234_5678_9ABC_DEF0
    words = orc.philox([photon & 0xFFFFFFFF, photon >> 32, step, stream],
                       [seed & 0xFFFFFFFF, seed >> 32])
    u = orc.uniforms(photon, step, stream, seed)
    assert u == [(w >> 8) / 2.0**24 for w in words]
    assert all(0.0 <= x < 1.0 for x in u)


def test_uniforms_are_uniform(orc):
    # 4 * 20000 uniforms: mean, variance and a 20-bin chi^2
    us = np.array([orc.uniforms(p, 3, 1, 99) for p in range(20000)]).ravel()
    assert abs(us.mean() - 0.5) < 4 * np.sqrt(1 / 12 / us.size)
    assert abs(us.var() - 1 / 12) < 0.003
    h, _ = np.histogram(us, bins=20, range=(0, 1))
    e = us.size / 20
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 50  # 19 dof, p ~ 1e-4
