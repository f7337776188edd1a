"""Pins of the oracle's counter-based generator (Philox4x32-10) and of the
uniform map used by the null-collision MCC."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    out = orc.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expect


def test_u01_is_odd_multiple_of_2m24(orc):
    for r in [0, 1, 511, 512, 0x7FFFFFFF, 0xFFFFFFFF, 0x12345678]:
        u = orc.u01(r)
        k = u * 2 ** 24
        assert 0.0 < u < 1.0
        assert k == int(k) and int(k) % 2 == 1
        assert int(k) == 2 * (r >> 9) + 1
    # float32 represents every value exactly
    u = orc.u01(0xFFFFFFFF)
    assert float(np.float32(u)) == u


def test_philox_uniformity_and_independence(orc):
    # chi-square of 20000 draws of word 0 in 64 bins, and lag correlation of
    # successive counters; a wrong multiplier or a dropped key bump keeps
    # neither the KAT values nor these
    n = 20000
    vals = np.array([orc.philox4x32_10([i, 0, 7, 0], [0xC1, 0])[0] for i in range(n)],
                    dtype=np.float64) / 2 ** 32
    hist, _ = np.histogram(vals, bins=64, range=(0, 1))
    chi2 = ((hist - n / 64) ** 2 / (n / 64)).sum()
    assert chi2 < 120  # 63 dof: p ~ 3e-5
    c = np.corrcoef(vals[:-1], vals[1:])[0, 1]
    assert abs(c) < 5 / np.sqrt(n)
