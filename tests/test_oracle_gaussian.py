"""Pins of the oracle's Gaussian tensor generator (Philox4x32-10 + Box-Muller; the Gaussian tensor
columns of Alg. 6): published known-answer vectors of the generator, the tensor layout, and the
distribution of the draws."""
import json
import math
import os

import numpy as np
import pytest

from oracle import gaussian as ga

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.json")) as fh:
        kat = json.load(fh)
    for v in kat["vectors"]:
        ctr = [np.array([int(w, 16)], dtype=np.uint64) for w in v["counter"]]
        key = [int(w, 16) for w in v["key"]]
        out = ga.philox4x32_10(ctr, key)
        assert ["%08x" % int(o[0]) for o in out] == v["out"]


def test_philox_is_a_function_of_counter_and_key_only():
    # vectorized evaluation over many counters equals one-at-a-time evaluation
    q = np.arange(37, dtype=np.uint64) * np.uint64(2654435761)
    key = (0x12345678, 0x9abcdef0)
    z = np.zeros_like(q)
    allv = ga.philox4x32_10((q & np.uint64(0xFFFFFFFF), q >> np.uint64(32), z, z), key)
    for i in (0, 5, 36):
        one = ga.philox4x32_10(([int(q[i]) & 0xFFFFFFFF], [int(q[i]) >> 32], [0], [0]), key)
        assert [int(o[0]) for o in one] == [int(a[i]) for a in allv]


def _pair_by_hand(seed, q):
    """Box-Muller pair of pair index q written out with Python integers and math."""
    x0, x1, x2, x3 = (int(o[0]) for o in ga.philox4x32_10(([q & 0xFFFFFFFF], [q >> 32], [0], [0]),
                                                           (seed & 0xFFFFFFFF, seed >> 32)))
    u1 = (float(((x1 << 32) | x0) >> 11) + 0.5) / 2.0 ** 53
    u2 = float(((x3 << 32) | x2) >> 11) / 2.0 ** 53
    rad = math.sqrt(-2.0 * math.log(u1))
    return rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2)


def test_tensor_layout():
    seed, m, r, n = 0x0123456789ABCDEF, 5, 3, 7          # odd element count: last pair half used
    om = ga.gaussian_tensor(seed, m, r, n)
    assert om.shape == (m, r, n)
    for (i, j, t) in [(0, 0, 0), (1, 0, 0), (4, 2, 6), (2, 1, 3), (3, 2, 0)]:
        e = i + m * j + m * r * t
        z0, z1 = _pair_by_hand(seed, e // 2)
        assert om[i, j, t] == pytest.approx(z0 if e % 2 == 0 else z1, abs=1e-15)
    # a different seed gives a different tensor; the same seed the same one
    assert not np.allclose(om, ga.gaussian_tensor(seed + 1, m, r, n))
    np.testing.assert_array_equal(om, ga.gaussian_tensor(seed, m, r, n))


def test_draws_are_standard_normal():
    from scipy import stats
    z = ga.gaussian_tensor(211002485, 64, 64, 64).ravel()      # 262144 draws
    nz = z.size
    assert abs(z.mean()) < 5.0 / math.sqrt(nz)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / nz)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 5.0 * math.sqrt(24.0 / nz)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a pair are uncorrelated, and so are neighbouring pairs
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5.0 / math.sqrt(nz / 2)
    assert abs(np.corrcoef(z[:-2], z[2:])[0, 1]) < 5.0 / math.sqrt(nz)
