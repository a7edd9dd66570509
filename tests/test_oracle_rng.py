"""Pins of the oracle's random-number path: the Philox-4x32-10 known-answer
vectors published with the generator, the exact uniform mapping, symmetry of
the pair draw and the Gaussian statistics the paper asks of xi (Section 2.1:
zero mean, unit variance, symmetric)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox4x32, u01, pair_normals, pair_normals4, pair_normals_batch
from paper_1611_06163_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert [int(x) for x in philox4x32(ctr, key, 10)] == out


def test_uniform_mapping_exact_and_open():
    assert u01(0) == 2.0 ** -24
    assert u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for b in (0, 1 << 9, 12345678, 0xFFFFFFFF):
        u = u01(b)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in FP32


def test_pair_draw_symmetric_in_the_pair():
    cfg = I.c1()
    for (i, j) in [(0, 1), (5, 77), (3999, 12)]:
        for st in (0, 1, 64):
            a = pair_normals(cfg, 17, i, j, st)
            b = pair_normals(cfg, 17, j, i, st)
            assert np.array_equal(a, b)


def test_gaussian_statistics():
    cfg = I.c1()
    n = 200000
    gi = np.arange(n, dtype=np.uint32)
    gj = gi + 1
    z = pair_normals_batch(cfg, 3, gi, gj, 0).ravel()
    m, v = z.mean(), z.var()
    assert abs(m) < 5.0 / np.sqrt(z.size)
    assert abs(v - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 0.05
    assert abs(stats.skew(z)) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_draws_decorrelated_across_steps_and_streams():
    cfg = I.c1()
    n = 100000
    gi = np.arange(n, dtype=np.uint32)
    gj = gi + 7
    a = pair_normals_batch(cfg, 1, gi, gj, 0)[:, 0]
    b = pair_normals_batch(cfg, 2, gi, gj, 0)[:, 0]
    c = pair_normals_batch(cfg, 1, gi, gj, 1)[:, 0]
    d = pair_normals_batch(cfg, 1, gi, gj, 0)[:, 1]
    for x in (b, c, d):
        assert abs(np.corrcoef(a, x)[0, 1]) < 5.0 / np.sqrt(n)


def test_four_normals_per_draw():
    """The cos and sin Box-Muller partners are independent standard normals,
    and the cos ones equal the single-normal draws."""
    cfg = I.c1()
    z = np.array([pair_normals4(cfg, 5, i, i + 3, 64 + (i % 3)) for i in range(20000)])
    one = np.array([pair_normals(cfg, 5, i, i + 3, 64 + (i % 3)) for i in range(20000)])
    # (the compiler may evaluate cos and sin together, so allow last-ulp changes)
    assert np.allclose(z[:, 0], one[:, 0], rtol=1e-14, atol=1e-15)
    assert np.allclose(z[:, 2], one[:, 1], rtol=1e-14, atol=1e-15)
    for c in range(4):
        assert abs(z[:, c].mean()) < 5.0 / np.sqrt(z.shape[0])
        assert abs(z[:, c].var() - 1.0) < 5.0 * np.sqrt(2.0 / z.shape[0])
    cc = np.corrcoef(z.T)
    assert np.abs(cc - np.eye(4)).max() < 5.0 / np.sqrt(z.shape[0])
    assert stats.kstest(z[:, 1], "norm").pvalue > 1e-4
