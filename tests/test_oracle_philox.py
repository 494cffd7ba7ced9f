"""Pins for the oracle's Philox4x32-10 (Salmon et al., SC'11)."""
import os

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox(ctr, key)
        assert [int(x) for x in got] == want


def test_u01_mapping():
    # 24 high bits scaled by 2^-24
    assert oracle.u01(0) == 0.0
    assert oracle.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert oracle.u01(0x80000000) == 0.5
    assert oracle.u01(0x000000FF) == 0.0


def test_uniformity_chi_square():
    # 4 * 4096 words from consecutive counters; 16-bin chi-square well inside
    # the 99.9 % quantile (37.7 for 15 dof) and no strong lag-1 correlation.
    words = []
    for i in range(4096):
        words.extend(int(x) for x in oracle.philox([i, 7, 0, 0], [12345, 678]))
    u = np.array([(w >> 8) * 2.0 ** -24 for w in words])
    counts = np.bincount((u * 16).astype(int), minlength=16)
    exp = len(u) / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 37.7
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 4.0 / np.sqrt(len(u))


def test_many_is_the_generator_applied_per_pair():
    # the batched entry point applies the generator to pair i alone: the
    # known-answer vectors at shuffled positions among other pairs
    rows = _kat()
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(11, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(11, 2), dtype=np.uint64).astype(np.uint32)
    at = [7, 0, 10]
    for (c, k, _), i in zip(rows, at):
        ctr[i], key[i] = c, k
    got = oracle.philox_many(ctr, key)
    for (_, _, want), i in zip(rows, at):
        assert [int(x) for x in got[i]] == want
    for i in range(11):
        assert np.array_equal(got[i], oracle.philox(ctr[i], key[i]))
