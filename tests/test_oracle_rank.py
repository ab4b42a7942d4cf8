"""Pins of the oracle's determinant hashing (Sec. 2.2, Eq. 12, Tables 1-2)."""
import itertools
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table2_hash_6o3e.txt")


def _bits(s):  # leftmost character is orbital 1 = bit 0
    return sum(1 << p for p, ch in enumerate(s) if ch == "1")


def _table2():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        s, v = line.split()
        rows.append((s, int(v)))
    return rows


def test_table2_hash_values(orc):
    rows = _table2()
    assert len(rows) == 20
    for s, v in rows:
        assert orc.str_rank(_bits(s)) == v, s


def test_worked_example_101010(orc):
    # Sec. 2.2: contributions 4 + 1 + 0.
    assert orc.str_rank(_bits("101010")) == 5


def test_gchain_reproduces_table1(orc):
    rows = _table2()
    x = _bits("111000")
    chain = [x]
    while True:
        y = orc.gchain_next(x, 6)
        if y is None:
            break
        chain.append(y)
        x = y
    assert chain == [_bits(s) for s, _ in rows]
    assert chain[-1] == _bits("000111")


@pytest.mark.parametrize("n", range(1, 15))
def test_rank_is_bijection_onto_consecutive_integers(orc, n):
    # Brute force: every k-subset of n orbitals maps to a distinct value in
    # [0, C(n,k)), and unrank inverts it.
    for k in range(0, n + 1):
        N = orc.binom(n, k)
        seen = np.zeros(N, dtype=bool)
        for occ in itertools.combinations(range(n), k):
            b = sum(1 << p for p in occ)
            r = orc.str_rank(b)
            assert 0 <= r < N
            assert not seen[r]
            seen[r] = True
            assert orc.str_unrank(r, k) == b
        assert seen.all()


@pytest.mark.parametrize("n,k", [(8, 3), (10, 5), (12, 6), (14, 4)])
def test_gchain_order_equals_hash_order(orc, n, k):
    # Distance along the g-chain from 11..100..0 equals the hash (Sec. 2.2).
    x = (1 << k) - 1
    d = 0
    while x is not None:
        assert orc.str_rank(x) == d
        x = orc.gchain_next(x, n)
        d += 1
    assert d == orc.binom(n, k)


def test_boundaries_and_binomials(orc):
    from math import comb

    for a in range(0, 65):
        for b in range(0, 65):
            assert orc.binom(a, b) == (comb(a, b) if b <= a else 0)
    for n, k in [(26, 5), (28, 6), (32, 16), (20, 4)]:
        first = (1 << k) - 1
        last = first << (n - k)
        assert orc.str_rank(first) == 0
        assert orc.str_rank(last) == comb(n, k) - 1
        assert orc.str_unrank(comb(n, k) - 1, k) == last


def test_large_n_roundtrip(orc):
    from math import comb

    rng = np.random.default_rng(7)
    for n, k in [(26, 5), (28, 6), (32, 16), (32, 1)]:
        for _ in range(200):
            occ = sorted(rng.choice(n, size=k, replace=False).tolist())
            b = sum(1 << int(p) for p in occ)
            r = orc.str_rank(b)
            assert r == sum(comb(c, t + 1) for t, c in enumerate(occ))  # combinatorial number system
            assert orc.str_unrank(r, k) == b


def test_det_rank_alpha_major(orc):
    from math import comb

    P = orc.Problem(8, 3, 2, np.zeros((8, 8)), np.zeros(8 ** 4))
    assert P.n_det == comb(8, 3) * comb(8, 2)
    ranks = np.arange(P.n_det, dtype=np.uint64)
    a, b = P.unrank(ranks)
    assert np.array_equal(P.rank(a, b), ranks)
    # alpha rank ranges are contiguous rank ranges; bucket = floor(h / N_B)
    ra = ranks // np.uint64(comb(8, 2))
    assert np.array_equal(np.array([orc.str_rank(int(x)) for x in a], dtype=np.uint64), ra)
    NB = 37
    buckets = ranks // np.uint64(NB)
    assert np.all(np.diff(buckets.astype(np.int64)) >= 0) and buckets[-1] == (P.n_det - 1) // NB
