"""Pins of the oracle's Hamiltonian application and truncation.

The Slater-Condon generation (orc_sigma) is checked against explicit
second-quantized operator application on tiny spaces, whose determinants are
enumerated along the paper's g-chain (Sec. 2.2); the per-entry pull form
against the push form bit for bit; top-M against a full sort.
"""
import itertools
from math import comb

import numpy as np
import pytest

from paper_2312_01846_amd import synth


def _rand_integrals(n, seed, rank=None):
    return synth.molecule_like(n, rank or 2 * n, seed)


SPACES = [(4, 2, 1), (5, 2, 2), (6, 3, 2), (6, 1, 3), (7, 3, 3), (8, 3, 3)]


@pytest.mark.parametrize("n,na,nb", SPACES)
def test_sigma_matches_explicit_second_quantization(orc, n, na, nb):
    h, g = _rand_integrals(n, seed=n * 10 + na)
    P = orc.Problem(n, na, nb, h, g)
    r, a = synth.random_sparse_vector(P.n_det, max(1, P.n_det // 3), seed=5)
    sr, sa, sab = P.sigma(r, a, with_abs=True)
    dense = P.sigma_explicit_dense(r, a)
    full = np.zeros(P.n_det)
    full[sr.astype(np.int64)] = sa
    # Entries absent from the push result must be (numerically) zero.
    scale = np.zeros(P.n_det)
    scale[sr.astype(np.int64)] = sab
    err = np.abs(full - dense)
    assert np.all(err <= 1e-13 * np.maximum(scale, 1.0))


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 2), (8, 3, 3)])
def test_dense_H_from_gchain_matches_sigma(orc, n, na, nb):
    h, g = _rand_integrals(n, seed=3)
    P = orc.Problem(n, na, nb, h, g)
    H = P.dense_H()
    assert np.max(np.abs(H - H.T)) < 1e-13
    r, a = synth.random_sparse_vector(P.n_det, P.n_det // 2, seed=9)
    v = np.zeros(P.n_det)
    v[r.astype(np.int64)] = a
    sr, sa = P.sigma(r, a)
    y = np.zeros(P.n_det)
    y[sr.astype(np.int64)] = sa
    assert np.max(np.abs(H @ v - y)) < 1e-12


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 2), (7, 2, 3)])
def test_elements_bitwise_hermitian(orc, n, na, nb):
    h, g = _rand_integrals(n, seed=11)
    P = orc.Problem(n, na, nb, h, g)
    for src in range(P.n_det):
        tgt, el = P.source_terms(src)
        for t, e in zip(tgt, el):
            assert P.element(int(t), src) == e  # exact, not approximate


@pytest.mark.parametrize("n,na,nb", [(6, 2, 3), (8, 3, 3), (10, 4, 3)])
def test_connection_count_formula(orc, n, na, nb):
    # 1 + s_a + s_b + d_aa + d_bb + d_ab connections per source for generic integrals.
    h, g = _rand_integrals(n, seed=1)
    P = orc.Problem(n, na, nb, h, g)
    sa, sb = na * (n - na), nb * (n - nb)
    daa = comb(na, 2) * comb(n - na, 2)
    dbb = comb(nb, 2) * comb(n - nb, 2)
    want = 1 + sa + sb + daa + dbb + sa * sb
    for src in [0, P.n_det // 3, P.n_det - 1]:
        tgt, el = P.source_terms(src)
        assert len(tgt) == want
        assert len(np.unique(tgt)) == want  # one term per (source, target) pair
        assert np.all(tgt < P.n_det)


def test_connected_targets_conserve_particle_number_and_sz(orc):
    n, na, nb = 7, 3, 2
    h, g = _rand_integrals(n, seed=2)
    P = orc.Problem(n, na, nb, h, g)
    for src in range(0, P.n_det, 7):
        tgt, _ = P.source_terms(src)
        a, b = P.unrank(tgt)
        assert all(bin(int(x)).count("1") == na for x in a)
        assert all(bin(int(x)).count("1") == nb for x in b)
        a0, b0 = P.unrank([src])
        # at most two electrons move in total
        moved = [bin(int(x) ^ int(a0[0])).count("1") + bin(int(y) ^ int(b0[0])).count("1") for x, y in zip(a, b)]
        assert max(moved) <= 4


def test_spin_flip_symmetry(orc):
    # Spin flip F sends |A,B> to (-1)^(na*nb) |B,A>; H commutes with F and
    # the common factor cancels, so sigma(swap v) = swap(sigma v) exactly.
    n, na = 7, 3
    h, g = _rand_integrals(n, seed=4)
    P = orc.Problem(n, na, na, h, g)
    r, a = synth.random_sparse_vector(P.n_det, 60, seed=3)
    A, B = P.unrank(r)
    rf = P.rank(B, A)
    o = np.argsort(rf)
    sr, sa = P.sigma(r, a)
    fr, fa = P.sigma(rf[o], a[o])
    A2, B2 = P.unrank(sr)
    back = P.rank(B2, A2)
    oo = np.argsort(back)
    assert np.array_equal(back[oo], fr)
    assert np.allclose(fa, sa[oo], atol=1e-13, rtol=0)


def test_sigma_entry_pull_equals_push_bitwise(orc):
    n, na, nb = 8, 3, 3
    h, g = _rand_integrals(n, seed=0, rank=16)
    P = orc.Problem(n, na, nb, h, g)
    r, a = synth.random_sparse_vector(P.n_det, 700, seed=1)
    sr, sa, sab = P.sigma(r, a, with_abs=True)
    rng = np.random.default_rng(0)
    for idx in rng.choice(len(sr), 150, replace=False):
        v, ab = P.sigma_entry(r, a, int(sr[idx]))
        assert v == sa[idx]
        assert ab == sab[idx]


def test_hubbard_sigma_sparse_structure(orc):
    # On a ring at U=0 each determinant connects to its hops only (plus no
    # diagonal since h_pp = 0): at most 2 hops per electron.
    h, g = synth.hubbard_ring(6, 1.0, 0.0)
    P = orc.Problem(6, 3, 3, h, g)
    for src in range(P.n_det):
        tgt, el = P.source_terms(src)
        assert np.all(np.abs(el) == 1.0)
        assert len(tgt) <= 12


def test_topm_matches_full_sort_and_ties(orc):
    rng = np.random.default_rng(3)
    ranks = np.sort(rng.choice(10_000, 2000, replace=False)).astype(np.uint64)
    amps = rng.normal(size=2000)
    # plant exact magnitude ties of both signs and zeros
    amps[100:140] = 0.25
    amps[140:160] = -0.25
    amps[160:180] = 0.0
    for M in [1, 10, 50, 110, 1000, 1990, 5000, None]:
        kr, ka = orc.topm(ranks, amps, M)
        keys = sorted([(-abs(x), int(r), x) for r, x in zip(ranks, amps) if x != 0.0])
        keep = keys if M is None else keys[:M]
        if M is not None and 0 < M < len(keys):
            # plus everything within a relative 2^-36 of the M-th magnitude, if that adds <= 256
            thr = -keep[-1][0] * (1.0 - 2.0 ** -36)
            extra = [k for k in keys[M:] if -k[0] >= thr]
            if len(extra) <= 256:
                keep = keep + extra
        want = sorted((r, x) for _, r, x in keep)
        assert [int(x) for x in kr] == [r for r, _ in want]
        assert np.array_equal(ka, np.array([x for _, x in want]))
    # the 60 planted ties of magnitude 0.25 are split only when more than 256 would have to be added
    many = amps.copy()
    many[:400] = 0.5
    kr, _ = orc.topm(ranks, many, 100)
    assert len(kr) == 100
    above = int(np.sum(np.abs(amps) > 0.25))
    kr, _ = orc.topm(ranks, amps, above + 5)  # the M-th entry is one of the 0.25 ties: all 60 are kept
    assert len(kr) == above + 60
    assert np.sum(np.abs(amps[np.isin(ranks, kr)]) == 0.25) == 60


def test_topm_keeps_near_ties(orc):
    # partners equal up to rounding are kept together; a real gap still cuts
    ranks = np.arange(10, dtype=np.uint64)
    amps = np.array([1.0, 0.9, 0.8, 0.7, 0.7 * (1 + 2.0 ** -52), 0.6, 0.5, 0.4, 0.3, 0.2])
    kr, ka = orc.topm(ranks, amps, 4)
    assert kr.tolist() == [0, 1, 2, 3, 4]
    kr, ka = orc.topm(ranks, amps, 3)
    assert kr.tolist() == [0, 1, 2]


def test_normalize(orc):
    a = np.array([3.0, 4.0])
    out, nrm = orc.normalize(a)
    assert nrm == 5.0 and np.array_equal(out, [0.6, 0.8])
