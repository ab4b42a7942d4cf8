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


def _check_is_top_m(ranks, amps, M, kr, ka):
    """The defining properties of the truncation (Sec. 2.1, Eqs. 10-11): the
    kept set holds min(M, nonzero) entries, unchanged and by ascending rank;
    no dropped entry is larger in magnitude than a kept one; where magnitudes
    tie across the cut, the kept entries have the lower ranks; zeros never stay."""
    nz = amps != 0.0
    want_n = int(nz.sum()) if M is None else min(int(M), int(nz.sum()))
    assert len(kr) == want_n
    assert np.all(np.diff(kr.astype(np.int64)) > 0)
    pos = np.searchsorted(ranks, kr)
    assert np.array_equal(ranks[pos], kr) and np.array_equal(amps[pos], ka)
    assert np.all(ka != 0.0)
    dropped = np.ones(len(ranks), dtype=bool)
    dropped[pos] = False
    dropped &= nz
    if want_n and dropped.any():
        kmin = np.abs(ka).min()
        dmax = np.abs(amps[dropped]).max()
        assert kmin >= dmax
        if kmin == dmax:
            assert kr[np.abs(ka) == kmin].max() < ranks[dropped & (np.abs(amps) == kmin)].min()


def test_topm_is_the_M_largest(orc):
    rng = np.random.default_rng(3)
    ranks = np.sort(rng.choice(10_000, 2000, replace=False)).astype(np.uint64)
    amps = rng.normal(size=2000)
    # plant exact magnitude ties of both signs and zeros
    amps[100:140] = 0.25
    amps[140:160] = -0.25
    amps[160:180] = 0.0
    above = int(np.sum(np.abs(amps) > 0.25))
    for M in [0, 1, 10, 50, 110, above + 5, above + 59, above + 60, 1000, 1820, 1990, 5000, None]:
        kr, ka = orc.topm(ranks, amps, M)
        _check_is_top_m(ranks, amps, M, kr, ka)
    # the library sort: numpy's lexsort on (rank, -|c|) and the first M
    for M in [7, above + 5, 1234]:
        order = np.lexsort((ranks, -np.abs(amps)))
        order = order[amps[order] != 0.0][:M]
        kr, ka = orc.topm(ranks, amps, M)
        assert np.array_equal(kr, np.sort(ranks[order]))


def test_topm_hand_cases(orc):
    ranks = np.arange(10, dtype=np.uint64)
    # a one-ulp near-tie straddling the cut is cut: 0.7 (rank 3) is smaller than 0.7 (1 + 2^-52) (rank 4)
    amps = np.array([1.0, 0.9, 0.8, 0.7, 0.7 * (1 + 2.0 ** -52), 0.6, 0.5, 0.4, 0.3, 0.2])
    assert amps[4] > amps[3]
    assert orc.topm(ranks, amps, 4)[0].tolist() == [0, 1, 2, 4]
    assert orc.topm(ranks, amps, 3)[0].tolist() == [0, 1, 2]
    assert orc.topm(ranks, amps, 5)[0].tolist() == [0, 1, 2, 3, 4]
    # exact ties across the cut go to the lower rank, whatever the sign
    r = np.array([3, 5, 7, 9], dtype=np.uint64)
    a = np.array([0.5, -0.5, 0.75, 0.5])
    assert orc.topm(r, a, 2)[0].tolist() == [3, 7]
    assert orc.topm(r, a, 3)[0].tolist() == [3, 5, 7]
    # M = 0 keeps nothing; M >= nonzero keeps every nonzero entry
    assert len(orc.topm(r, a, 0)[0]) == 0
    z = np.array([0.0, 1.0, 0.0, -2.0])
    assert orc.topm(r, z, 3)[0].tolist() == [5, 9]


def test_topm_band_extension(orc):
    # the opt-in extension: entries within a relative 2^-36 of the M-th |c|
    # stay with it, unless more than 256 would be added
    ranks = np.arange(10, dtype=np.uint64)
    amps = np.array([1.0, 0.9, 0.8, 0.7 * (1 + 2.0 ** -52), 0.7, 0.6, 0.5, 0.4, 0.3, 0.2])
    assert orc.topm(ranks, amps, 4, tie_band=True)[0].tolist() == [0, 1, 2, 3, 4]
    assert orc.topm(ranks, amps, 4)[0].tolist() == [0, 1, 2, 3]
    gap = amps.copy()
    gap[4] = 0.7 * (1 - 2.0 ** -30)  # a real gap still cuts
    assert orc.topm(ranks, gap, 4, tie_band=True)[0].tolist() == [0, 1, 2, 3]
    rng = np.random.default_rng(3)
    r = np.sort(rng.choice(10_000, 2000, replace=False)).astype(np.uint64)
    x = rng.normal(size=2000)
    x[100:160] = 0.25 * np.sign(rng.normal(size=60))
    above = int(np.sum(np.abs(x) > 0.25))
    kr, _ = orc.topm(r, x, above + 5, tie_band=True)  # the M-th entry is one of 60 ties: all kept
    assert len(kr) == above + 60
    x[:400] = 0.5
    kr, _ = orc.topm(r, x, 100, tie_band=True)  # 400 ties: more than 256 extra, exactly M kept
    assert len(kr) == 100


def test_normalize(orc):
    a = np.array([3.0, 4.0])
    out, nrm = orc.normalize(a)
    assert nrm == 5.0 and np.array_equal(out, [0.6, 0.8])


def _distinct_tiny(n, seed, tiny):
    """Integrals whose (pq|rs) with four distinct indices are tiny (scale
    `tiny`) and all others O(1): the two-body integrals a double excitation
    with four distinct orbitals uses are then tiny, while every single,
    diagonal and repeated-orbital alpha-beta double element stays O(1)."""
    h, g = synth.molecule_like(n, 2 * n, seed)
    g = g.reshape(n, n, n, n).copy()
    rng = np.random.default_rng(seed + 100)
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    if len({p, q, r, s}) == 4 and (p, q, r, s) == min(
                            [(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r), (r, s, p, q), (s, r, p, q),
                             (r, s, q, p), (s, r, q, p)]):
                        v = tiny * rng.uniform(0.5, 1.0)
                        for t in [(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r), (r, s, p, q), (s, r, p, q),
                                  (r, s, q, p), (s, r, q, p)]:
                            g[t] = v
    return h, g


def test_excitation_screen_zero_is_identity(orc):
    h, g = synth.molecule_like(8, 16, 0)
    P = orc.Problem(8, 3, 3, h, g)
    r, a = synth.random_sparse_vector(P.n_det, 400, seed=5)
    full = P.sigma(r, a, with_abs=True)
    zero = P.sigma(r, a, with_abs=True, eps_x=0.0)
    for x, y in zip(full, zero):
        assert np.array_equal(x, y)


def test_excitation_screen_hand_count(orc):
    # One source determinant (aufbau of 2 alpha + 2 beta in 6 orbitals) with
    # amplitude 1.  With the four-distinct-orbital integrals at 1e-9 and the
    # screen at 1e-6, exactly those doubles go: 6 alpha-alpha (C(2,2) C(4,2)),
    # 6 beta-beta, and the 2*4*1*3 = 24 alpha-beta doubles with i, a, j, b
    # all different; the 64 - 24 = 40 alpha-beta doubles sharing an orbital
    # (j = i or b = a) and every single and the diagonal stay.
    h, g = _distinct_tiny(6, 3, 1e-9)
    P = orc.Problem(6, 2, 2, h, g)
    r0 = np.array([0], dtype=np.uint64)
    full = P.sigma(r0, np.array([1.0]))
    scr = P.sigma(r0, np.array([1.0]), eps_x=1e-6)
    assert len(full[0]) == 1 + 8 + 8 + 6 + 6 + 64
    assert len(scr[0]) == len(full[0]) - 36
    assert np.isin(scr[0], full[0]).all()
    pos = np.searchsorted(full[0], scr[0])
    assert np.array_equal(full[1][pos], scr[1])  # one term per target: the kept values are unchanged


def test_excitation_screen_equals_dropping_the_tiny_integrals(orc):
    # Several sources with |v_i| in [0.5, 1]: the screened sigma equals sigma
    # of the Hamiltonian without the four-distinct-orbital integrals (which
    # enter only those doubles), by explicit second quantization
    h, g = _distinct_tiny(7, 4, 1e-10)
    P = orc.Problem(7, 3, 2, h, g)
    rng = np.random.default_rng(2)
    r = np.sort(rng.choice(P.n_det, 60, replace=False)).astype(np.uint64)
    a = rng.uniform(0.5, 1.0, 60) * rng.choice([-1.0, 1.0], 60)
    sr, sa, sab = P.sigma(r, a, with_abs=True, eps_x=1e-7)
    g0 = g.copy()
    g0[np.abs(g0) < 1e-8] = 0.0
    ref = orc.Problem(7, 3, 2, h, g0).sigma_explicit_dense(r, a)
    dense = np.zeros(P.n_det)
    dense[sr.astype(np.int64)] = sa
    assert np.all(np.abs(dense - ref) <= 1e-13 * np.maximum(1.0, np.abs(ref)))
