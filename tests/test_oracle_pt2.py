"""Pins of the oracle's second-order Epstein-Nesbet correction.

E0 = <Psi|H|Psi>/<Psi|Psi> and E2 = sum over k outside supp(Psi) of
(H Psi)_k^2 / (E0 - H_kk), divided by <Psi|Psi>, checked against the same
formulas evaluated with the dense H of tiny spaces (explicit second
quantization over the g-chain enumeration, an independent path), and against
the special cases that fix them: an exact eigenvector over the whole space has
no external determinants, and the correction does not depend on the norm of
Psi."""
import numpy as np
import pytest

from paper_2312_01846_amd import synth

SPACES = [(6, 2, 2), (7, 3, 2), (8, 3, 3)]


def _problem(orc, n, na, nb, seed):
    h, g = synth.molecule_like(n, 2 * n, seed)
    return orc.Problem(n, na, nb, h, g)


def _brute(H, ranks, amps):
    psi = np.zeros(H.shape[0])
    psi[ranks.astype(np.int64)] = amps
    y = H @ psi
    nn = psi @ psi
    e0 = (psi @ y) / nn
    ext = (psi == 0.0) & (y != 0.0)
    d = e0 - np.diag(H)[ext]
    terms = y[ext] ** 2 / d
    e2 = np.sum(terms) / nn
    # rounding bound: a few ulps per term (the two sides sum and form y in
    # different orders), plus E0's own rounding (~1e-14 relative) times the
    # sensitivity of each term to E0, which small denominators amplify
    tol = (1e-12 * np.sum(np.abs(terms)) + 1e-13 * max(1.0, abs(e0)) * np.sum(y[ext] ** 2 / d ** 2)) / nn
    # entries that cancel to zero in one summation order may leave a residue
    # of a few ulps in another: such entries may be counted on one side only
    tiny = int(np.sum(ext & (np.abs(y) < 1e-13 * np.abs(y).max())))
    return e0, e2, int(ext.sum()), tol, tiny


def _vectors(N, rng, H):
    out = [(np.array([0], dtype=np.uint64), np.array([1.0]))]  # a single determinant
    for frac in (0.02, 0.2):
        k = max(2, int(frac * N))
        r = np.sort(rng.choice(N, size=k, replace=False)).astype(np.uint64)
        out.append((r, rng.standard_normal(k)))
    # the largest entries of the ground state: a truncated variational vector
    w, V = np.linalg.eigh(H)
    v = V[:, 0]
    r = np.sort(np.argsort(-np.abs(v), kind="stable")[: max(3, N // 10)]).astype(np.uint64)
    out.append((r, v[r.astype(np.int64)]))
    return out


@pytest.mark.parametrize("n,na,nb", SPACES)
def test_pt2_matches_dense_formula(orc, n, na, nb):
    P = _problem(orc, n, na, nb, 11)
    H = P.dense_H()
    rng = np.random.default_rng(5)
    vecs = _vectors(P.n_det, rng, H)
    for r, a in vecs:
        e0, e2, ne = P.pt2(r, a)
        b0, b2, bn, tol, tiny = _brute(H, r, a)
        assert bn - tiny <= ne <= bn
        assert abs(e0 - b0) <= 1e-12 * max(1.0, abs(b0))
        assert abs(e2 - b2) <= tol, (e2, b2, tol)
    # the truncated ground state: E0 lies below every external diagonal, so
    # each term, and the correction, is negative
    assert P.pt2(*vecs[-1])[1] < 0.0


def test_pt2_of_exact_eigenvector_vanishes(orc):
    P = _problem(orc, 6, 2, 2, 3)
    H = P.dense_H()
    w, V = np.linalg.eigh(H)
    v = V[:, 0]
    r = np.arange(P.n_det, dtype=np.uint64)
    e0, e2, ne = P.pt2(r, v)
    assert ne == 0 and e2 == 0.0
    assert abs(e0 - w[0]) < 1e-10


def test_pt2_independent_of_norm(orc):
    P = _problem(orc, 7, 3, 2, 4)
    rng = np.random.default_rng(9)
    r = np.sort(rng.choice(P.n_det, size=60, replace=False)).astype(np.uint64)
    a = rng.standard_normal(60)
    e0, e2, ne = P.pt2(r, a)
    f0, f2, fn = P.pt2(r, 3.0 * a)
    assert fn == ne
    assert abs(f0 - e0) <= 1e-13 * abs(e0) and abs(f2 - e2) <= 1e-12 * abs(e2)


def test_pt2_rejects_unsorted(orc):
    P = _problem(orc, 6, 2, 2, 3)
    with pytest.raises(ValueError):
        P.pt2(np.array([3, 1], dtype=np.uint64), np.array([1.0, 1.0]))
