"""Pins of the oracle's backward: vbar = H sbar on supp(v), and the transition
1-/2-RDM gradients of sbar^T H(h, g) v with respect to h and (pq|rs)."""
import numpy as np
import pytest

from paper_2312_01846_amd import synth


def _sym_pert_h(n, rng):
    X = rng.normal(size=(n, n))
    return X + X.T


def _sym_pert_g(n, rng):
    X = rng.normal(size=(n, n, n, n))
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0),
             (3, 2, 1, 0)]
    return sum(X.transpose(p) for p in perms) / 8.0


def _L(orc, n, na, nb, h, g, vr, va, sr, sa):
    P = orc.Problem(n, na, nb, h, g)
    yr, ya = P.sigma(vr, va)
    d = dict(zip(yr.tolist(), ya.tolist()))
    return sum(s * d.get(int(r), 0.0) for r, s in zip(sr, sa))


@pytest.mark.parametrize("n,na,nb", [(5, 2, 2), (6, 3, 2)])
def test_explicit_equals_slater_condon_backward(orc, n, na, nb):
    h, g = synth.molecule_like(n, 2 * n, 1)
    P = orc.Problem(n, na, nb, h, g)
    vr, va = synth.random_sparse_vector(P.n_det, P.n_det // 3, 2)
    sr, sa = synth.random_sparse_vector(P.n_det, P.n_det // 2, 3)
    v1, h1, g1 = P.backward(vr, va, sr, sa, explicit=True)
    v2, h2, g2 = P.backward(vr, va, sr, sa, explicit=False)
    assert np.allclose(v1, v2, atol=1e-12)
    assert np.allclose(h1, h2, atol=1e-12)
    assert np.allclose(g1, g2, atol=1e-12)
    # vbar against the dense matrix
    H = P.dense_H()
    s = np.zeros(P.n_det)
    s[sr.astype(np.int64)] = sa
    assert np.allclose(v1, (H @ s)[vr.astype(np.int64)], atol=1e-12)


def test_finite_differences(orc):
    n, na, nb = 5, 2, 2
    h, g = synth.molecule_like(n, 10, 4)
    P = orc.Problem(n, na, nb, h, g)
    vr, va = synth.random_sparse_vector(P.n_det, 40, 5)
    sr, sa = synth.random_sparse_vector(P.n_det, 60, 6)
    _, dh, dg = P.backward(vr, va, sr, sa)
    rng = np.random.default_rng(0)
    Dh = _sym_pert_h(n, rng)
    Dg = _sym_pert_g(n, rng)
    eps = 1e-4
    fd_h = (_L(orc, n, na, nb, h + eps * Dh, g, vr, va, sr, sa) - _L(orc, n, na, nb, h - eps * Dh, g, vr, va, sr, sa)) / (2 * eps)
    fd_g = (_L(orc, n, na, nb, h, g + eps * Dg, vr, va, sr, sa) - _L(orc, n, na, nb, h, g - eps * Dg, vr, va, sr, sa)) / (2 * eps)
    # sigma is linear in (h, g): central differences are exact up to rounding
    assert abs(fd_h - np.sum(dh * Dh)) <= 1e-8 * max(1.0, abs(fd_h))
    assert abs(fd_g - np.sum(dg * Dg)) <= 1e-8 * max(1.0, abs(fd_g))


def test_hellmann_feynman_and_traces(orc):
    # For the dense eigenvector psi: E = sum dh*h + sum dg*g (H is linear in
    # the integrals), sum_p gamma_pp = N_e, sum_pr Gamma_pprr = N_e (N_e - 1).
    n, na, nb = 6, 2, 2
    h, g = synth.molecule_like(n, 12, 8)
    P = orc.Problem(n, na, nb, h, g)
    H = P.dense_H()
    w, V = np.linalg.eigh(H)
    psi = V[:, 0]
    r = np.arange(P.n_det, dtype=np.uint64)
    _, dh, dg = P.backward(r, psi, r, psi)
    E = np.sum(dh * h) + np.sum(dg * g)
    assert abs(E - w[0]) < 1e-10
    ne = na + nb
    assert abs(np.trace(dh) - ne) < 1e-10
    Gam = 2.0 * dg  # symmetrised Gamma
    assert abs(np.einsum("pprr->", Gam) - ne * (ne - 1)) < 1e-9
