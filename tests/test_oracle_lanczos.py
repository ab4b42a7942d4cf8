"""Pins of the oracle's SFCI iteration (Sec. 2.1, Eqs. 1-11) and its small solver."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2312_01846_amd import synth


def _closed_form_ring(L, ne):
    eps = np.sort(-2.0 * np.cos(2.0 * np.pi * np.arange(L) / L))
    return 2.0 * eps[:ne].sum()


def test_jacobi_matches_lapack(orc):
    rng = np.random.default_rng(0)
    for m in [1, 2, 3, 7, 10, 20]:
        A = rng.normal(size=(m, m))
        A = A + A.T
        w, V = orc.jacobi(A)
        o = np.argsort(w)
        assert np.allclose(w[o], np.linalg.eigvalsh(A), atol=1e-12)
        assert np.allclose(V.T @ V, np.eye(m), atol=1e-12)
        assert np.allclose(A @ V, V * w, atol=1e-11)


def test_geneig_matches_scipy(orc):
    rng = np.random.default_rng(1)
    for m in [2, 5, 10]:
        B = rng.normal(size=(m, m))
        S = B @ B.T + m * np.eye(m)
        T = rng.normal(size=(m, m))
        T = T + T.T
        lam, x, r = orc.geneig(T, S)
        assert r == m
        ref = sla.eigh(T, S, eigvals_only=True)[0]
        assert abs(lam - ref) < 1e-12
        assert np.allclose(T @ x, lam * (S @ x), atol=1e-11)
        assert x[np.argmax(np.abs(x))] > 0


def test_geneig_drops_null_directions(orc):
    # Duplicate basis vectors make S singular; canonical orthogonalisation
    # removes the null direction and the lowest eigenvalue is unchanged.
    rng = np.random.default_rng(2)
    n = 30
    H = rng.normal(size=(n, n))
    H = H + H.T
    W = rng.normal(size=(n, 4))
    W = np.concatenate([W, W[:, :1]], axis=1)
    T = W.T @ H @ W
    S = W.T @ W
    lam, x, r = orc.geneig(T, S)
    assert r == 4
    ref = sla.eigh(W[:, :4].T @ H @ W[:, :4], W[:, :4].T @ W[:, :4], eigvals_only=True)[0]
    assert abs(lam - ref) < 1e-9


@pytest.mark.parametrize("L,ne", [(6, 3), (8, 4)])
def test_hubbard_U0_closed_form(orc, L, ne):
    h, g = synth.hubbard_ring(L, 1.0, 0.0)
    P = orc.Problem(L, ne, ne, h, g)
    a, b = synth.neel_bits(L)
    r0 = P.rank([a], [b])
    out = P.lanczos(r0, np.array([1.0]), None, 10, 60)
    assert abs(out["energies"][-1] - _closed_form_ring(L, ne)) < 1e-9


def _dense_case(orc):
    h, g = synth.molecule_like(8, 16, 0)
    P = orc.Problem(8, 3, 3, h, g)
    return P, P.dense_H()


def test_untruncated_block_is_rayleigh_ritz(orc):
    # With M = all, T = W^T H W and S = W^T W exactly; the block energy is the
    # lowest generalized eigenvalue, Psi's Rayleigh quotient under the dense H
    # (built independently from the g-chain) equals it, and the first block's
    # T is tridiagonal (Eq. 7).
    P, H = _dense_case(orc)
    out = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), None, 10, 30, want_T=True)
    E = out["energies"]
    for b in range(3):
        ref = sla.eigh(out["T"][b], out["S"][b], eigvals_only=True)[0]
        assert abs(E[b] - ref) < 1e-10
    psi = np.zeros(P.n_det)
    psi[out["psi_rank"].astype(np.int64)] = out["psi_amp"]
    rq = psi @ H @ psi / (psi @ psi)
    assert abs(rq - E[-1]) < 1e-10
    T0 = out["T"][0]
    off = np.abs(np.triu(T0, 2))
    assert off.max() < 1e-10
    assert np.allclose(out["S"][0], np.eye(10), atol=1e-10)
    # monotone: each block contains the previous Psi
    assert np.all(np.diff(E) <= 1e-12)
    # lowest eigenvalue reachable from the closed-shell start (spin-free H):
    w, V = np.linalg.eigh(H)
    reach = w[V[0, :] ** 2 > 1e-12][0]
    assert E[-1] >= reach - 1e-10
    assert E[-1] - reach < 1e-3


def test_truncated_blocks_are_variational(orc):
    P, H = _dense_case(orc)
    w, V = np.linalg.eigh(H)
    reach = w[V[0, :] ** 2 > 1e-12][0]
    last = []
    for M in [100, 400, 1600]:
        out = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), M, 10, 20, want_T=True)
        E = out["energies"]
        assert np.all(E >= reach - 1e-10)
        for b in range(2):
            ref = sla.eigh(out["T"][b], out["S"][b], eigvals_only=True)[0]
            assert abs(E[b] - ref) < 1e-9
        last.append(E[-1])
    # error shrinks as the truncation grows (Sec. 4, Table 3 trend)
    assert last[0] > last[1] > last[2]


def test_truncated_vectors_have_M_entries(orc):
    # Sec. 2.1: every basis vector holds N_d = M entries (the start vector
    # holds its own single determinant).  The closed-shell start gives
    # alpha/beta-exchanged partners of equal magnitude, so ties reach the cut.
    P, _ = _dense_case(orc)
    out = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 50, 10, 30)
    bn = out["basis_nnz"]
    assert bn[0, 0] == 1
    assert np.all(bn.ravel()[1:] == 50)
    assert np.all(np.diff(out["psi_rank"].astype(np.int64)) > 0)
    assert len(out["psi_rank"]) <= 10 * 50
    band = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 50, 10, 30, tie_band=True)
    assert band["basis_nnz"].max() > 50  # the extension keeps tied partners together


def test_screening_matches_manual_block(orc):
    # Sec. 3 screening: entries of H w_j below eps do not enter v.  First block
    # with N_L = 2, no truncation, rebuilt from the oracle's sigma (pinned
    # elsewhere) with the screen applied by hand.
    P, _ = _dense_case(orc)
    eps = 0.05
    out = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), None, 2, 2, want_T=True, eps=eps)

    def screened_sigma(r, a):
        sr, sa = P.sigma(r, a)
        keep = ~(np.abs(sa) < eps)
        return sr[keep], sa[keep]

    def dot(x, y):
        _, ix, iy = np.intersect1d(x[0], y[0], return_indices=True)
        return float(x[1][ix] @ y[1][iy])

    w0 = (np.array([0], dtype=np.uint64), np.array([1.0]))
    y0 = screened_sigma(*w0)
    t00 = dot(w0, y0)
    u = dict(zip(y0[0].tolist(), y0[1].tolist()))
    u[0] = u.get(0, 0.0) - t00
    ur = np.array(sorted(k for k, v in u.items() if v != 0.0), dtype=np.uint64)
    ua = np.array([u[int(k)] for k in ur])
    w1 = (ur, ua / np.sqrt(ua @ ua))
    y1 = screened_sigma(*w1)
    T = out["T"][0]
    assert abs(T[0, 0] - t00) < 1e-12
    assert abs(T[0, 1] - dot(w0, y1)) < 1e-12 and abs(T[1, 1] - dot(w1, y1)) < 1e-12
    # screening made a difference here
    plain = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), None, 2, 2, want_T=True)
    assert abs(plain["T"][0][1, 1] - T[1, 1]) > 1e-6


def test_screening_tiny_eps_is_identity(orc):
    P, _ = _dense_case(orc)
    a = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 30, want_T=True)
    b = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 30, want_T=True, eps=1e-300)
    assert np.array_equal(a["energies"], b["energies"]) and np.array_equal(a["T"], b["T"])
    # the paper's setting leaves the energy nearly unchanged on this case
    c = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 30, eps=5e-5)
    assert abs(c["energies"][-1] - a["energies"][-1]) < 1e-3


def _dense_setup(orc, n, na, nb, seed):
    h, g = synth.molecule_like(n, 2 * n, seed)
    P = orc.Problem(n, na, nb, h, g)
    H = P.dense_H()
    w, V = np.linalg.eigh(H)
    return P, w, V


def test_excited_state_by_projection_converges_to_next_eigenvalue(orc):
    # Sec. 4: project the found eigenvectors out of the effective Hamiltonian.
    # From a start that breaks every symmetry but S_z, the untruncated
    # iteration with the exact ground state projected out converges to the
    # second eigenvalue of the dense H, with two roots to the third.
    P, w, V = _dense_setup(orc, 6, 2, 2, 21)
    N = P.n_det
    rng = np.random.default_rng(3)
    r0 = np.arange(N, dtype=np.uint64)
    a0 = rng.standard_normal(N)
    root0 = (r0, V[:, 0])
    out = P.lanczos(r0, a0, None, 10, 80, roots=[root0])
    assert abs(out["energies"][-1] - w[1]) < 1e-8
    out2 = P.lanczos(r0, a0, None, 10, 80, roots=[root0, (r0, V[:, 1])])
    assert abs(out2["energies"][-1] - w[2]) < 1e-8
    # the final Psi is orthogonal to the roots
    psi = np.zeros(N)
    psi[out2["psi_rank"].astype(np.int64)] = out2["psi_amp"]
    assert abs(psi @ V[:, 0]) < 1e-10 * np.linalg.norm(psi)
    assert abs(psi @ V[:, 1]) < 1e-10 * np.linalg.norm(psi)


def test_no_roots_is_the_plain_iteration(orc):
    h, g = synth.molecule_like(8, 16, 0)
    P = orc.Problem(8, 3, 3, h, g)
    a = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 20)
    b = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 20, roots=[])
    assert np.array_equal(a["energies"], b["energies"]) and np.array_equal(a["psi_amp"], b["psi_amp"])


def test_halting_stops_at_the_first_small_change(orc):
    # Sec. 2.1: the run halts after block n once E(n-1) - E(n) < eps; the
    # blocks it runs are the full run's blocks, bit for bit
    P, _ = _dense_case(orc)
    full = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 5, 50)
    E = full["energies"]
    assert full["blocks_run"] == 10
    for eps in (1.0, 1e-2, 1e-4, 1e-6, 1e-12):
        out = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 5, 50, conv_eps=eps)
        nb = out["blocks_run"]
        assert np.array_equal(out["energies"][:nb], E[:nb])
        assert np.all(out["energies"][nb:] == 0.0)
        drops = E[:-1] - E[1:]
        first = next((b + 2 for b in range(len(drops)) if drops[b] < eps), 10)
        assert nb == first, (eps, nb, first)
    # eps = 1: the first block with a predecessor already halts
    assert P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 5, 50, conv_eps=1.0)["blocks_run"] == 2


def test_thread_count_does_not_change_bits(orc):
    # the bucketed parallel sigma (Sec. 2.2) and the parallel truncation sort
    # give the sequential results bit for bit
    P, _ = _dense_case(orc)
    rng = np.random.default_rng(8)
    r = np.sort(rng.choice(P.n_det, 600, replace=False)).astype(np.uint64)
    a = rng.normal(size=600)
    old = orc.get_threads()
    try:
        orc.set_threads(1)
        s1 = P.sigma(r, a, with_abs=True)
        l1 = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 200, 10, 20, want_T=True)
        orc.set_threads(5)
        s5 = P.sigma(r, a, with_abs=True)
        l5 = P.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 200, 10, 20, want_T=True)
    finally:
        orc.set_threads(old)
    for x, y in zip(s1, s5):
        assert np.array_equal(x, y)
    for k in ("energies", "psi_rank", "psi_amp", "T", "S"):
        assert np.array_equal(l1[k], l5[k]), k
