"""Second-order Epstein-Nesbet correction on the GPU against the oracle.

Deterministic mode (sort-path sigma, every sum in ascending rank, the
diagonal element in its fixed addition order, IEEE division on both sides)
must give E0, E2 and the external count bit for bit; the fast mode (dense
tile kernel, tree sums) within 1e-12 relative on E0 and 1e-10 on E2 (each
sigma entry carries ~1e-16 relative rounding, squared and divided by
denominators bounded away from zero for these vectors)."""
import numpy as np
import pytest

from paper_2312_01846_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def S():
    from paper_2312_01846_amd import sfci

    sfci.load_library()
    return sfci


def _np(t):
    return t.detach().cpu().numpy()


def _perturbed(P):
    st = synth.perturbed_start(P.n, P.na, P.nb)
    r0 = P.rank([t[0] for t in st], [t[1] for t in st]).cpu().numpy()
    a0 = np.array([t[2] for t in st])
    o = np.argsort(r0, kind="stable")
    return r0[o], a0[o]


def _case(S, name):
    if name == "n8":
        h, g = synth.molecule_like(8, 16, 0)
        return S.Problem(8, 3, 3, h, g), (8, 3, 3, h, g)
    if name == "n20":
        _, h, g = synth.bond_stretch_batch(20, 32, 40)[12]
        return S.Problem(20, 4, 4, h, g), (20, 4, 4, h, g)
    if name == "n26":
        h, g = synth.molecule_like(26, 52, 2)
        return S.Problem(26, 5, 5, h, g), (26, 5, 5, h, g)
    h, g = synth.molecule_like(28, 56, 3)
    return S.Problem(28, 6, 6, h, g), (28, 6, 6, h, g)


def _vectors(P, name):
    out = [(np.array([0], dtype=np.int64), np.array([1.0])), _perturbed(P)]
    if name in ("n8", "n20"):
        # a truncated variational vector from a short deterministic run
        M = 300 if name == "n8" else 2000
        run = P.lanczos(*_perturbed(P), M=M, n_L=5, n_iter=10, deterministic=True)
        r, a = P.topm(run["psi_rank"], run["psi_amp"], M, normalise=True)
        out.append((_np(r), _np(a)))
    return out


@pytest.mark.parametrize("name", ["n8", "n20", "n26", "n28"])
def test_pt2_deterministic_matches_oracle_bitwise(torch, S, orc, name):
    P, args = _case(S, name)
    Po = orc.Problem(*args)
    for r, a in _vectors(P, name):
        e0, e2, ne = P.pt2(r, a, deterministic=True)
        o0, o2, on = Po.pt2(np.ascontiguousarray(r, dtype=np.uint64), np.ascontiguousarray(a))
        assert (e0, e2, ne) == (o0, o2, on), (name, len(r))


def _e2_bound(Po, args, r, a, e0):
    """Rounding bound of E2 when sigma and the sums are reordered: ~1e-12 per
    term (relative) plus E0's error (1e-12 relative, tested) times the
    sensitivity sum y^2 / (E0 - H_kk)^2, which small denominators amplify.
    The diagonal elements here only size the tolerance."""
    n, na, nb, h, g = args
    yr, ya = Po.sigma(r, a)
    ext = ~np.isin(yr, r)
    yr, ya = yr[ext], ya[ext]
    A, B = Po.unrank(yr)
    occA = ((A[:, None] >> np.arange(n, dtype=np.uint64)) & 1).astype(bool)
    occB = ((B[:, None] >> np.arange(n, dtype=np.uint64)) & 1).astype(bool)
    hd = np.diag(h)
    J = np.einsum("ppqq->pq", g)
    K = np.einsum("pqqp->pq", g)
    JK = np.triu(J - K, 1)
    fa, fb = occA.astype(float), occB.astype(float)
    hkk = (fa @ hd + fb @ hd + np.einsum("ip,pq,iq->i", fa, JK, fa) + np.einsum("ip,pq,iq->i", fb, JK, fb)
           + np.einsum("ip,pq,iq->i", fa, J, fb))
    d = e0 - hkk
    nn = float(a @ a)
    return (1e-12 * np.sum(np.abs(ya ** 2 / d)) + 1e-12 * abs(e0) * np.sum(ya ** 2 / d ** 2)) / nn


@pytest.mark.parametrize("name", ["n8", "n20", "n26", "n28"])
def test_pt2_fast_within_tolerance(torch, S, orc, name):
    P, args = _case(S, name)
    Po = orc.Problem(*args)
    for r, a in _vectors(P, name):
        r = np.ascontiguousarray(r, dtype=np.uint64)
        a = np.ascontiguousarray(a)
        e0, e2, ne = P.pt2(r.astype(np.int64), a, deterministic=False)
        o0, o2, on = Po.pt2(r, a)
        assert ne == on
        assert abs(e0 - o0) <= 1e-12 * abs(o0)
        tol = _e2_bound(Po, args, r, a, o0)
        assert abs(e2 - o2) <= tol, (name, len(r), e2, o2, tol)


def test_pt2_rejects_empty(torch, S):
    P, _ = _case(S, "n8")
    with pytest.raises(S.SfciError):
        P.pt2(np.zeros(0, dtype=np.int64), np.zeros(0))
