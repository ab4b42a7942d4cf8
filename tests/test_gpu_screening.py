"""The excitation screen (a double excitation's term H_ki v_i is dropped when
|H_ki v_i| < eps_x: the heat-bath idea named for future work in Sec. 4) on
the GPU against the oracle's screened sigma and iteration.  A term's value has
the same bits on both sides, so both take the same screening decisions:
deterministic mode is bit for bit, the fast modes differ only by summation
order."""
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


CASES = [("n10_4_3", 10, 4, 3, lambda: synth.molecule_like(10, 20, 5), 2500),
         ("n14_5_5_tiles", 14, 5, 5, lambda: synth.molecule_like(14, 28, 6), 3000),
         ("n20_4_4", 20, 4, 4, lambda: synth.molecule_like(20, 40, 9), 400)]


@pytest.mark.parametrize("name,n,na,nb,mk,nnz", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", ["dense", "dense_atomic", "sort"])
def test_screened_sigma_matches_oracle(torch, S, orc, monkeypatch, name, n, na, nb, mk, nnz, mode):
    if name.endswith("tiles"):
        monkeypatch.setenv("SFCI_TILE_MAX", "1024")  # rows of several tiles
    h, g = mk()
    P = S.Problem(n, na, nb, h, g)
    Po = orc.Problem(n, na, nb, h, g)
    r, a = synth.random_sparse_vector(P.n_det, nnz, seed=23)
    full_terms = P.sigma(r.astype(np.int64), a, dedup=mode, deterministic=(mode == "sort"))[2]["terms_emitted"]
    for eps in (1e-6, 1e-4):
        orr, oa, oab = Po.sigma(r, a, with_abs=True, eps_x=eps)
        gr, ga, st = P.sigma(r.astype(np.int64), a, dedup=mode, deterministic=(mode == "sort"), excite_eps=eps)
        gr, ga = _np(gr).astype(np.uint64), _np(ga)
        assert np.array_equal(gr, orr), eps
        if mode == "sort":
            assert np.array_equal(ga, oa)
        else:
            assert np.all(np.abs(ga - oa) <= 1e-12 * oab)
        assert st["terms_emitted"] < full_terms


@pytest.mark.parametrize("det", [True, False], ids=["deterministic", "fast"])
@pytest.mark.parametrize("no_dense", [False, True], ids=["dense", "list"])
def test_screened_iteration_matches_oracle(torch, S, orc, det, no_dense):
    # 10 orbitals with 4 alpha and 3 beta electrons: no alpha/beta exchange
    # symmetry, so no exact ties reach a truncation cut and the fast mode
    # must follow the oracle to 1e-9 Ha
    h, g = synth.molecule_like(10, 20, 5)
    P = S.Problem(10, 4, 3, h, g)
    Po = orc.Problem(10, 4, 3, h, g)
    eps = 1e-5
    ref = Po.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 1500, 10, 30, eps_x=eps)
    out = P.lanczos(np.array([0], dtype=np.int64), np.array([1.0]), M=1500, n_L=10, n_iter=30, deterministic=det,
                    excite_eps=eps, no_dense=no_dense)
    if det:
        assert np.array_equal(out["energies"], ref["energies"])
        assert np.array_equal(_np(out["psi_rank"]).astype(np.uint64), ref["psi_rank"])
    else:
        assert np.all(np.abs(out["energies"] - ref["energies"]) < 1e-9)
    unscreened = Po.lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 1500, 10, 30)
    assert not np.array_equal(unscreened["energies"], ref["energies"])


def test_screened_batch_deterministic(torch, S, orc):
    h, g = synth.molecule_like(10, 20, 5)
    P = S.Problem(10, 4, 3, h, g)
    B = S.Batch([P])
    out = B.lanczos([(np.array([0], dtype=np.int64), np.array([1.0]))], [1500], n_L=10, n_iter=20,
                    deterministic=True, want_grad=False, excite_eps=1e-5)
    ref = orc.Problem(10, 4, 3, h, g).lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 1500, 10, 20,
                                              eps_x=1e-5)
    assert np.array_equal(out["energies"][0], ref["energies"])
