"""The SFCI iteration and truncated sigma without an N_det array (sort path,
alpha-range passes, running top-M candidate list).

With the tuple buffer forced small, every sigma runs as many passes; the
deterministic results must still equal the oracle's goldens and the dense
deterministic iteration bit for bit (T, S, energies, Psi)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2312_01846_amd import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lanczos_energies.json")


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


def _gold(name):
    data = json.load(open(GOLD)) if os.path.exists(GOLD) else {}
    if name not in data:
        pytest.skip(f"golden value {name} not generated")
    return data[name]


def _sha(r):
    return hashlib.sha256(np.ascontiguousarray(r, dtype=np.uint64).tobytes()).hexdigest()[:16]


def _np(t):
    return t.detach().cpu().numpy()


AUFBAU = (np.array([0], dtype=np.int64), np.array([1.0]))


def _perturbed(P):
    st = synth.perturbed_start(P.n, P.na, P.nb)
    r0 = P.rank([t[0] for t in st], [t[1] for t in st]).cpu().numpy()
    a0 = np.array([t[2] for t in st])
    o = np.argsort(r0, kind="stable")
    return r0[o], a0[o]


def _case(S, name):
    """(problem, start, tuple cap forcing several passes) for a golden case."""
    if name.startswith("c0"):
        h, g = synth.molecule_like(8, 16, 0)
        P = S.Problem(8, 3, 3, h, g)
        return P, (_perturbed(P) if name.startswith("c0p") else AUFBAU), 20_000
    if name.startswith("c1"):
        h, g = synth.hubbard_ring(12, 1.0, 4.0)
        P = S.Problem(12, 6, 6, h, g)
        a, b = synth.neel_bits(12)
        return P, (P.rank([a], [b]).cpu().numpy(), np.array([1.0])), 1 << 20
    if name.startswith("c2"):
        h, g = synth.molecule_like(26, 52, 2)
        P = S.Problem(26, 5, 5, h, g)
        return P, (_perturbed(P) if name.startswith("c2p") else AUFBAU), 1 << 23
    if name.startswith("c3"):
        h, g = synth.molecule_like(28, 56, 3)
        P = S.Problem(28, 6, 6, h, g)
        return P, (_perturbed(P) if name.startswith("c3p") else AUFBAU), 1 << 23
    j = int(name.split("_")[1].replace("inst", ""))
    _, h, g = synth.bond_stretch_batch(20, 32, 40)[j]
    P = S.Problem(20, 4, 4, h, g)
    return P, (_perturbed(P) if name.startswith("c4p") else AUFBAU), 1 << 22


@pytest.mark.parametrize("name", ["c0_M300_30", "c0p_M300_30", "c1_U4_M2e3_20", "c2_M2e3_20", "c2p_M2e3_20",
                                  "c4_inst31_M3e3_30", "c3_M1e3_10", "c3p_M1e3_10"])
def test_list_iteration_matches_goldens(torch, S, monkeypatch, name):
    # c3*: 12 electrons in 28 orbitals, 1.42e11 determinants -- the N_det
    # array (1.14 TB) cannot exist, so this is the only way the space runs
    gd = _gold(name)
    P, start, tup_cap = _case(S, name)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", str(tup_cap))
    out = P.lanczos(*start, M=gd["M"], n_L=gd["n_L"], n_iter=gd["n_iter"], deterministic=True, no_dense=True)
    assert out["energies"].tolist() == gd["energies"]
    assert _sha(_np(out["psi_rank"])) == gd["psi_support_sha"]
    assert int(out["psi_rank"].numel()) == gd["psi_nnz"]


def test_list_iteration_equals_dense_bitwise(torch, S, monkeypatch):
    # same T, S, energies and untruncated Psi as the dense deterministic iteration
    P, start, tup_cap = _case(S, "c4p_inst31_M3e3_30")
    dense = P.lanczos(*start, M=3000, n_L=10, n_iter=20, deterministic=True, want_T=True)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", str(tup_cap))
    lst = P.lanczos(*start, M=3000, n_L=10, n_iter=20, deterministic=True, want_T=True, no_dense=True)
    assert np.array_equal(lst["T"], dense["T"]) and np.array_equal(lst["S"], dense["S"])
    assert np.array_equal(lst["energies"], dense["energies"])
    assert np.array_equal(_np(lst["psi_rank"]), _np(dense["psi_rank"]))
    assert np.array_equal(_np(lst["psi_amp"]), _np(dense["psi_amp"]))
    assert lst["stats"]["terms_emitted"] == dense["stats"]["terms_emitted"]


def test_list_iteration_untruncated_matches_oracle(torch, S, orc, monkeypatch):
    # M = all: the candidate list is never cut; plain Lanczos, bit for bit
    gd = _gold("c0_Mall_30")
    h, g = synth.molecule_like(8, 16, 0)
    P = S.Problem(8, 3, 3, h, g)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", "50000")
    out = P.lanczos(*AUFBAU, M=None, n_L=10, n_iter=30, deterministic=True, want_T=True, no_dense=True)
    ref = orc.Problem(8, 3, 3, h, g).lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), None, 10, 30,
                                             want_T=True)
    assert out["energies"].tolist() == gd["energies"]
    assert np.array_equal(out["T"], ref["T"]) and np.array_equal(out["S"], ref["S"])
    assert np.array_equal(_np(out["psi_rank"]).astype(np.uint64), ref["psi_rank"])
    assert np.array_equal(_np(out["psi_amp"]), ref["psi_amp"])


@pytest.mark.parametrize("sigma", ["tile", "sort", "auto"])
@pytest.mark.parametrize("name,rows", [("c2p_M2e3_20", 5000), ("c4p_inst31_M3e3_30", 700), ("c3p_M1e3_10", 30000)])
def test_list_iteration_fast_mode(torch, S, monkeypatch, name, rows, sigma):
    # fast mode: sigma through the tile kernel (its finished tiles consumed in
    # the kernel, a range of target rows per pass), or through the sort path,
    # or the per-sigma choice between them; tree reductions; perturbed starts
    # with the tie band (near-ties at a cut kept together): energies within
    # 1e-9 Ha of the oracle's iteration with the band at equal M
    gd = _gold(name.replace("p_", "pband_", 1))
    P, start, _ = _case(S, name)
    monkeypatch.setenv("SFCI_LIST_PASS_ROWS", str(rows))
    if sigma != "auto":
        monkeypatch.setenv("SFCI_LIST_SIGMA", sigma)
    out = P.lanczos(*start, M=gd["M"], n_L=gd["n_L"], n_iter=gd["n_iter"], deterministic=False, no_dense=True,
                    tie_band=True)
    dE = np.abs(out["energies"] - np.array(gd["energies"]))
    assert np.all(dE < 1e-9), dE


@pytest.mark.parametrize("eps", [5e-5, 2e-3])
def test_list_iteration_screening_matches_oracle(torch, S, orc, monkeypatch, eps):
    h, g = synth.molecule_like(8, 16, 0)
    P = S.Problem(8, 3, 3, h, g)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", "20000")
    out = P.lanczos(*AUFBAU, M=300, n_L=10, n_iter=30, deterministic=True, screen_eps=eps, no_dense=True)
    ref = orc.Problem(8, 3, 3, h, g).lanczos(np.array([0], dtype=np.uint64), np.array([1.0]), 300, 10, 30, eps=eps)
    assert np.array_equal(out["energies"], ref["energies"])
    assert np.array_equal(_np(out["psi_rank"]).astype(np.uint64), ref["psi_rank"])


@pytest.mark.parametrize("M", [1, 257, 5000, None])
def test_sigma_topm_in_passes_matches_oracle(torch, S, orc, monkeypatch, M):
    # sfci_sigma's sort path: passes + running candidate list, the same top-M
    # (tie rule included) as the oracle's full sort, sorted by rank
    _, h, g = synth.bond_stretch_batch(20, 32, 40)[5]
    P = S.Problem(20, 4, 4, h, g)
    r0, a0 = _perturbed(P)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", str(1 << 17))
    r, a, st = P.sigma(r0, a0, M=M, deterministic=True)
    Po = orc.Problem(20, 4, 4, h, g)
    fr, fa = Po.sigma(np.ascontiguousarray(r0, dtype=np.uint64), np.ascontiguousarray(a0))
    rr, ra = (fr, fa) if M is None else orc.topm(fr, fa, M)
    assert np.array_equal(_np(r).astype(np.uint64), rr)
    assert np.array_equal(_np(a), ra)
    assert st["candidates"] == int(np.count_nonzero(fa))


@pytest.mark.parametrize("case", ["c0", "hubbard", "n20", "n26"])
def test_row_emission_equals_source_emission(torch, S, monkeypatch, case):
    # target-row-driven passes (per-row counts, sorted pair lists, exact-zero
    # elements emitted) against the source-driven passes: identical sigma,
    # identical count of nonzero elements
    if case == "c0":
        h, g = synth.molecule_like(8, 16, 0)
        P = S.Problem(8, 3, 3, h, g)
    elif case == "hubbard":
        h, g = synth.hubbard_ring(12, 1.0, 4.0)
        P = S.Problem(12, 6, 6, h, g)
    elif case == "n20":
        _, h, g = synth.bond_stretch_batch(20, 32, 40)[9]
        P = S.Problem(20, 4, 4, h, g)
    else:
        h, g = synth.molecule_like(26, 52, 2)
        P = S.Problem(26, 5, 5, h, g)
    r0, a0 = _perturbed(P)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", str(1 << 20))
    r1, a1, s1 = P.sigma(r0, a0, deterministic=True)
    # without the beta-single table the alpha-single pairs rank every option
    monkeypatch.setenv("SFCI_RP_NO_T1", "1")
    r3, a3, s3 = P.sigma(r0, a0, deterministic=True)
    monkeypatch.delenv("SFCI_RP_NO_T1")
    monkeypatch.setenv("SFCI_SORT_EMIT", "source")
    r2, a2, s2 = P.sigma(r0, a0, deterministic=True)
    for r, a, s in ((r2, a2, s2), (r3, a3, s3)):
        assert np.array_equal(_np(r1), _np(r))
        assert np.array_equal(_np(a1), _np(a))
        assert s1["terms_emitted"] == s["terms_emitted"]


@pytest.mark.parametrize("mode", ["deterministic", "fast_band", "fast"])
def test_28_orbitals_M1e4_goldens(torch, S, monkeypatch, mode):
    # 12 electrons in 28 orbitals at M = 1e4, two blocks of N_L = 5 (2.5e8
    # terms per sigma): deterministic from the aufbau determinant bit for bit
    # against the oracle; fast (the tile kernel forced, finished tiles
    # consumed in the kernel) from the perturbed start with the tie band within
    # 1e-9 Ha of the oracle's iteration with the band, and under the paper's
    # rule reported against the oracle (ties at a cut may split differently)
    name = {"deterministic": "c3_M1e4_10", "fast_band": "c3pband_M1e4_10", "fast": "c3p_M1e4_10"}[mode]
    gd = _gold(name)
    P, start, tup_cap = _case(S, name)
    monkeypatch.setenv("SFCI_SORT_TUPLE_CAP", str(tup_cap))
    if mode != "deterministic":
        monkeypatch.setenv("SFCI_LIST_SIGMA", "tile")
    out = P.lanczos(*start, M=gd["M"], n_L=gd["n_L"], n_iter=gd["n_iter"], deterministic=(mode == "deterministic"),
                    no_dense=True, tie_band=(mode == "fast_band"))
    dE = np.abs(out["energies"] - np.array(gd["energies"]))
    if mode == "deterministic":
        assert out["energies"].tolist() == gd["energies"]
        assert _sha(_np(out["psi_rank"])) == gd["psi_support_sha"]
    elif mode == "fast_band":
        assert np.all(dE < 1e-9), dE
    else:
        print(f"28 orbitals, M = 1e4, fast under the paper's rule: |dE| = {dE}")
        assert np.all(dE < 1e-2), dE
