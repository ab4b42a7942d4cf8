"""The allocation-free truncation entry point (sfci_topm_noalloc) against
sfci_topm through the C ABI: same kept entries, same bits, on two calls in a
row with the second input smaller, plus the size limit."""
import ctypes as C

import numpy as np
import pytest

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


def _noalloc(S, torch, P, ranks, amps, M, normalise=False, tie_band=False):
    r = torch.as_tensor(ranks.astype(np.int64), device="cuda")
    a = torch.as_tensor(amps, dtype=torch.float64, device="cuda")
    cap = max(1, len(ranks))
    o_r = torch.empty(cap, dtype=torch.int64, device="cuda")
    o_a = torch.empty(cap, dtype=torch.float64, device="cuda")
    out = S.SVec(o_r.data_ptr(), o_a.data_ptr(), 0, cap)
    rc = S.load_library().sfci_topm_noalloc(P._h, C.byref(S._svec(r, a)), S.UINT64_MAX if M is None else int(M),
                                             1 if normalise else 0, 1 if tie_band else 0, C.byref(out))
    S._check(rc)
    k = int(out.nnz)
    return o_r[:k].cpu().numpy(), o_a[:k].cpu().numpy()


def test_noalloc_topm_matches_topm(torch, S):
    P = S.Problem(12, 6, 6, np.zeros((12, 12)), np.zeros(12 ** 4))
    rng = np.random.default_rng(21)
    big_r = np.sort(rng.choice(P.n_det, 300_000, replace=False)).astype(np.uint64)
    big_a = rng.normal(size=300_000)
    big_a[::9] = 0.25  # exact ties at the cut
    small_r = np.sort(rng.choice(P.n_det, 5_000, replace=False)).astype(np.uint64)
    small_a = rng.normal(size=5_000)
    for (r, a, M, norm, band) in [(big_r, big_a, 40_000, True, False), (small_r, small_a, 700, False, False),
                                  (small_r, small_a, 700, True, True), (big_r, big_a, None, False, False)]:
        gr, ga = P.topm(r.astype(np.int64), a, M, normalise=norm, tie_band=band)
        nr, na = _noalloc(S, torch, P, r, a, M, normalise=norm, tie_band=band)
        assert np.array_equal(nr, gr.cpu().numpy()), (len(r), M)
        assert np.array_equal(na, ga.cpu().numpy()), (len(r), M)


def test_noalloc_limits_and_errors(torch, S):
    P = S.Problem(8, 3, 3, np.zeros((8, 8)), np.zeros(8 ** 4))
    r = torch.as_tensor(np.array([1, 5, 9], dtype=np.int64), device="cuda")
    a = torch.ones(3, dtype=torch.float64, device="cuda")
    o = torch.empty(3, dtype=torch.int64, device="cuda")
    oa = torch.empty(3, dtype=torch.float64, device="cuda")
    out = S.SVec(o.data_ptr(), oa.data_ptr(), 0, 3)
    lib = S.load_library()
    too_big = S.SVec(r.data_ptr(), a.data_ptr(), (1 << 24) + 1, (1 << 24) + 1)  # rejected before any read
    assert lib.sfci_topm_noalloc(P._h, C.byref(too_big), 2, 0, 0, C.byref(out)) == -1
    assert b"at most" in lib.sfci_last_error()
    bad = torch.as_tensor(np.array([5, 1, 9], dtype=np.int64), device="cuda")
    assert lib.sfci_topm_noalloc(P._h, C.byref(S._svec(bad, a)), 2, 0, 0, C.byref(out)) == -3
    # still usable, and the capacity protocol reports the size needed
    small = S.SVec(o.data_ptr(), oa.data_ptr(), 0, 1)
    assert lib.sfci_topm_noalloc(P._h, C.byref(S._svec(r, a)), 2, 0, 0, C.byref(small)) == -4
    assert small.nnz == 2
    assert lib.sfci_topm_noalloc(P._h, C.byref(S._svec(r, a)), 2, 0, 0, C.byref(out)) == 0
    assert out.nnz == 2 and o[:2].cpu().tolist() == [1, 5]
