"""Host-side checks of the C ABI: the library loads and exports every symbol
that include/sfci.h declares; pure host calls work without a GPU."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2312_01846_amd import sfci

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sfci.LIB_PATH):
        from paper_2312_01846_amd import build

        build.build()
    return sfci.load_library()


def test_every_declared_symbol_is_exported(lib):
    declared = sfci.declared_symbols()
    assert "sfci_sigma" in declared and "sfci_lanczos" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", sfci.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {ln.split()[-1] for ln in out.stdout.splitlines() if " T " in ln}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(lib, s)
    # and the binding knows every declared call
    assert set(declared) <= set(sfci._SIGS)


def test_space_size_host_only(lib):
    from math import comb

    assert sfci.space_size(8, 3, 3) == 3136
    assert sfci.space_size(12, 6, 6) == 853776
    assert sfci.space_size(26, 5, 5) == comb(26, 5) ** 2
    assert sfci.space_size(28, 6, 6) == 141933027600
    assert sfci.space_size(32, 16, 16) == comb(32, 16) ** 2


def test_space_size_errors(lib):
    with pytest.raises(sfci.SfciError) as e:
        sfci.space_size(33, 1, 1)
    assert e.value.code == -8
    with pytest.raises(sfci.SfciError) as e:
        sfci.space_size(8, 9, 1)
    assert e.value.code == -1


def test_null_arguments_rejected(lib):
    rc = lib.sfci_problem_create(None, None, None, None, None)
    assert rc == -1
    assert b"NULL" in lib.sfci_last_error()
    assert lib.sfci_problem_destroy(None) == 0


def test_terms_per_source_formula():
    from math import comb

    for n, na, nb in [(8, 3, 3), (26, 5, 5), (28, 6, 6), (20, 4, 4), (12, 6, 6)]:
        sa, sb = na * (n - na), nb * (n - nb)
        want = 1 + sa + sb + comb(na, 2) * comb(n - na, 2) + comb(nb, 2) * comb(n - nb, 2) + sa * sb
        assert sfci.terms_per_source(n, na, nb) == want
    assert sfci.terms_per_source(26, 5, 5) == 15436
    assert sfci.terms_per_source(28, 6, 6) == 24619
