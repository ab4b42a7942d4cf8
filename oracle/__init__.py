"""CPU oracle for the sparse-FCI sigma = H v path -- TEST INFRASTRUCTURE ONLY.

Loads ``liboracle.so`` (built from ``sfci_oracle.cpp`` by :func:`build`) and
wraps it with numpy.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the product library never imports it.

Parity status of each function is listed in the header of sfci_oracle.cpp;
every function here is pinned by tests under ``tests/`` (none is unpinned).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfci_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain host code; no GPU involvement)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", *CFLAGS, "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        i32, i64, u64, dbl = C.c_int, C.c_int64, C.c_uint64, C.c_double
        vp = C.c_void_p
        L.orc_binom.restype = u64; L.orc_binom.argtypes = [i32, i32]
        L.orc_str_rank.restype = u64; L.orc_str_rank.argtypes = [u64]
        L.orc_str_unrank.restype = u64; L.orc_str_unrank.argtypes = [u64, i32]
        L.orc_gchain_next.restype = i32; L.orc_gchain_next.argtypes = [u64, i32, C.POINTER(u64)]
        L.orc_space_size.restype = u64; L.orc_space_size.argtypes = [i32, i32, i32]
        L.orc_det_rank.restype = None; L.orc_det_rank.argtypes = [i32, i32, i32, u64p, u64p, i64, u64p]
        L.orc_det_unrank.restype = None; L.orc_det_unrank.argtypes = [i32, i32, i32, u64p, i64, u64p, u64p]
        L.orc_sigma_explicit.restype = i32
        L.orc_sigma_explicit.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, f64p]
        L.orc_dense_H.restype = i32; L.orc_dense_H.argtypes = [i32, i32, i32, f64p, f64p, f64p]
        L.orc_element.restype = dbl; L.orc_element.argtypes = [i32, i32, i32, f64p, f64p, u64, u64]
        L.orc_source_terms.restype = i64
        L.orc_source_terms.argtypes = [i32, i32, i32, f64p, f64p, u64, vp, vp, i64]
        L.orc_sigma.restype = i64
        L.orc_sigma.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, vp, vp, vp, i64]
        L.orc_sigma_x.restype = i64
        L.orc_sigma_x.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, vp, vp, vp, i64, dbl]
        L.orc_sigma_entry.restype = dbl
        L.orc_sigma_entry.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, u64, C.POINTER(dbl)]
        L.orc_topm.restype = i64; L.orc_topm.argtypes = [i64, u64p, f64p, i64, u64p, f64p]
        L.orc_topm_band.restype = i64; L.orc_topm_band.argtypes = [i64, u64p, f64p, i64, u64p, f64p, i32]
        L.orc_normalize.restype = dbl; L.orc_normalize.argtypes = [i64, f64p]
        L.orc_jacobi.restype = None; L.orc_jacobi.argtypes = [i32, f64p, f64p, f64p]
        L.orc_geneig.restype = i32; L.orc_geneig.argtypes = [i32, f64p, f64p, C.POINTER(dbl), f64p]
        L.orc_lanczos.restype = i64
        L.orc_lanczos.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, i64, i32, i32, f64p, vp, vp, vp,
                                  vp, i64, dbl]
        L.orc_lanczos_roots.restype = i64
        L.orc_lanczos_roots.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, i64, i32, i32, f64p, vp, vp,
                                        vp, vp, i64, dbl, i32, vp, vp, vp]
        L.orc_lanczos_ex.restype = i64
        L.orc_lanczos_ex.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, i64, i32, i32, f64p, vp, vp,
                                     vp, vp, i64, dbl, i32, vp, vp, vp, i32, dbl, C.POINTER(i32), vp, dbl]
        L.orc_set_threads.restype = None; L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32; L.orc_get_threads.argtypes = []
        L.orc_pt2.restype = i32
        L.orc_pt2.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, C.POINTER(dbl), C.POINTER(dbl),
                              C.POINTER(u64)]
        for nm in ("orc_backward_explicit", "orc_backward_sc"):
            f = getattr(L, nm)
            f.restype = i32
            f.argtypes = [i32, i32, i32, f64p, f64p, i64, u64p, f64p, i64, u64p, f64p, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


class Problem:
    """Integrals (h, g) of one (n, n_alpha, n_beta) space, as the oracle sees them."""

    def __init__(self, n, na, nb, h, g):
        self.n, self.na, self.nb = int(n), int(na), int(nb)
        self.h = _f64(h).reshape(self.n, self.n)
        self.g = _f64(g).reshape(self.n, self.n, self.n, self.n)
        self.hf = self.h.ravel()
        self.gf = self.g.ravel()
        self.n_det = int(lib().orc_space_size(self.n, self.na, self.nb))
        self.n_beta_str = int(lib().orc_binom(self.n, self.nb))

    def _a(self):
        return (self.n, self.na, self.nb, self.hf, self.gf)

    # ranks --------------------------------------------------------------
    def rank(self, a_bits, b_bits):
        a, b = _u64(a_bits), _u64(b_bits)
        out = np.empty(a.size, dtype=np.uint64)
        lib().orc_det_rank(self.n, self.na, self.nb, a, b, a.size, out)
        return out

    def unrank(self, ranks):
        r = _u64(ranks)
        a = np.empty(r.size, dtype=np.uint64)
        b = np.empty(r.size, dtype=np.uint64)
        lib().orc_det_unrank(self.n, self.na, self.nb, r, r.size, a, b)
        return a, b

    # sigma ----------------------------------------------------------------
    def sigma_explicit_dense(self, ranks, amps):
        out = np.zeros(self.n_det, dtype=np.float64)
        rc = lib().orc_sigma_explicit(*self._a(), len(ranks), _u64(ranks), _f64(amps), out)
        assert rc == 0
        return out

    def dense_H(self):
        N = self.n_det
        out = np.zeros(N * N, dtype=np.float64)
        rc = lib().orc_dense_H(*self._a(), out)
        assert rc == 0, rc
        return out.reshape(N, N)

    def element(self, src, tgt):
        return lib().orc_element(*self._a(), int(src), int(tgt))

    def source_terms(self, src):
        need = lib().orc_source_terms(*self._a(), int(src), None, None, 0)
        t = np.empty(need, dtype=np.uint64)
        e = np.empty(need, dtype=np.float64)
        lib().orc_source_terms(*self._a(), int(src), _ptr(t), _ptr(e), need)
        return t, e

    def sigma(self, ranks, amps, with_abs=False, eps_x=0.0):
        """eps_x > 0: double-excitation terms with |H_ki v_i| < eps_x are not generated."""
        r, a = _u64(ranks), _f64(amps)
        need = lib().orc_sigma_x(*self._a(), r.size, r, a, None, None, None, 0, float(eps_x))
        if need == -1:
            raise ValueError("invalid input vector")
        cnt = -need if need < 0 else need
        orank = np.empty(cnt, dtype=np.uint64)
        oamp = np.empty(cnt, dtype=np.float64)
        oabs = np.empty(cnt, dtype=np.float64)
        got = lib().orc_sigma_x(*self._a(), r.size, r, a, _ptr(orank), _ptr(oamp), _ptr(oabs), cnt, float(eps_x))
        assert got == cnt
        return (orank, oamp, oabs) if with_abs else (orank, oamp)

    def sigma_entry(self, ranks, amps, target):
        ab = C.c_double(0.0)
        v = lib().orc_sigma_entry(*self._a(), len(ranks), _u64(ranks), _f64(amps), int(target), C.byref(ab))
        return v, ab.value

    def lanczos(self, ranks0, amps0, M, n_L, n_iter, want_T=False, eps=0.0, roots=None, tie_band=False,
                conv_eps=0.0, eps_x=0.0):
        """roots: list of (ranks, amps) of previously found eigenvectors to project out.
        tie_band: the truncation extension of orc_topm_band (default: the paper's rule).
        conv_eps > 0: halt after block n >= 1 once E(n-1) - E(n) < conv_eps; the
        result's "blocks_run" says how many blocks ran (energies beyond it stay 0)."""
        M = -1 if M is None else int(M)
        nblk = n_iter // n_L
        en = np.zeros(nblk, dtype=np.float64)
        T = np.zeros(nblk * n_L * n_L, dtype=np.float64)
        S = np.zeros(nblk * n_L * n_L, dtype=np.float64)
        r0, a0 = _u64(ranks0), _f64(amps0)
        roots = roots or []
        off = np.zeros(len(roots) + 1, dtype=np.int64)
        for i, (rr, _) in enumerate(roots):
            off[i + 1] = off[i] + len(rr)
        rcat = _u64(np.concatenate([np.asarray(rr, dtype=np.uint64) for rr, _ in roots]) if roots
                    else np.zeros(1, dtype=np.uint64))
        acat = _f64(np.concatenate([np.asarray(aa, dtype=np.float64) for _, aa in roots]) if roots
                    else np.zeros(1))
        nrun = C.c_int(0)
        bnnz = np.zeros(nblk * n_L, dtype=np.int64)
        args = (float(eps), len(roots), _ptr(off), _ptr(rcat), _ptr(acat), 1 if tie_band else 0, float(conv_eps),
                C.byref(nrun), _ptr(bnnz), float(eps_x))
        # Psi holds at most n_L truncated vectors (or the whole space): one run
        # fills it; a second run happens only if that bound is too small
        cap = self.n_det if M < 0 else min(self.n_det, n_L * (M + (256 if tie_band else 0)))
        pr = np.empty(max(cap, 1), dtype=np.uint64)
        pa = np.empty(max(cap, 1), dtype=np.float64)
        need = lib().orc_lanczos_ex(*self._a(), r0.size, r0, a0, M, n_L, n_iter, en, _ptr(T), _ptr(S), _ptr(pr),
                                    _ptr(pa), cap, *args)
        if need < 0:
            raise RuntimeError("oracle lanczos failed")
        if need > cap:
            pr = np.empty(need, dtype=np.uint64)
            pa = np.empty(need, dtype=np.float64)
            lib().orc_lanczos_ex(*self._a(), r0.size, r0, a0, M, n_L, n_iter, en, None, None, _ptr(pr), _ptr(pa),
                                 need, *args)
        pr, pa = pr[:need].copy(), pa[:need].copy()
        out = dict(energies=en, psi_rank=pr, psi_amp=pa, blocks_run=int(nrun.value),
                   basis_nnz=bnnz.reshape(nblk, n_L))
        if want_T:
            out["T"] = T.reshape(nblk, n_L, n_L)
            out["S"] = S.reshape(nblk, n_L, n_L)
        return out

    def pt2(self, ranks, amps):
        """Second-order Epstein-Nesbet correction of Psi: (E0, E2, number of external determinants)."""
        e0, e2, ne = C.c_double(0.0), C.c_double(0.0), C.c_uint64(0)
        rc = lib().orc_pt2(*self._a(), len(ranks), _u64(ranks), _f64(amps), C.byref(e0), C.byref(e2), C.byref(ne))
        if rc != 0:
            raise ValueError("invalid input vector")
        return e0.value, e2.value, int(ne.value)

    def backward(self, v_rank, v_amp, s_rank, s_amp, explicit=False):
        n = self.n
        vbar = np.zeros(len(v_rank), dtype=np.float64)
        dh = np.zeros(n * n, dtype=np.float64)
        dg = np.zeros(n ** 4, dtype=np.float64)
        f = lib().orc_backward_explicit if explicit else lib().orc_backward_sc
        rc = f(*self._a(), len(v_rank), _u64(v_rank), _f64(v_amp), len(s_rank), _u64(s_rank), _f64(s_amp),
               _ptr(vbar), _ptr(dh), _ptr(dg))
        assert rc == 0
        return vbar, dh.reshape(n, n), dg.reshape(n, n, n, n)


# free functions ---------------------------------------------------------------
def set_threads(t):
    """Threads of the oracle's sigma (Sec. 2.2's parallel form: per-thread
    buckets, per-bucket stable sort and merge) and of its truncation sort.
    Every result has the same bits for any thread count."""
    lib().orc_set_threads(int(t))


def get_threads():
    return int(lib().orc_get_threads())

def binom(a, b):
    return int(lib().orc_binom(int(a), int(b)))


def str_rank(bits):
    return int(lib().orc_str_rank(int(bits)))


def str_unrank(r, k):
    return int(lib().orc_str_unrank(int(r), int(k)))


def gchain_next(bits, n):
    out = C.c_uint64(0)
    ok = lib().orc_gchain_next(int(bits), int(n), C.byref(out))
    return int(out.value) if ok else None


def space_size(n, na, nb):
    return int(lib().orc_space_size(n, na, nb))


def topm(ranks, amps, M, tie_band=False):
    r, a = _u64(ranks), _f64(amps)
    orank = np.empty(r.size, dtype=np.uint64)
    oamp = np.empty(r.size, dtype=np.float64)
    k = lib().orc_topm_band(r.size, r, a, -1 if M is None else int(M), orank, oamp, 1 if tie_band else 0)
    return orank[:k].copy(), oamp[:k].copy()


def normalize(amps):
    a = _f64(amps).copy()
    nrm = lib().orc_normalize(a.size, a)
    return a, nrm


def jacobi(A):
    A = _f64(A).copy()
    m = A.shape[0]
    V = np.zeros((m, m), dtype=np.float64)
    w = np.zeros(m, dtype=np.float64)
    lib().orc_jacobi(m, A.ravel(), V.ravel(), w)
    return w, V


def geneig(T, S):
    m = T.shape[0]
    lam = C.c_double(0.0)
    x = np.zeros(m, dtype=np.float64)
    r = lib().orc_geneig(m, _f64(T).ravel(), _f64(S).ravel(), C.byref(lam), x)
    return lam.value, x, r
