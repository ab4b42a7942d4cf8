"""Python binding of libsfci (ctypes).  Argument marshalling only: every step
of sigma = H v, truncation and the SFCI iteration runs in the HIP kernels of
``libsfci.so``.  PyTorch provides device memory and the stream.

If the library is missing or the GPU is absent, calls raise -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfci.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADER = os.path.join(INCLUDE, "sfci.h")

UINT64_MAX = (1 << 64) - 1
TIE_SLACK = 256  # SFCI_TIE_SLACK: with the tie band a truncated vector holds at most M + TIE_SLACK entries

SFCI_OK = 0
STATUS = {0: "SFCI_OK", -1: "SFCI_E_ARG", -2: "SFCI_E_RANGE", -3: "SFCI_E_DUP", -4: "SFCI_E_CAPACITY",
          -5: "SFCI_E_NOMEM", -6: "SFCI_E_DEVICE", -7: "SFCI_E_NOTSYM", -8: "SFCI_E_UNSUPPORTED"}
DEDUP = {"auto": 0, "dense": 1, "sort": 2, "dense_atomic": 3}


class SfciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Space(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32)]


class SVec(C.Structure):
    _fields_ = [("rank", C.c_void_p), ("amp", C.c_void_p), ("nnz", C.c_uint64), ("capacity", C.c_uint64)]


class SigmaOpts(C.Structure):
    _fields_ = [("M", C.c_uint64), ("dedup", C.c_int32), ("deterministic", C.c_int32), ("screen_eps", C.c_double),
                ("tie_band", C.c_int32), ("reserved", C.c_int32), ("excite_eps", C.c_double)]


class SigmaStats(C.Structure):
    _fields_ = [("terms_enumerated", C.c_uint64), ("terms_emitted", C.c_uint64), ("candidates", C.c_uint64),
                ("ms", C.c_double)]


class LanczosOpts(C.Structure):
    _fields_ = [("M", C.c_uint64), ("n_L", C.c_int32), ("n_iter", C.c_int32), ("deterministic", C.c_int32),
                ("dedup", C.c_int32), ("screen_eps", C.c_double), ("no_dense", C.c_int32),
                ("autotune", C.c_int32), ("conv_eps", C.c_double), ("tie_band", C.c_int32), ("reserved", C.c_int32),
                ("excite_eps", C.c_double)]


class LanczosStats(C.Structure):
    _fields_ = [("sigma_calls", C.c_uint64), ("terms_enumerated", C.c_uint64), ("terms_emitted", C.c_uint64),
                ("sigma_ms", C.c_double), ("total_ms", C.c_double), ("blocks_run", C.c_int32),
                ("reserved", C.c_int32)]


class BatchStats(C.Structure):
    _fields_ = [("fwd_ms", C.c_double), ("bwd_ms", C.c_double), ("sigma_ms", C.c_double),
                ("terms_emitted", C.c_uint64), ("nnz_in_total", C.c_uint64), ("sigma_calls", C.c_uint64),
                ("psi_nnz_total", C.c_uint64),
                ("graph_replayed_blocks", C.c_int32), ("batched_sigma", C.c_int32), ("tune_trials", C.c_int32),
                ("tune_b1_chunk", C.c_uint32), ("tune_bb_chunk", C.c_uint32), ("tune_per_cu", C.c_uint32),
                ("tune_default_ms", C.c_double), ("tune_best_ms", C.c_double), ("sigma_in_graph", C.c_int32),
                ("graphs_reused", C.c_int32)]


class Roof(C.Structure):
    _fields_ = [("copy_GBps", C.c_double), ("gather_Gops", C.c_double * 3), ("atomic_Gops", C.c_double * 3),
                ("lds_atomic_Gops", C.c_double * 2), ("lds_read_Gops", C.c_double), ("big_bytes", C.c_uint64)]


_lib = None

# Every function the header declares, with its ctypes signature.
_SIGS = {
    "sfci_space_size": (C.c_int, [C.POINTER(Space), C.POINTER(C.c_uint64)]),
    "sfci_problem_create": (C.c_int, [C.POINTER(Space), C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "sfci_problem_destroy": (C.c_int, [C.c_void_p]),
    "sfci_rank": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "sfci_unrank": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "sfci_sigma": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.POINTER(SigmaOpts), C.POINTER(SVec),
                             C.POINTER(SigmaStats)]),
    "sfci_topm": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.c_uint64, C.c_int32, C.c_int32, C.POINTER(SVec)]),
    "sfci_lanczos": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.POINTER(LanczosOpts), C.c_void_p, C.POINTER(SVec),
                               C.c_void_p, C.c_void_p, C.POINTER(LanczosStats)]),
    "sfci_lanczos_roots": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.POINTER(LanczosOpts), C.POINTER(SVec),
                                     C.c_int32, C.c_void_p, C.POINTER(SVec), C.c_void_p, C.c_void_p,
                                     C.POINTER(LanczosStats)]),
    "sfci_sigma_backward": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.POINTER(SVec), C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "sfci_pt2": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                           C.POINTER(C.c_uint64)]),
    "sfci_energy_gradients": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                                        C.c_void_p]),
    "sfci_batch_create": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "sfci_batch_destroy": (C.c_int, [C.c_void_p]),
    "sfci_batch_lanczos": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.POINTER(C.c_uint64), C.POINTER(LanczosOpts),
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(BatchStats)]),
    "sfci_last_error": (C.c_char_p, []),
    "sfci_roof_probe": (C.c_int, [C.c_uint64, C.c_void_p, C.POINTER(Roof)]),
    "sfci_topm_noalloc": (C.c_int, [C.c_void_p, C.POINTER(SVec), C.c_uint64, C.c_int32, C.c_int32, C.POINTER(SVec)]),
}


def load_library(path: str = LIB_PATH):
    """Load libsfci.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2312_01846_amd.build`")
        L = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SFCI_OK:
        msg = load_library().sfci_last_error().decode(errors="replace")
        raise SfciError(rc, msg)


def space_size(n, na, nb) -> int:
    out = C.c_uint64(0)
    _check(load_library().sfci_space_size(C.byref(Space(n, na, nb)), C.byref(out)))
    return int(out.value)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("libsfci needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _svec(ranks, amps, capacity=None):
    n = int(ranks.numel())
    return SVec(ranks.data_ptr() if n or capacity else None, amps.data_ptr() if n or capacity else None, n,
                int(capacity if capacity is not None else n))


class Problem:
    """A (space, integrals) instance on the current GPU; integrals are host numpy arrays."""

    def __init__(self, n, na, nb, h, g, stream=None):
        torch = _torch()
        self.n, self.na, self.nb = int(n), int(na), int(nb)
        self.h = np.ascontiguousarray(h, dtype=np.float64).reshape(self.n, self.n)
        self.g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.n, self.n, self.n, self.n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n_det = space_size(self.n, self.na, self.nb)
        self.tps = terms_per_source(self.n, self.na, self.nb)
        handle = C.c_void_p(None)
        _check(load_library().sfci_problem_create(C.byref(Space(self.n, self.na, self.nb)),
                                                  self.h.ctypes.data_as(C.c_void_p), self.g.ctypes.data_as(C.c_void_p),
                                                  C.c_void_p(self.stream.cuda_stream), C.byref(handle)))
        self._h = handle

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sfci_problem_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Eq. 12 ----------------------------------------------------------------
    def rank(self, a_bits, b_bits):
        torch = _torch()
        a = torch.as_tensor(np.asarray(a_bits, dtype=np.int64), device="cuda")
        b = torch.as_tensor(np.asarray(b_bits, dtype=np.int64), device="cuda")
        out = torch.empty_like(a)
        _check(load_library().sfci_rank(self._h, a.data_ptr(), b.data_ptr(), a.numel(), out.data_ptr()))
        return out

    def unrank(self, ranks):
        torch = _torch()
        r = torch.as_tensor(ranks, device="cuda").to(torch.int64)
        a = torch.empty_like(r)
        b = torch.empty_like(r)
        _check(load_library().sfci_unrank(self._h, r.data_ptr(), r.numel(), a.data_ptr(), b.data_ptr()))
        return a, b

    # -- sigma = H v, truncated ----------------------------------------------------
    def sigma(self, ranks, amps, M=None, dedup="auto", deterministic=False, capacity=None, screen_eps=0.0,
              tie_band=False, excite_eps=0.0):
        """Returns (ranks int64, amps float64, stats dict) on the GPU."""
        torch = _torch()
        r = torch.as_tensor(ranks, device="cuda").to(torch.int64).contiguous()
        a = torch.as_tensor(amps, device="cuda").to(torch.float64).contiguous()
        Mv = UINT64_MAX if M is None else int(M)
        cap = capacity
        if cap is None:
            cap = min(self.n_det, max(1, r.numel()) * self.tps)
            if M is not None:
                cap = min(cap, int(M) + (TIE_SLACK if tie_band else 0))
        opts = SigmaOpts(Mv, DEDUP[dedup], 1 if deterministic else 0, float(screen_eps), 1 if tie_band else 0, 0,
                         float(excite_eps))
        for _ in range(2):
            o_r = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
            o_a = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
            out = SVec(o_r.data_ptr(), o_a.data_ptr(), 0, cap)
            st = SigmaStats()
            rc = load_library().sfci_sigma(self._h, C.byref(_svec(r, a)), C.byref(opts), C.byref(out), C.byref(st))
            if rc == -4:
                cap = int(out.nnz)
                continue
            _check(rc)
            k = int(out.nnz)
            stats = dict(terms_enumerated=st.terms_enumerated, terms_emitted=st.terms_emitted,
                         candidates=st.candidates, ms=st.ms)
            return o_r[:k], o_a[:k], stats
        raise SfciError(-4, "capacity retry failed")

    def topm(self, ranks, amps, M, normalise=False, tie_band=False):
        torch = _torch()
        r = torch.as_tensor(ranks, device="cuda").to(torch.int64).contiguous()
        a = torch.as_tensor(amps, device="cuda").to(torch.float64).contiguous()
        cap = max(1, r.numel())
        o_r = torch.empty(cap, dtype=torch.int64, device="cuda")
        o_a = torch.empty(cap, dtype=torch.float64, device="cuda")
        out = SVec(o_r.data_ptr(), o_a.data_ptr(), 0, cap)
        Mv = UINT64_MAX if M is None else int(M)
        _check(load_library().sfci_topm(self._h, C.byref(_svec(r, a)), Mv, 1 if normalise else 0,
                                        1 if tie_band else 0, C.byref(out)))
        k = int(out.nnz)
        return o_r[:k], o_a[:k]

    # -- backward of sigma = H(h, g) v -----------------------------------------------
    def pt2(self, ranks, amps, deterministic=False):
        """Second-order Epstein-Nesbet correction of Psi: (E0, E2, number of external determinants)."""
        torch = _torch()
        r = torch.as_tensor(ranks, device="cuda").to(torch.int64).contiguous()
        a = torch.as_tensor(amps, device="cuda").to(torch.float64).contiguous()
        e0, e2, ne = C.c_double(0.0), C.c_double(0.0), C.c_uint64(0)
        _check(load_library().sfci_pt2(self._h, C.byref(_svec(r, a)), 1 if deterministic else 0, C.byref(e0),
                                       C.byref(e2), C.byref(ne)))
        return e0.value, e2.value, int(ne.value)

    def sigma_backward(self, v_rank, v_amp, s_rank, s_amp, want_vbar=True, want_dh=True, want_dg=True):
        """vbar = H sbar on supp(v); dh, dg = gradients of sbar^T H v along symmetric perturbations."""
        torch = _torch()
        vr = torch.as_tensor(v_rank, device="cuda").to(torch.int64).contiguous()
        va = torch.as_tensor(v_amp, device="cuda").to(torch.float64).contiguous()
        sr = torch.as_tensor(s_rank, device="cuda").to(torch.int64).contiguous()
        sa = torch.as_tensor(s_amp, device="cuda").to(torch.float64).contiguous()
        n = self.n
        vbar = torch.empty(max(1, vr.numel()), dtype=torch.float64, device="cuda") if want_vbar else None
        dh = torch.empty((n, n), dtype=torch.float64, device="cuda") if want_dh else None
        dg = torch.empty((n, n, n, n), dtype=torch.float64, device="cuda") if want_dg else None
        _check(load_library().sfci_sigma_backward(self._h, C.byref(_svec(vr, va)), C.byref(_svec(sr, sa)),
                                                  vbar.data_ptr() if vbar is not None else None,
                                                  dh.data_ptr() if dh is not None else None,
                                                  dg.data_ptr() if dg is not None else None))
        return (vbar[:vr.numel()] if vbar is not None else None), dh, dg

    def energy_gradients(self, psi_rank, psi_amp, deterministic=False, want_grad=True):
        """E = <psi|H|psi>/<psi|psi> and its gradients dE/dh, dE/d(pq|rs) at fixed psi
        (Hellmann-Feynman form), all computed by sfci_energy_gradients."""
        torch = _torch()
        r = torch.as_tensor(psi_rank, device="cuda").to(torch.int64).contiguous()
        a = torch.as_tensor(psi_amp, device="cuda").to(torch.float64).contiguous()
        n = self.n
        dh = torch.empty((n, n), dtype=torch.float64, device="cuda") if want_grad else None
        dg = torch.empty((n, n, n, n), dtype=torch.float64, device="cuda") if want_grad else None
        e = C.c_double(0.0)
        _check(load_library().sfci_energy_gradients(self._h, C.byref(_svec(r, a)), 1 if deterministic else 0,
                                                    C.byref(e), dh.data_ptr() if want_grad else None,
                                                    dg.data_ptr() if want_grad else None))
        return e.value, dh, dg

    # -- the SFCI iteration ----------------------------------------------------
    def lanczos(self, ranks0, amps0, M=None, n_L=10, n_iter=30, deterministic=False, dedup="auto", want_T=False,
                want_psi=True, psi_capacity=None, screen_eps=0.0, no_dense=False, roots=None, conv_eps=0.0,
                tie_band=False, excite_eps=0.0):
        """roots: list of (ranks, amps) of previously found eigenvectors projected out
        of the effective Hamiltonian (the iteration then finds the next state).
        conv_eps > 0: halt once a block lowers the energy by less than conv_eps
        (the result's "blocks_run"; energies of blocks not run are NaN)."""
        torch = _torch()
        r = torch.as_tensor(ranks0, device="cuda").to(torch.int64).contiguous()
        a = torch.as_tensor(amps0, device="cuda").to(torch.float64).contiguous()
        nblk = n_iter // n_L
        energies = np.zeros(nblk, dtype=np.float64)
        T = np.zeros(nblk * n_L * n_L) if want_T else None
        S = np.zeros(nblk * n_L * n_L) if want_T else None
        Mv = UINT64_MAX if M is None else int(M)
        opts = LanczosOpts(Mv, n_L, n_iter, 1 if deterministic else 0, DEDUP[dedup], float(screen_eps),
                           1 if no_dense else 0, 0, float(conv_eps), 1 if tie_band else 0, 0, float(excite_eps))
        st = LanczosStats()
        psi = None
        if want_psi:
            extra = TIE_SLACK if tie_band else 0
            cap = psi_capacity or min(self.n_det, n_L * (Mv + extra if M is not None else self.n_det))
            p_r = torch.empty(cap, dtype=torch.int64, device="cuda")
            p_a = torch.empty(cap, dtype=torch.float64, device="cuda")
            psi = SVec(p_r.data_ptr(), p_a.data_ptr(), 0, cap)
        keep = []
        rvecs = None
        if roots:
            rvecs = (SVec * len(roots))()
            for i, (rr, ra) in enumerate(roots):
                tr = torch.as_tensor(rr, device="cuda").to(torch.int64).contiguous()
                ta = torch.as_tensor(ra, device="cuda").to(torch.float64).contiguous()
                keep.append((tr, ta))
                rvecs[i] = _svec(tr, ta)
        rc = load_library().sfci_lanczos_roots(self._h, C.byref(_svec(r, a)), C.byref(opts), rvecs,
                                               len(roots) if roots else 0, energies.ctypes.data_as(C.c_void_p),
                                               C.byref(psi) if psi else None,
                                               T.ctypes.data_as(C.c_void_p) if want_T else None,
                                               S.ctypes.data_as(C.c_void_p) if want_T else None, C.byref(st))
        _check(rc)
        out = dict(energies=energies, blocks_run=int(st.blocks_run),
                   stats=dict(sigma_calls=st.sigma_calls, terms_enumerated=st.terms_enumerated,
                              terms_emitted=st.terms_emitted, sigma_ms=st.sigma_ms, total_ms=st.total_ms))
        if want_psi:
            k = int(psi.nnz)
            out["psi_rank"] = p_r[:k]
            out["psi_amp"] = p_a[:k]
        if want_T:
            out["T"] = T.reshape(nblk, n_L, n_L)
            out["S"] = S.reshape(nblk, n_L, n_L)
        return out


class Batch:
    """Several Problems (one device, one stream) iterated together: one
    target-owned tile launch per sigma step for all instances, later blocks
    replayed from captured hipGraphs, Hellmann-Feynman gradients at the end."""

    def __init__(self, problems):
        _torch()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        handle = C.c_void_p(None)
        _check(load_library().sfci_batch_create(len(self.problems), arr, C.byref(handle)))
        self._h = handle

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sfci_batch_destroy(self._h)
            self._h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lanczos(self, starts, Ms, n_L=10, n_iter=30, deterministic=False, dedup="auto", want_grad=True,
                screen_eps=0.0, autotune=False, tie_band=False, conv_eps=0.0, excite_eps=0.0):
        """starts: list of (ranks, amps); Ms: truncation per instance.  Returns
        dict(energies (n_inst, n_blocks), dh [list of (n,n)], dg [list of (n,n,n,n)], stats)."""
        torch = _torch()
        n_inst = len(self.problems)
        if len(starts) != n_inst or len(Ms) != n_inst:
            raise ValueError("one start vector and one M per instance")
        keep = []
        vecs = (SVec * n_inst)()
        for k, (r0, a0) in enumerate(starts):
            r = torch.as_tensor(r0, device="cuda").to(torch.int64).contiguous()
            a = torch.as_tensor(a0, device="cuda").to(torch.float64).contiguous()
            keep.append((r, a))
            vecs[k] = _svec(r, a)
        Marr = (C.c_uint64 * n_inst)(*[UINT64_MAX if m is None else int(m) for m in Ms])
        nblk = n_iter // n_L
        energies = np.zeros(n_inst * nblk, dtype=np.float64)
        dh_all = dg_all = None
        if want_grad:
            n2 = sum(p.n * p.n for p in self.problems)
            n4 = sum(p.n ** 4 for p in self.problems)
            dh_all = torch.empty(n2, dtype=torch.float64, device="cuda")
            dg_all = torch.empty(n4, dtype=torch.float64, device="cuda")
        opts = LanczosOpts(UINT64_MAX, n_L, n_iter, 1 if deterministic else 0, DEDUP[dedup], float(screen_eps), 0,
                           1 if autotune else 0, float(conv_eps), 1 if tie_band else 0, 0, float(excite_eps))
        st = BatchStats()
        rc = load_library().sfci_batch_lanczos(self._h, vecs, Marr, C.byref(opts),
                                               energies.ctypes.data_as(C.c_void_p),
                                               dh_all.data_ptr() if want_grad else None,
                                               dg_all.data_ptr() if want_grad else None, C.byref(st))
        _check(rc)
        out = dict(energies=energies.reshape(n_inst, nblk),
                   stats=dict(fwd_ms=st.fwd_ms, bwd_ms=st.bwd_ms, sigma_ms=st.sigma_ms,
                              terms_emitted=st.terms_emitted, nnz_in_total=st.nnz_in_total,
                              sigma_calls=st.sigma_calls,
                              psi_nnz_total=st.psi_nnz_total, graph_replayed_blocks=st.graph_replayed_blocks,
                              batched_sigma=st.batched_sigma, tune_trials=st.tune_trials,
                              sigma_in_graph=st.sigma_in_graph, graphs_reused=st.graphs_reused,
                              tune=dict(b1_chunk=st.tune_b1_chunk, bb_chunk=st.tune_bb_chunk,
                                        per_cu=st.tune_per_cu, default_ms=st.tune_default_ms,
                                        best_ms=st.tune_best_ms)))
        if want_grad:
            dh, dg, oh, og = [], [], 0, 0
            for p in self.problems:
                dh.append(dh_all[oh:oh + p.n * p.n].view(p.n, p.n))
                dg.append(dg_all[og:og + p.n ** 4].view(p.n, p.n, p.n, p.n))
                oh += p.n * p.n
                og += p.n ** 4
            out["dh"], out["dg"] = dh, dg
        return out


def terms_per_source(n, na, nb):
    """(source, excitation) pairs per source: 1 + singles + doubles of both spins."""
    sa, sb = na * (n - na), nb * (n - nb)
    pa, qa = na * (na - 1) // 2, (n - na) * (n - na - 1) // 2
    pb, qb = nb * (nb - 1) // 2, (n - nb) * (n - nb - 1) // 2
    return 1 + sa + sb + pa * qa + pb * qb + sa * sb


def declared_symbols(header: str | None = None):
    """Function names declared in include/*.h (or in one header)."""
    import glob
    import re

    files = [header] if header else sorted(glob.glob(os.path.join(INCLUDE, "*.h")))
    text = "".join(open(f).read() for f in files)
    return sorted(set(re.findall(r"\b(sfci_[a-z_]+)\s*\(", text)))


def roof_probe(big_bytes=1 << 30):
    """Device ceilings (sfci_roof_probe) as a dict: copy GB/s and rates in
    operations per ns for random gathers / global FP64 atomics (2 MiB,
    128 MiB, big_bytes arrays) and LDS FP64 atomics / reads."""
    torch = _torch()
    out = Roof()
    _check(load_library().sfci_roof_probe(int(big_bytes), C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                          C.byref(out)))
    return dict(copy_GBps=out.copy_GBps, gather_Gops=list(out.gather_Gops), atomic_Gops=list(out.atomic_Gops),
                lds_atomic_Gops=list(out.lds_atomic_Gops), lds_read_Gops=out.lds_read_Gops,
                big_bytes=int(out.big_bytes))
