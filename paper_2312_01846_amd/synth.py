"""Seeded synthetic inputs for the sparse-FCI sigma = H v path.

This module only draws numbers: it holds none of the method's arithmetic
(no ranking, no excitations, no matrix elements).  Both the CPU oracle and
the HIP path take their inputs from here, so they see identical bits.

The molecular integrals behind the paper's benchmarks (Sec. 3, MolPro RHF
integrals for C2, N2, Ne, CO, F2) are not available; these generators stand
in for them with the same shapes (orbital and electron counts of Table 3 and
Table 5, without point-group symmetry).

Recipes (draw order within one seed is part of the contract):

* ``molecule_like(n, rank, seed)``
    1. diag(h) = sort(U[-2, -0.5], n) ascending,
    2. off-diagonal h_pq ~ N(0, 0.05) for p < q in row-major order, mirrored,
    3. L[k, p, q] ~ N(0, 0.1) for k-major, p <= q row-major, mirrored,
    4. (pq|rs) = sum_k L[k,p,q] L[k,r,s], summed over k in ascending order.
  Step 4 gives a tensor that is exactly (bitwise) 8-fold symmetric and
  positive semidefinite as a (pq),(rs) matrix.
* ``hubbard_ring(n_sites, t, U)``: h_{p,p+-1 mod n} = -t, (pp|pp) = U.
* ``bond_stretch_batch(...)``: h(lam) = h0 + lam h1 and L(lam) = L0 + lam L1.

Start determinants are returned as occupation bit strings (bit p set means
spatial orbital p is occupied); each side ranks them with its own code.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "molecule_like",
    "hubbard_ring",
    "bond_stretch_batch",
    "eri_from_factors",
    "aufbau_bits",
    "neel_bits",
    "random_sparse_vector",
    "CONFIGS",
]


def eri_from_factors(L: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_k L[k,p,q] L[k,r,s], accumulated over k in ascending order.

    The explicit k loop fixes the floating-point summation order, which is
    what makes the result bitwise symmetric under (pq)<->(rs), p<->q, r<->s.
    """
    nk, n, _ = L.shape
    g = np.zeros((n, n, n, n), dtype=np.float64)
    for k in range(nk):
        g += np.multiply.outer(L[k], L[k])
    return g


def _sym_factor_draw(rng: np.random.Generator, rank: int, n: int, std: float) -> np.ndarray:
    L = np.zeros((rank, n, n), dtype=np.float64)
    iu = np.triu_indices(n)
    for k in range(rank):
        vals = rng.normal(0.0, std, size=iu[0].size)
        L[k][iu] = vals
        L[k].T[iu] = vals
    return L


def _h_draw(rng: np.random.Generator, n: int) -> np.ndarray:
    h = np.zeros((n, n), dtype=np.float64)
    h[np.diag_indices(n)] = np.sort(rng.uniform(-2.0, -0.5, size=n))
    iu = np.triu_indices(n, k=1)
    vals = rng.normal(0.0, 0.05, size=iu[0].size)
    h[iu] = vals
    h.T[iu] = vals
    return h


def molecule_like(n: int, rank: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Molecule-like integrals (h, g) with g = (pq|rs) in chemist order, row-major n^4."""
    rng = np.random.default_rng(seed)
    h = _h_draw(rng, n)
    L = _sym_factor_draw(rng, rank, n, 0.1)
    return h, eri_from_factors(L)


def hubbard_ring(n_sites: int, t: float = 1.0, U: float = 4.0) -> tuple[np.ndarray, np.ndarray]:
    """1D periodic Hubbard ring as second-quantized integrals."""
    n = n_sites
    h = np.zeros((n, n), dtype=np.float64)
    for p in range(n):
        q = (p + 1) % n
        h[p, q] = -t
        h[q, p] = -t
    g = np.zeros((n, n, n, n), dtype=np.float64)
    for p in range(n):
        g[p, p, p, p] = U
    return h, g


def bond_stretch_batch(n: int, n_inst: int, rank: int, seeds=(40, 41, 42, 43), lam=None):
    """Integrals along a synthetic bond-stretch parameter lam in [0, 1].

    h0 follows the molecule-like h recipe; h1 draws every entry (diagonal
    included) like h0's off-diagonal, symmetric; L0, L1 are drawn like the
    molecule-like factors.  Returns a list of (lam, h, g).
    """
    h0 = _h_draw(np.random.default_rng(seeds[0]), n)
    rng1 = np.random.default_rng(seeds[1])
    h1 = np.zeros((n, n), dtype=np.float64)
    iu = np.triu_indices(n)
    vals = rng1.normal(0.0, 0.05, size=iu[0].size)
    h1[iu] = vals
    h1.T[iu] = vals
    L0 = _sym_factor_draw(np.random.default_rng(seeds[2]), rank, n, 0.1)
    L1 = _sym_factor_draw(np.random.default_rng(seeds[3]), rank, n, 0.1)
    if lam is None:
        lam = [j / (n_inst - 1) for j in range(n_inst)] if n_inst > 1 else [0.0]
    out = []
    for lj in lam:
        h = h0 + lj * h1
        L = L0 + lj * L1
        out.append((float(lj), h, eri_from_factors(L)))
    return out


def batch_truncations(n_inst: int, seed: int = 44, lo: float = 4.0, hi: float = 6.0) -> list[int]:
    """M_j = round(10^(lo + (hi-lo) u_j)), u_j ~ U[0, 1) from one seed."""
    u = np.random.default_rng(seed).uniform(0.0, 1.0, size=n_inst)
    return [int(round(10.0 ** (lo + (hi - lo) * x))) for x in u]


def aufbau_bits(n_elec: int) -> int:
    """Lowest n_elec orbitals occupied."""
    return (1 << n_elec) - 1


def perturbed_start(n: int, na: int, nb: int, seed: int = 7, weight: float = 0.1) -> list[tuple[int, int, float]]:
    """Start vector as (alpha bits, beta bits, amplitude) triples: the aufbau
    determinant with amplitude 1 plus every single excitation of it, alpha
    singles then beta singles (occupied i ascending, virtual a ascending),
    with amplitudes weight * N(0, 1) drawn in that order from one seed.

    With n_alpha = n_beta the Hamiltonian commutes with exchanging the alpha
    and beta strings.  A start vector that is symmetric (or antisymmetric)
    under that exchange keeps every iterate so, and the two partners of an
    exchanged pair then carry amplitudes of equal magnitude: the top-M cut
    through such a pair is decided by the last bit of rounding.  Independent
    random amplitudes on both spins give both the exchange-symmetric and the
    antisymmetric part of the vector the same support, so the partners differ.
    """
    rng = np.random.default_rng(seed)
    a0, b0 = aufbau_bits(na), aufbau_bits(nb)
    out = [(a0, b0, 1.0)]
    for i in range(na):
        for a in range(na, n):
            out.append((a0 ^ (1 << i) ^ (1 << a), b0, float(weight * rng.normal())))
    for i in range(nb):
        for a in range(nb, n):
            out.append((a0, b0 ^ (1 << i) ^ (1 << a), float(weight * rng.normal())))
    return out


def neel_bits(n_sites: int) -> tuple[int, int]:
    """Neel determinant: alpha on even sites, beta on odd sites."""
    a = sum(1 << p for p in range(0, n_sites, 2))
    b = sum(1 << p for p in range(1, n_sites, 2))
    return a, b


def random_sparse_vector(n_det: int, nnz: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """nnz distinct ranks in [0, n_det), ascending, with N(0,1) amplitudes."""
    rng = np.random.default_rng(seed)
    nnz = min(nnz, n_det)
    if n_det <= 4 * nnz or n_det < (1 << 24):
        ranks = np.sort(rng.choice(n_det, size=nnz, replace=False)).astype(np.uint64)
    else:
        got = np.unique(rng.integers(0, n_det, size=int(nnz * 1.1) + 16, dtype=np.uint64))
        while got.size < nnz:
            got = np.unique(np.concatenate([got, rng.integers(0, n_det, size=nnz, dtype=np.uint64)]))
        ranks = np.sort(rng.choice(got, size=nnz, replace=False)).astype(np.uint64)
    amps = rng.normal(0.0, 1.0, size=nnz)
    return ranks, amps


# The five workloads (orbitals, alpha/beta electrons, truncation, sigma count).
CONFIGS = {
    "c0_small_molecule": dict(n=8, na=3, nb=3, rank=16, seed=0, M=None, n_iter=30, n_L=10),
    "c1_hubbard12": dict(n=12, na=6, nb=6, t=1.0, U=4.0, M=100_000, n_iter=60, n_L=10),
    "c2_26o10e": dict(n=26, na=5, nb=5, rank=52, seed=2, M=(100_000, 1_000_000, 10_000_000),
                      n_iter=30, n_L=10),
    "c3_28o12e": dict(n=28, na=6, nb=6, rank=56, seed=3, M=10_000_000, n_iter=40, n_L=10),
    "c4_batch_20o8e": dict(n=20, na=4, nb=4, rank=40, n_inst=32, n_iter=30, n_L=10),
}
