// sigma = H v kernels: dense FP64-atomic accumulation, exact per-source
// counting and deterministic tuple emission (for the sort path), plus the
// Eq. 12 rank/unrank kernels.
#include "sfci_internal.h"

namespace {

struct SigmaParams {
    SpaceDev sp;
    Ints I;
    const u64* binom;
    const u64* v_rank;
    const double* v_amp;
    const u64* v_nnz;
    double eps_x;  // excitation screen of the doubles (0 = off)
};

// A term that survives the excitation screen (doubles with |e c| < eps_x go).
__device__ __forceinline__ bool kept_term(bool ok, double e, double c, const Term& tm, double eps_x) {
    return ok && !(tm.cls >= 3 && xscreened(e * c, eps_x));
}

// Dense dedup: every term is added into D[target] with a hardware FP64 atomic.
struct SinkDense {
    double* D;
    u64 cnt;
    double eps_x;
    __device__ __forceinline__ void operator()(bool ok, u64 tgt, double e, double c, const Term& tm) {
        if (kept_term(ok, e, c, tm, eps_x)) {
            unsafeAtomicAdd(D + tgt, e * c);
            ++cnt;
        }
    }
};

struct SinkCount {
    u64 cnt;
    double eps_x;
    __device__ __forceinline__ void operator()(bool ok, u64, double e, double c, const Term& tm) {
        cnt += kept_term(ok, e, c, tm, eps_x) ? 1 : 0;
    }
};

// Tuple emission at deterministic positions: within one source, lanes write
// in (class, term) order via a wave prefix of the ballot.
struct SinkEmit {
    u64* keys;
    double* vals;
    u64 pos;       // next slot of this source (wave-uniform)
    u64 key_base;  // subtracted from the rank to form the sort key
    double eps_x;
    __device__ __forceinline__ void operator()(bool ok_, u64 tgt, double e, double c, const Term& tm) {
        const bool ok = kept_term(ok_, e, c, tm, eps_x);
        u64 m = __ballot(ok);
        if (ok) {
            u64 below = m & ((1ull << lane_id()) - 1ull);
            u64 at = pos + (u64)__popcll(below);
            keys[at] = tgt - key_base;
            vals[at] = e * c;
        }
        pos += (u64)__popcll(m);
    }
};

__device__ __forceinline__ u64 wave_sum_u64(u64 x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__global__ __launch_bounds__(SFCI_BLOCK) void k_sigma_dense(SigmaParams p, double* __restrict__ D,
                                                            unsigned long long* emitted) {
    __shared__ BinomLds sB;
    __shared__ WaveLds sW[SFCI_WAVES_PER_BLOCK];
    load_binom(sB, p.binom);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const u64 nnz = *p.v_nnz;
    SinkDense sink{D, 0, p.eps_x};
    AlphaRange all{0, 0};
    for (u64 s = (u64)blockIdx.x * SFCI_WAVES_PER_BLOCK + wave; s < nnz; s += (u64)gridDim.x * SFCI_WAVES_PER_BLOCK) {
        enumerate_source<false>(p.sp, p.I, sB, sW[wave], p.v_rank[s], p.v_amp[s], all, sink);
    }
    u64 tot = wave_sum_u64(sink.cnt);
    if (lane_id() == 0 && emitted && tot) atomicAdd(emitted, (unsigned long long)tot);
}

__global__ __launch_bounds__(SFCI_BLOCK) void k_sigma_count(SigmaParams p, AlphaRange rng, u64* __restrict__ counts) {
    __shared__ BinomLds sB;
    __shared__ WaveLds sW[SFCI_WAVES_PER_BLOCK];
    load_binom(sB, p.binom);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const u64 nnz = *p.v_nnz;
    for (u64 s = (u64)blockIdx.x * SFCI_WAVES_PER_BLOCK + wave; s < nnz; s += (u64)gridDim.x * SFCI_WAVES_PER_BLOCK) {
        SinkCount sink{0, p.eps_x};
        enumerate_source<true>(p.sp, p.I, sB, sW[wave], p.v_rank[s], p.v_amp[s], rng, sink);
        u64 tot = wave_sum_u64(sink.cnt);
        if (lane_id() == 0) counts[s] = tot;
    }
}

__global__ __launch_bounds__(SFCI_BLOCK) void k_sigma_emit(SigmaParams p, AlphaRange rng, const u64* __restrict__ offs,
                                                           u64 key_base, u64* __restrict__ keys,
                                                           double* __restrict__ vals) {
    __shared__ BinomLds sB;
    __shared__ WaveLds sW[SFCI_WAVES_PER_BLOCK];
    load_binom(sB, p.binom);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const u64 nnz = *p.v_nnz;
    for (u64 s = (u64)blockIdx.x * SFCI_WAVES_PER_BLOCK + wave; s < nnz; s += (u64)gridDim.x * SFCI_WAVES_PER_BLOCK) {
        SinkEmit sink{keys, vals, offs[s], key_base, p.eps_x};
        enumerate_source<true>(p.sp, p.I, sB, sW[wave], p.v_rank[s], p.v_amp[s], rng, sink);
    }
}

// ---- Eq. 12 rank / unrank of explicit strings ----
__global__ void k_rank(SpaceDev sp, const u64* __restrict__ binom, const u64* __restrict__ a,
                       const u64* __restrict__ b, u64 cnt, u64* __restrict__ out, int* bad) {
    __shared__ BinomLds sB;
    load_binom(sB, binom);
    __syncthreads();
    const u64 mask = (sp.n == 64) ? ~0ull : ((1ull << sp.n) - 1ull);
    for (u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += (u64)gridDim.x * blockDim.x) {
        u64 x = a[t], y = b[t];
        if ((x & ~mask) || (y & ~mask) || __popcll(x) != sp.na || __popcll(y) != sp.nb) {
            *bad = 1;
            out[t] = ~0ull;
            continue;
        }
        out[t] = str_rank((u32)x, sB) * sp.Nb + str_rank((u32)y, sB);
    }
}

__global__ void k_unrank(SpaceDev sp, const u64* __restrict__ binom, const u64* __restrict__ r, u64 cnt,
                         u64* __restrict__ a, u64* __restrict__ b, int* bad) {
    __shared__ BinomLds sB;
    load_binom(sB, binom);
    __syncthreads();
    const u64 ndet = sp.Na * sp.Nb;
    for (u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += (u64)gridDim.x * blockDim.x) {
        u64 R = r[t];
        if (R >= ndet) {
            *bad = 1;
            a[t] = 0; b[t] = 0;
            continue;
        }
        u64 ra = R / sp.Nb;
        a[t] = str_unrank(ra, sp.na, sp.n, sB);
        b[t] = str_unrank(R - ra * sp.Nb, sp.nb, sp.n, sB);
    }
}

SigmaParams make_params(sfci_problem* P, const SigmaLaunch& v) {
    SigmaParams p;
    p.sp = SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb};
    p.I = Ints{P->d_h, P->d_g, P->n};
    p.binom = P->d_binom;
    p.v_rank = v.v_rank;
    p.v_amp = v.v_amp;
    p.v_nnz = v.v_nnz;
    p.eps_x = P->excite_eps;
    return p;
}

unsigned grid_for_sources(sfci_problem* P, u64 cap) {
    u64 want = (cap + SFCI_WAVES_PER_BLOCK - 1) / SFCI_WAVES_PER_BLOCK;
    u64 maxg = (u64)P->num_cu * 8;
    if (want > maxg) want = maxg;
    if (want < 1) want = 1;
    return (unsigned)want;
}

}  // namespace

void launch_sigma_dense(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted) {
    SigmaParams p = make_params(P, v);
    hipLaunchKernelGGL(k_sigma_dense, dim3(grid_for_sources(P, v.cap)), dim3(SFCI_BLOCK), 0, P->stream, p, D, emitted);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_sigma_count(sfci_problem* P, const SigmaLaunch& v, u64 alo, u64 ahi, u64* counts) {
    SigmaParams p = make_params(P, v);
    hipLaunchKernelGGL(k_sigma_count, dim3(grid_for_sources(P, v.cap)), dim3(SFCI_BLOCK), 0, P->stream, p,
                       AlphaRange{alo, ahi}, counts);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_sigma_emit(sfci_problem* P, const SigmaLaunch& v, u64 alo, u64 ahi, const u64* offs, u64 key_base,
                       u64* keys, double* vals) {
    SigmaParams p = make_params(P, v);
    hipLaunchKernelGGL(k_sigma_emit, dim3(grid_for_sources(P, v.cap)), dim3(SFCI_BLOCK), 0, P->stream, p,
                       AlphaRange{alo, ahi}, offs, key_base, keys, vals);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_rank(sfci_problem* P, const u64* a, const u64* b, u64 cnt, u64* rank, int* bad) {
    if (cnt == 0) return;
    u64 g = (cnt + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_rank, dim3((unsigned)g), dim3(256), 0, P->stream, SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb},
                       P->d_binom, a, b, cnt, rank, bad);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_unrank(sfci_problem* P, const u64* rank, u64 cnt, u64* a, u64* b, int* bad) {
    if (cnt == 0) return;
    u64 g = (cnt + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_unrank, dim3((unsigned)g), dim3(256), 0, P->stream,
                       SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb}, P->d_binom, rank, cnt, a, b, bad);
    SFCI_CHECK_HIP(hipGetLastError());
}
