// Backward of sigma = H(h, g) v for a cotangent sbar.  With L = sbar^T H v:
//   vbar_i = sum_k H_ki sbar_k                 (gather form: walk the targets of
//                                               source i, read sbar at each)
//   dL/dh, dL/d(pq|rs): every term adds sbar_k v_i times the coefficient of
//   each integral in its Slater-Condon element to a raw gradient; the raw
//   gradients are then projected onto symmetric tensors (the derivative along
//   symmetric perturbations, which is what a finite difference measures).
// Terms with a zero element are visited too: their element vanishes but its
// derivative does not.
#include "sfci_internal.h"

namespace {

struct BackParams {
    SpaceDev sp;
    Ints I;
    const u64* binom;
    const u64* v_rank;
    const double* v_amp;
    const u64* v_nnz;
};

struct SinkBack {
    const double* __restrict__ Sd;  // sbar scattered into the dense array
    double* __restrict__ Rh;        // raw dL/dh, n*n
    double* __restrict__ Rg;        // raw dL/dg, n^4
    int n;
    double acc;  // this lane's share of vbar_i
    __device__ __forceinline__ int G(int p, int q, int r, int s) const { return ((p * n + q) * n + r) * n + s; }
    __device__ __forceinline__ void operator()(bool ok, u64 tgt, double e, double c, const Term& t) {
        if (!ok) return;
        const double sb = Sd[tgt];
        if (sb == 0.0) return;
        acc += e * sb;
        const double w = sb * c;
        switch (t.cls) {
            case 0: {  // diagonal
                for (u32 m = t.A; m; m &= m - 1u) { int p = __builtin_ctz(m); unsafeAtomicAdd(Rh + p * n + p, w); }
                for (u32 m = t.Bs; m; m &= m - 1u) { int p = __builtin_ctz(m); unsafeAtomicAdd(Rh + p * n + p, w); }
                for (int sp = 0; sp < 2; ++sp) {
                    u32 S = sp == 0 ? t.A : t.Bs;
                    for (u32 m = S; m; m &= m - 1u) {
                        int p = __builtin_ctz(m);
                        for (u32 m2 = m & (m - 1u); m2; m2 &= m2 - 1u) {
                            int q = __builtin_ctz(m2);
                            unsafeAtomicAdd(Rg + G(p, p, q, q), w);
                            unsafeAtomicAdd(Rg + G(p, q, q, p), -w);
                        }
                    }
                }
                for (u32 m = t.A; m; m &= m - 1u) {
                    int p = __builtin_ctz(m);
                    for (u32 m2 = t.Bs; m2; m2 &= m2 - 1u) unsafeAtomicAdd(Rg + G(p, p, __builtin_ctz(m2), __builtin_ctz(m2)), w);
                }
                break;
            }
            case 1:
            case 2: {  // single i -> a in the same-spin string
                const u32 Ss = t.cls == 1 ? t.A : t.Bs;
                const u32 So = t.cls == 1 ? t.Bs : t.A;
                const double ws = t.par ? -w : w;
                const int i = t.i, a = t.a;
                unsafeAtomicAdd(Rh + i * n + a, ws);
                for (u32 m = Ss & ~(1u << i); m; m &= m - 1u) {
                    int k = __builtin_ctz(m);
                    unsafeAtomicAdd(Rg + G(i, a, k, k), ws);
                    unsafeAtomicAdd(Rg + G(i, k, k, a), -ws);
                }
                for (u32 m = So; m; m &= m - 1u) {
                    int k = __builtin_ctz(m);
                    unsafeAtomicAdd(Rg + G(i, a, k, k), ws);
                }
                break;
            }
            case 3:
            case 4: {  // same-spin double: (ia|jb) - (ib|ja)
                const double wd = t.par ? -w : w;
                unsafeAtomicAdd(Rg + G(t.i, t.a, t.j, t.b), wd);
                unsafeAtomicAdd(Rg + G(t.i, t.b, t.j, t.a), -wd);
                break;
            }
            default: {  // alpha-beta double: (ia|jb)
                const double wd = t.par ? -w : w;
                unsafeAtomicAdd(Rg + G(t.i, t.a, t.j, t.b), wd);
                break;
            }
        }
    }
};

__device__ __forceinline__ double wave_sum_f64(double x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__global__ __launch_bounds__(SFCI_BLOCK) void k_backward(BackParams p, const double* __restrict__ Sd,
                                                         double* __restrict__ vbar, double* __restrict__ Rh,
                                                         double* __restrict__ Rg) {
    __shared__ BinomLds sB;
    __shared__ WaveLds sW[SFCI_WAVES_PER_BLOCK];
    load_binom(sB, p.binom);
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const u64 nnz = *p.v_nnz;
    AlphaRange all{0, 0};
    for (u64 s = (u64)blockIdx.x * SFCI_WAVES_PER_BLOCK + wave; s < nnz; s += (u64)gridDim.x * SFCI_WAVES_PER_BLOCK) {
        SinkBack sink{Sd, Rh, Rg, p.sp.n, 0.0};
        enumerate_source<false, SinkBack, true>(p.sp, p.I, sB, sW[wave], p.v_rank[s], p.v_amp[s], all, sink);
        double tot = wave_sum_f64(sink.acc);
        if (vbar && lane_id() == 0) vbar[s] = tot;
    }
}

// dh = (R + R^T) / 2;  dg = the mean of R over the 8 index permutations of (pq|rs).
__global__ void k_symmetrise(int n, const double* __restrict__ Rh, const double* __restrict__ Rg,
                             double* __restrict__ dh, double* __restrict__ dg) {
    const int n2 = n * n, n4 = n2 * n2;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n4; t += gridDim.x * blockDim.x) {
        int s = t % n, r = (t / n) % n, q = (t / n2) % n, p = t / (n2 * n);
        auto G = [&](int a, int b, int c, int d) { return Rg[((a * n + b) * n + c) * n + d]; };
        if (dg) {
            double v = G(p, q, r, s) + G(q, p, r, s) + G(p, q, s, r) + G(q, p, s, r) + G(r, s, p, q) + G(s, r, p, q) +
                       G(r, s, q, p) + G(s, r, q, p);
            dg[t] = v / 8.0;
        }
        if (dh && t < n2) {
            int a = t / n, b = t % n;
            dh[t] = 0.5 * (Rh[a * n + b] + Rh[b * n + a]);
        }
    }
}

__global__ void k_scatter_zero(double* __restrict__ D, const u64* __restrict__ r, const u64* __restrict__ nnz) {
    const u64 n = *nnz;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) D[r[i]] = 0.0;
}

unsigned gsz(u64 n) {
    u64 g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

}  // namespace

// sbar must already be scattered into the (otherwise zero) dense array D.
void launch_backward_dense(sfci_problem* P, const SigmaLaunch& v, const double* D, double* vbar, double* dh, double* dg,
                           double* Rh, double* Rg) {
    const int n = P->n;
    const u64 n2 = (u64)n * n, n4 = n2 * n2;
    launch_fill_f64(Rh, n2, 0.0, P->stream);
    launch_fill_f64(Rg, n4, 0.0, P->stream);
    BackParams p{SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb}, Ints{P->d_h, P->d_g, P->n}, P->d_binom, v.v_rank, v.v_amp,
                 v.v_nnz};
    u64 want = (v.cap + SFCI_WAVES_PER_BLOCK - 1) / SFCI_WAVES_PER_BLOCK;
    u64 maxg = (u64)P->num_cu * 8;
    unsigned grid = (unsigned)(want < 1 ? 1 : (want > maxg ? maxg : want));
    hipLaunchKernelGGL(k_backward, dim3(grid), dim3(SFCI_BLOCK), 0, P->stream, p, D, vbar, Rh, Rg);
    if (dh || dg) hipLaunchKernelGGL(k_symmetrise, dim3(gsz(n4)), dim3(256), 0, P->stream, n, Rh, Rg, dh, dg);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_symmetrise(sfci_problem* P, const double* Rh, const double* Rg, double* dh, double* dg) {
    const u64 n2 = (u64)P->n * P->n, n4 = n2 * n2;
    if (!dh && !dg) return;
    hipLaunchKernelGGL(k_symmetrise, dim3(gsz(n4)), dim3(256), 0, P->stream, P->n, Rh, Rg, dh, dg);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_scatter_zero(sfci_problem* P, double* D, const u64* r, const u64* nnz, u64 cap) {
    hipLaunchKernelGGL(k_scatter_zero, dim3(gsz(cap)), dim3(256), 0, P->stream, D, r, nnz);
    SFCI_CHECK_HIP(hipGetLastError());
}
