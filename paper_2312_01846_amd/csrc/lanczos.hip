// Truncated-Lanczos vector algebra (Sec. 2.1, Eqs. 10-11) and the small
// generalized eigenproblem T x = lambda S x, all on the device.
//
// Reductions come in two flavours:
//   fast    -- fixed-grid tree (run-to-run reproducible, not sequential order);
//   ordered -- one wavefront adds the products strictly in ascending-rank
//              order, which reproduces a sequential CPU sum bit for bit.
#include <algorithm>
#include <vector>

#include "sfci_internal.h"

namespace {

constexpr int RB = 256;
constexpr int RGRID = 1024;

__device__ __forceinline__ double block_sum(double x, double* sh) {
    // fixed shape tree over 256 threads
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double y_at(const u64* __restrict__ yr, const double* __restrict__ ya, u64 yn, u64 key) {
    // lower bound in the ascending rank list
    u64 lo = 0, hi = yn;
    while (lo < hi) {
        u64 mid = lo + ((hi - lo) >> 1);
        if (yr[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < yn && yr[lo] == key) ? ya[lo] : 0.0;
}

// y value paired with entry i of x: D[x_rank[i]] (dense) or Y[i] (already
// gathered, GATHERED): the products and their order are the same either way.
template <bool GATHERED>
__device__ __forceinline__ double y_of(const u64* __restrict__ r, const double* __restrict__ D, u64 i) {
    return GATHERED ? D[i] : D[r[i]];
}

// partial[b] = sum over a grid-stride slice of x_amp[i] * D[x_rank[i]]
template <bool GATHERED>
__global__ __launch_bounds__(RB) void k_dot_dense_part(const u64* __restrict__ r, const double* __restrict__ a,
                                                       const u64* __restrict__ nnz, const double* __restrict__ D,
                                                       double* __restrict__ part) {
    __shared__ double sh[RB];
    const u64 n = *nnz;
    double s = 0.0;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)gridDim.x * RB) s += a[i] * y_of<GATHERED>(r, D, i);
    double b = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(RB) void k_dot_sparse_part(const u64* __restrict__ xr, const double* __restrict__ xa,
                                                        const u64* __restrict__ xn, const u64* __restrict__ yr,
                                                        const double* __restrict__ ya, const u64* __restrict__ yn,
                                                        double* __restrict__ part) {
    __shared__ double sh[RB];
    const u64 n = *xn, m = *yn;
    double s = 0.0;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)gridDim.x * RB) {
        double yv = y_at(yr, ya, m, xr[i]);
        if (yv != 0.0) s += xa[i] * yv;
    }
    double b = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(RB) void k_dot_final(const double* __restrict__ part, int np, double* out1, double* out2) {
    __shared__ double sh[RB];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += RB) s += part[i];
    double b = block_sum(s, sh);
    if (threadIdx.x == 0) {
        *out1 = b;
        if (out2) *out2 = b;
    }
}

// Ordered sums: acc = ((0 + t_0) + t_1) + ... strictly in index order, t_i
// the term of entry i (x_i; a_i * D[r_i]; a_i * Y_i; a_i * a_i).  One
// wavefront streams the terms: while lane 0 adds a group of OS_DEPTH chunks of
// 64 terms from LDS, the next group's loads are in flight, so the global
// latency hides behind the add chain (wavefront-scope syncs only: a block
// barrier would wait for those loads).
enum { OS_SUM = 0, OS_DOT = 1, OS_DOT_GATHERED = 2, OS_SUMSQ = 3 };
constexpr int OS_DEPTH = 8;

template <int MODE>
__device__ __forceinline__ void os_load(const u64* __restrict__ r, const double* __restrict__ a,
                                        const double* __restrict__ D, u64 i, u64 n, double& x, double& y) {
    x = 0.0;
    y = 0.0;
    if (i < n) {
        x = a[i];
        if (MODE == OS_DOT) y = D[r[i]];
        if (MODE == OS_DOT_GATHERED) y = D[i];
    }
}

template <int MODE>
__device__ __forceinline__ double os_term(double x, double y) {
    if (MODE == OS_SUM) return x;
    if (MODE == OS_SUMSQ) return x * x;
    return x * y;
}

template <int MODE>
__global__ __launch_bounds__(64) void k_ordered(const u64* __restrict__ r, const double* __restrict__ a,
                                                const u64* __restrict__ nnz, const double* __restrict__ D,
                                                double* out1, double* out2) {
    constexpr int G = 64 * OS_DEPTH;
    __shared__ double stage[G];
    const u64 n = *nnz;
    const int lane = threadIdx.x;
    double x[OS_DEPTH], y[OS_DEPTH];
#pragma unroll
    for (int k = 0; k < OS_DEPTH; ++k) os_load<MODE>(r, a, D, (u64)k * 64 + lane, n, x[k], y[k]);
    double acc = 0.0;
    for (u64 base = 0; base < n; base += G) {
#pragma unroll
        for (int k = 0; k < OS_DEPTH; ++k) stage[k * 64 + lane] = os_term<MODE>(x[k], y[k]);
#pragma unroll
        for (int k = 0; k < OS_DEPTH; ++k) os_load<MODE>(r, a, D, base + G + (u64)k * 64 + lane, n, x[k], y[k]);
        wave_sync();
        if (lane == 0) {
            if (n - base >= (u64)G) {
                for (int q = 0; q < G; q += 64) {
#pragma unroll
                    for (int k = 0; k < 64; ++k) acc += stage[q + k];
                }
            } else {
                const int cnt = (int)(n - base);
                for (int q = 0; q < cnt; ++q) acc += stage[q];
            }
        }
        wave_sync();
    }
    if (lane == 0) {
        *out1 = acc;
        if (out2) *out2 = acc;
    }
}

// Sparse-sparse products x_i * y(rank_i) (0 where y has no entry), formed
// in parallel; the ordered sum below then adds them in index order.  Adding
// +0 for a missing entry changes nothing: the running sum starts at +0 and
// round-to-nearest never turns it into -0.
__global__ __launch_bounds__(RB) void k_sparse_products(const u64* __restrict__ xr, const double* __restrict__ xa,
                                                        const u64* __restrict__ xn, const u64* __restrict__ yr,
                                                        const double* __restrict__ ya, const u64* __restrict__ yn,
                                                        double* __restrict__ prod) {
    const u64 n = *xn, m = *yn;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)gridDim.x * RB) {
        const double yv = y_at(yr, ya, m, xr[i]);
        prod[i] = (yv != 0.0) ? xa[i] * yv : 0.0;
    }
}

// D[r_i] = D[r_i] - coef * a_i  (SUB)   or   D[r_i] = D[r_i] + coef * a_i  (ADD)
template <bool ADD>
__global__ void k_axpy_scatter(double* __restrict__ D, const u64* __restrict__ r, const double* __restrict__ a,
                               const u64* __restrict__ nnz, const double* __restrict__ coef) {
    const u64 n = *nnz;
    const double c = *coef;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        double prod = c * a[i];
        u64 k = r[i];
        if (ADD) D[k] = D[k] + prod;
        else D[k] = D[k] - prod;
    }
}

__global__ void k_scatter_set(double* __restrict__ D, const u64* __restrict__ r, const double* __restrict__ a,
                              const u64* __restrict__ nnz) {
    const u64 n = *nnz;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) D[r[i]] = a[i];
}

__global__ __launch_bounds__(RB) void k_sumsq_part(const double* __restrict__ a, const u64* __restrict__ nnz,
                                                   double* __restrict__ part) {
    __shared__ double sh[RB];
    const u64 n = *nnz;
    double s = 0.0;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)gridDim.x * RB) s += a[i] * a[i];
    double b = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ __launch_bounds__(RB) void k_sum_part(const double* __restrict__ x, const u64* __restrict__ nnz,
                                                 double* __restrict__ part) {
    __shared__ double sh[RB];
    const u64 n = *nnz;
    double s = 0.0;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)gridDim.x * RB) s += x[i];
    double b = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// Eq. 11: a_i = a_i / sqrt(sum of squares); untouched when the sum is 0.
__global__ void k_div_norm(double* __restrict__ a, const u64* __restrict__ nnz, const double* __restrict__ ss) {
    const u64 n = *nnz;
    const double s = *ss;
    if (!(s > 0.0)) return;
    const double nrm = sqrt(s);
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) a[i] = a[i] / nrm;
}

__global__ void k_copy_vec(const u64* __restrict__ r, const double* __restrict__ a, const u64* __restrict__ nnz,
                           u64* __restrict__ r2, double* __restrict__ a2, u64* __restrict__ nnz2) {
    const u64 n = *nnz;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        r2[i] = r[i];
        a2[i] = a[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *nnz2 = n;
}

// ---- generalized eigenproblem, one wavefront (m <= 32) ----
#define GE_MAX 32

// Cyclic Jacobi on the m x m symmetric matrix A (row-major, stride GE_MAX),
// eigenvectors into V's columns, eigenvalues into w.  Same rotation rule,
// sweep order and stopping rule as the CPU reference.  Lane r updates row r
// of every rotation; the rows are independent, so the results are the same
// bits as a sequential sweep.
__device__ void jacobi_dev(int m, double (*A)[GE_MAX], double (*V)[GE_MAX], double* w, int* flag) {
    const int r = threadIdx.x;
    if (r < m)
        for (int q = 0; q < m; ++q) V[r][q] = (r == q) ? 1.0 : 0.0;
    wave_sync();
    for (int sweep = 0; sweep < 64; ++sweep) {
        if (r == 0) {
            double off = 0.0, dg = 0.0;
            for (int p = 0; p < m; ++p) {
                dg += A[p][p] * A[p][p];
                for (int q = p + 1; q < m; ++q) off += A[p][q] * A[p][q];
            }
            *flag = (off <= 1e-30 * dg) ? 1 : 0;
        }
        wave_sync();
        if (*flag) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double app = A[p][p], aqq = A[q][q];
                const double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(t * t + 1.0);
                const double s = t * c;
                const double tau = s / (1.0 + c);
                const bool row = r < m && r != p && r != q;
                double arp = 0.0, arq = 0.0, vrp = 0.0, vrq = 0.0;
                if (row) {
                    arp = A[r][p];
                    arq = A[r][q];
                }
                if (r < m) {
                    vrp = V[r][p];
                    vrq = V[r][q];
                }
                wave_sync();  // every read of this rotation before any write
                if (r == 0) {
                    A[p][p] = app - t * apq;
                    A[q][q] = aqq + t * apq;
                    A[p][q] = 0.0;
                    A[q][p] = 0.0;
                }
                if (row) {
                    const double nrp = arp - s * (arq + tau * arp);
                    const double nrq = arq + s * (arp - tau * arq);
                    A[r][p] = nrp;
                    A[p][r] = nrp;
                    A[r][q] = nrq;
                    A[q][r] = nrq;
                }
                if (r < m) {
                    V[r][p] = vrp - s * (vrq + tau * vrp);
                    V[r][q] = vrq + s * (vrp - tau * vrq);
                }
                wave_sync();
            }
    }
    if (r < m) w[r] = A[r][r];
    wave_sync();
}

// Canonical orthogonalisation: S = U s U^T, keep s_k > 1e-10 max s,
// X = U_k s_k^(-1/2), Jacobi on X^T T X, x = X y for the lowest eigenvalue,
// sign fixed so that the largest |x_i| (lowest i on ties) is positive.
// One wavefront; every sum keeps the reference's order.
__device__ __forceinline__ void geneig_body(int m, const double* __restrict__ T, const double* __restrict__ S,
                                            double* lambda, double* x, double* energy_slot, const int* blk,
                                            int* status) {
    __shared__ double A[GE_MAX][GE_MAX], U[GE_MAX][GE_MAX], X[GE_MAX][GE_MAX], TX[GE_MAX][GE_MAX];
    __shared__ double sv[GE_MAX], lam[GE_MAX], xs[GE_MAX];
    __shared__ int keep[GE_MAX];
    __shared__ int s_r, s_best, s_flag;
    const int i = threadIdx.x;
    if (i < m)
        for (int j = 0; j < m; ++j) A[i][j] = S[i * m + j];
    wave_sync();
    jacobi_dev(m, A, U, sv, &s_flag);
    if (i == 0) {
        double smax = 0.0;
        for (int k = 0; k < m; ++k)
            if (sv[k] > smax) smax = sv[k];
        int r = 0;
        for (int k = 0; k < m; ++k)
            if (sv[k] > 1e-10 * smax) keep[r++] = k;
        s_r = r;
    }
    wave_sync();
    const int r = s_r;
    if (r == 0) {
        if (i == 0) *status = 1;
        return;
    }
    if (i < m)
        for (int c = 0; c < r; ++c) X[i][c] = U[i][keep[c]] / sqrt(sv[keep[c]]);
    wave_sync();
    if (i < m)
        for (int c = 0; c < r; ++c) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += T[i * m + k] * X[k][c];
            TX[i][c] = acc;
        }
    wave_sync();
    if (i < r)
        for (int c = 0; c < r; ++c) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += X[k][i] * TX[k][c];
            A[i][c] = acc;
        }
    wave_sync();
    if (i < r)
        for (int c = i + 1; c < r; ++c) {
            const double v = 0.5 * (A[i][c] + A[c][i]);
            A[i][c] = v;
            A[c][i] = v;
        }
    wave_sync();
    jacobi_dev(r, A, U, lam, &s_flag);  // U now holds the eigenvectors y of X^T T X
    if (i == 0) {
        int best = 0;
        for (int k = 1; k < r; ++k)
            if (lam[k] < lam[best]) best = k;
        s_best = best;
    }
    wave_sync();
    const int best = s_best;
    if (i < m) {
        double acc = 0.0;
        for (int c = 0; c < r; ++c) acc += X[i][c] * U[c][best];
        xs[i] = acc;
    }
    wave_sync();
    if (i == 0) {
        int imax = 0;
        for (int k = 1; k < m; ++k)
            if (fabs(xs[k]) > fabs(xs[imax])) imax = k;
        s_flag = xs[imax] < 0.0 ? 1 : 0;
    }
    wave_sync();
    const bool neg = s_flag != 0;
    if (i < m) x[i] = neg ? -xs[i] : xs[i];
    if (i == 0) {
        *lambda = lam[best];
        if (energy_slot) energy_slot[blk ? *blk : 0] = lam[best];
        *status = 0;
    }
}

__global__ __launch_bounds__(64) void k_geneig(int m, const double* __restrict__ T, const double* __restrict__ S,
                                               double* lambda, double* x, double* energy_slot, const int* blk,
                                               int* status) {
    geneig_body(m, T, S, lambda, x, energy_slot, blk, status);
}

unsigned gsz(u64 cap) {
    u64 g = (cap + 255) / 256;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

}  // namespace

namespace {
template <bool GATHERED>
void dot_dense_impl(sfci_problem* P, const u64* r, const double* a, const u64* nnz, u64 cap, const double* D,
                    double* out1, double* out2, bool ordered) {
    if (ordered) {
        hipLaunchKernelGGL(k_ordered<GATHERED ? OS_DOT_GATHERED : OS_DOT>, dim3(1), dim3(64), 0, P->stream, r, a, nnz,
                           D, out1, out2);
    } else {
        double* part = (double*)P->ws_red.get(RGRID * sizeof(double));
        unsigned g = std::min<unsigned>(RGRID, gsz(cap));
        hipLaunchKernelGGL(k_dot_dense_part<GATHERED>, dim3(g), dim3(RB), 0, P->stream, r, a, nnz, D, part);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, out1, out2);
    }
    SFCI_CHECK_HIP(hipGetLastError());
}
}  // namespace

void launch_dot_dense(sfci_problem* P, const u64* r, const double* a, const u64* nnz, u64 cap, const double* D,
                      double* out1, double* out2, bool ordered) {
    dot_dense_impl<false>(P, r, a, nnz, cap, D, out1, out2, ordered);
}

void launch_dot_gathered(sfci_problem* P, const double* a, const u64* nnz, u64 cap, const double* Y, double* out1,
                         double* out2, bool ordered) {
    dot_dense_impl<true>(P, nullptr, a, nnz, cap, Y, out1, out2, ordered);
}

void launch_sum(sfci_problem* P, const double* x, const u64* nnz, u64 cap, double* out, bool ordered) {
    if (ordered) {
        hipLaunchKernelGGL(k_ordered<OS_SUM>, dim3(1), dim3(64), 0, P->stream, (const u64*)nullptr, x, nnz,
                           (const double*)nullptr, out, (double*)nullptr);
    } else {
        double* part = (double*)P->ws_red.get(RGRID * sizeof(double));
        unsigned g = std::min<unsigned>(RGRID, gsz(cap));
        hipLaunchKernelGGL(k_sum_part, dim3(g), dim3(RB), 0, P->stream, x, nnz, part);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, out, (double*)nullptr);
    }
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_sumsq(sfci_problem* P, const double* a, const u64* nnz, u64 cap, double* out, bool ordered) {
    if (ordered) {
        hipLaunchKernelGGL(k_ordered<OS_SUMSQ>, dim3(1), dim3(64), 0, P->stream, (const u64*)nullptr, a, nnz,
                           (const double*)nullptr, out, (double*)nullptr);
    } else {
        double* part = (double*)P->ws_red.get(RGRID * sizeof(double));
        unsigned g = std::min<unsigned>(RGRID, gsz(cap));
        hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(RB), 0, P->stream, a, nnz, part);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, out, (double*)nullptr);
    }
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_dot_sparse(sfci_problem* P, const u64* xr, const double* xa, const u64* xn, u64 xcap, const u64* yr,
                       const double* ya, const u64* yn, double* out1, double* out2, bool ordered) {
    if (ordered) {
        double* prod = (double*)P->ws_prod.get(std::max<u64>(1, xcap) * sizeof(double));
        hipLaunchKernelGGL(k_sparse_products, dim3(gsz(xcap)), dim3(RB), 0, P->stream, xr, xa, xn, yr, ya, yn, prod);
        hipLaunchKernelGGL(k_ordered<OS_SUM>, dim3(1), dim3(64), 0, P->stream, (const u64*)nullptr,
                           (const double*)prod, xn, (const double*)nullptr, out1, out2);
    } else {
        double* part = (double*)P->ws_red.get(RGRID * sizeof(double));
        unsigned g = std::min<unsigned>(RGRID, gsz(xcap));
        hipLaunchKernelGGL(k_dot_sparse_part, dim3(g), dim3(RB), 0, P->stream, xr, xa, xn, yr, ya, yn, part);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, out1, out2);
    }
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_axpy_scatter(sfci_problem* P, double* D, const u64* r, const double* a, const u64* nnz, u64 cap,
                         const double* coef, double sign) {
    if (sign > 0)
        hipLaunchKernelGGL(k_axpy_scatter<true>, dim3(gsz(cap)), dim3(256), 0, P->stream, D, r, a, nnz, coef);
    else
        hipLaunchKernelGGL(k_axpy_scatter<false>, dim3(gsz(cap)), dim3(256), 0, P->stream, D, r, a, nnz, coef);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_scatter_set(sfci_problem* P, double* D, const u64* r, const double* a, const u64* nnz, u64 cap) {
    hipLaunchKernelGGL(k_scatter_set, dim3(gsz(cap)), dim3(256), 0, P->stream, D, r, a, nnz);
    SFCI_CHECK_HIP(hipGetLastError());
}

u64 normalise_ws_doubles() { return RGRID + 8; }

void launch_normalise(sfci_problem* P, double* a, const u64* nnz, u64 cap, bool ordered, double* part_ws) {
    double* part = part_ws ? part_ws : (double*)P->ws_red.get((RGRID + 8) * sizeof(double));
    double* ss = part + RGRID;
    if (ordered) {
        hipLaunchKernelGGL(k_ordered<OS_SUMSQ>, dim3(1), dim3(64), 0, P->stream, (const u64*)nullptr, a, nnz,
                           (const double*)nullptr, ss, (double*)nullptr);
    } else {
        unsigned g = std::min<unsigned>(RGRID, gsz(cap));
        hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(RB), 0, P->stream, a, nnz, part);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, ss, (double*)nullptr);
    }
    hipLaunchKernelGGL(k_div_norm, dim3(gsz(cap)), dim3(256), 0, P->stream, a, nnz, ss);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_copy_vec(sfci_problem* P, const u64* r, const double* a, const u64* nnz, u64 cap, u64* r2, double* a2,
                     u64* nnz2) {
    hipLaunchKernelGGL(k_copy_vec, dim3(gsz(cap)), dim3(256), 0, P->stream, r, a, nnz, r2, a2, nnz2);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_geneig_full(sfci_problem* P, int m, const double* T, const double* S, double* lambda, double* x,
                        double* energy_slot, int* status, const int* blk) {
    hipLaunchKernelGGL(k_geneig, dim3(1), dim3(64), 0, P->stream, m, T, S, lambda, x, energy_slot, blk, status);
    SFCI_CHECK_HIP(hipGetLastError());
}

namespace {
__global__ void k_inc_int(int* p) {
    if (threadIdx.x == 0) *p += 1;
}
__global__ void k_screen(double* __restrict__ D, u64 n, double eps) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        const double v = D[i];
        if (v != 0.0 && fabs(v) < eps) D[i] = 0.0;
    }
}
__global__ void k_add_u64(u64* dst, const u64* src) {
    if (threadIdx.x == 0) *dst += *src;
}
__global__ void k_scale_copy(const double* __restrict__ a, const u64* __restrict__ nnz, const double* __restrict__ ss,
                             double* __restrict__ out) {
    const u64 n = *nnz;
    const double s = *ss;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        out[i] = (s > 0.0) ? a[i] / s : 0.0;
}
}  // namespace

void launch_inc_int(sfci_problem* P, int* p) {
    hipLaunchKernelGGL(k_inc_int, dim3(1), dim3(64), 0, P->stream, p);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_screen(sfci_problem* P, double* D, u64 n, double eps) {
    hipLaunchKernelGGL(k_screen, dim3(gsz(n)), dim3(256), 0, P->stream, D, n, eps);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_add_u64(sfci_problem* P, u64* dst, const u64* src) {
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, P->stream, dst, src);
    SFCI_CHECK_HIP(hipGetLastError());
}

// out = a / sum(a^2) (the cotangent of the Rayleigh quotient's numerator).
void launch_div_by_sumsq(sfci_problem* P, const double* a, const u64* nnz, u64 cap, double* out) {
    double* part = (double*)P->ws_red.get((RGRID + 8) * sizeof(double));
    double* ss = part + RGRID + 1;
    unsigned g = std::min<unsigned>(RGRID, gsz(cap));
    hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(RB), 0, P->stream, a, nnz, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(RB), 0, P->stream, part, (int)g, ss, (double*)nullptr);
    hipLaunchKernelGGL(k_scale_copy, dim3(gsz(cap)), dim3(256), 0, P->stream, a, nnz, ss, out);
    SFCI_CHECK_HIP(hipGetLastError());
}

// ---- batched steps: every instance of a batch in one launch (blockIdx.y or
// blockIdx.z picks the instance).  The same products and sums as the
// per-instance fast reductions above, over a fixed grid of BG partials.
namespace {

constexpr unsigned BG = 256;  // partial sums per dot

__device__ __forceinline__ void bvec(const BInst& b, int l, const u64*& r, const double*& a, u64& n) {
    r = b.Wr + (u64)l * b.cap;
    a = b.Wa + (u64)l * b.cap;
    n = b.sc[l];
}

__device__ __forceinline__ int bout_index(int kind, int j) { return kind == BOUT_W0 ? 0 : j + 1; }

// grid (BG, 2 (j + 1), n): y = 2 l, <w_l|D>; y = 2 l + 1, <w_l|w_j>
__global__ __launch_bounds__(RB) void k_bdot_part(const BInst* __restrict__ B, int j) {
    const BInst& b = B[blockIdx.z];
    __shared__ double sh[RB];
    const int l = (int)(blockIdx.y >> 1);
    const u64* xr;
    const double* xa;
    u64 nx;
    bvec(b, l, xr, xa, nx);
    double s = 0.0;
    if ((blockIdx.y & 1u) == 0) {
        for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < nx; i += (u64)BG * RB) s += xa[i] * b.D[xr[i]];
    } else {
        const u64* yr;
        const double* ya;
        u64 ny;
        bvec(b, j, yr, ya, ny);
        for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < nx; i += (u64)BG * RB) {
            const double yv = y_at(yr, ya, ny, xr[i]);
            if (yv != 0.0) s += xa[i] * yv;
        }
    }
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) b.red[(u64)blockIdx.y * BG + blockIdx.x] = t;
}

// grid (2 (j + 1), n): the BG partials of each dot into T or S (both triangles)
__global__ __launch_bounds__(RB) void k_bdot_final(const BInst* __restrict__ B, int j) {
    const BInst& b = B[blockIdx.y];
    __shared__ double sh[RB];
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < BG; i += RB) s += b.red[(u64)blockIdx.x * BG + i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) {
        const int l = (int)(blockIdx.x >> 1);
        double* M = (blockIdx.x & 1u) ? b.S : b.T;
        M[l * b.nL + j] = t;
        M[j * b.nL + l] = t;
    }
}

// kind 0: D[r_i] = D[r_i] - T[l][j] a_i;  kind 1: D[r_i] = D[r_i] + x[l] a_i
__global__ void k_baxpy(const BInst* __restrict__ B, int l, int j, int kind) {
    const BInst& b = B[blockIdx.y];
    const u64* r;
    const double* a;
    u64 n;
    bvec(b, l, r, a, n);
    const double c = kind ? b.x[l] : b.T[l * b.nL + j];
    double* D = b.D;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        const double prod = c * a[i];
        const u64 k = r[i];
        if (kind) D[k] = D[k] + prod;
        else D[k] = D[k] - prod;
    }
}

// Eq. 11 on w_{j+1} (or w_0): partial sums of squares, their sum, the division
__global__ __launch_bounds__(RB) void k_bsumsq_part(const BInst* __restrict__ B, int kind, int j) {
    const BInst& b = B[blockIdx.y];
    __shared__ double sh[RB];
    const u64* r;
    const double* a;
    u64 n;
    bvec(b, bout_index(kind, j), r, a, n);
    double s = 0.0;
    for (u64 i = (u64)blockIdx.x * RB + threadIdx.x; i < n; i += (u64)BG * RB) s += a[i] * a[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) b.red[(u64)2 * b.nL * BG + blockIdx.x] = t;
}

__global__ __launch_bounds__(RB) void k_bsumsq_final(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    __shared__ double sh[RB];
    const double* part = b.red + (u64)2 * b.nL * BG;
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < BG; i += RB) s += part[i];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) b.red[(u64)2 * b.nL * BG + BG] = t;
}

__global__ void k_bdiv(const BInst* __restrict__ B, int kind, int j) {
    const BInst& b = B[blockIdx.y];
    const double ss = b.red[(u64)2 * b.nL * BG + BG];
    if (!(ss > 0.0)) return;
    const double nrm = sqrt(ss);
    const int l = bout_index(kind, j);
    double* a = b.Wa + (u64)l * b.cap;
    const u64 n = b.sc[l];
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) a[i] = a[i] / nrm;
}

__global__ void k_bfill_zero(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < b.Ndet; i += (u64)gridDim.x * blockDim.x) b.D[i] = 0.0;
}

__global__ __launch_bounds__(64) void k_bgeneig(const BInst* __restrict__ B, int m) {
    const BInst& b = B[blockIdx.y];
    geneig_body(m, b.T, b.S, b.lam, b.x, b.energies, b.blk, b.status);
}

__global__ void k_binc_blk(const BInst* __restrict__ B) {
    if (threadIdx.x == 0) *B[blockIdx.y].blk += 1;
}

unsigned bgrid(u64 n, u64 per, u64 cap) {
    u64 g = (n + per - 1) / per;
    return (unsigned)std::max<u64>(1, std::min<u64>(g, cap));
}

}  // namespace

u64 bstep_red_doubles(int nL) { return (u64)2 * nL * BG + BG + 8; }

void bstep_dots(hipStream_t st, const BInst* d, int n, int j, int nL) {
    (void)nL;
    hipLaunchKernelGGL(k_bdot_part, dim3(BG, 2 * (j + 1), n), dim3(RB), 0, st, d, j);
    hipLaunchKernelGGL(k_bdot_final, dim3(2 * (j + 1), n), dim3(RB), 0, st, d, j);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bstep_axpy(hipStream_t st, const BInst* d, int n, int l, int j, int kind, u64 max_cap) {
    hipLaunchKernelGGL(k_baxpy, dim3(bgrid(max_cap, 256, 16384), n), dim3(256), 0, st, d, l, j, kind);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bstep_normalise(hipStream_t st, const BInst* d, int n, int out_kind, int j, u64 max_cap) {
    hipLaunchKernelGGL(k_bsumsq_part, dim3(BG, n), dim3(RB), 0, st, d, out_kind, j);
    hipLaunchKernelGGL(k_bsumsq_final, dim3(1, n), dim3(RB), 0, st, d);
    hipLaunchKernelGGL(k_bdiv, dim3(bgrid(max_cap, 256, 16384), n), dim3(256), 0, st, d, out_kind, j);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bstep_fill_zero(hipStream_t st, const BInst* d, int n, u64 max_ndet) {
    hipLaunchKernelGGL(k_bfill_zero, dim3(bgrid(max_ndet, 256 * 16, 65535), n), dim3(256), 0, st, d);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bstep_geneig(hipStream_t st, const BInst* d, int n, int nL) {
    hipLaunchKernelGGL(k_bgeneig, dim3(1, n), dim3(64), 0, st, d, nL);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bstep_inc_blk(hipStream_t st, const BInst* d, int n) {
    hipLaunchKernelGGL(k_binc_blk, dim3(1, n), dim3(64), 0, st, d);
    SFCI_CHECK_HIP(hipGetLastError());
}
