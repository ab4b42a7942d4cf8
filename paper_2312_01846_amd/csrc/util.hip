// Small device utilities: fills and a three-phase exclusive scan of u64 counts.
#include <algorithm>

#include "sfci_internal.h"

namespace {

__global__ void k_fill_f64(double* __restrict__ p, u64 n, double v) {
    for (u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (u64)gridDim.x * blockDim.x) p[t] = v;
}

__global__ void k_fill_u64(u64* __restrict__ p, u64 n, u64 v) {
    for (u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (u64)gridDim.x * blockDim.x) p[t] = v;
}

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr u64 SCAN_TILE = (u64)SCAN_BLOCK * SCAN_ITEMS;
constexpr int TOP_BLOCK = 1024;

__device__ __forceinline__ u64 shfl_up_u64(u64 x, int off) { return (u64)__shfl_up((long long)x, off); }
__device__ __forceinline__ u64 shfl_xor_u64(u64 x, int off) { return (u64)__shfl_xor((long long)x, off); }

// Exclusive scan of one value per thread over a block of NT threads (wavefront
// scans, then the wavefront totals); *total receives the block's sum.  sh
// holds NT / 64 entries.
template <int NT>
__device__ __forceinline__ u64 block_excl_scan(u64 x, u64* sh, u64* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u64 inc = x;
    for (int off = 1; off < 64; off <<= 1) {
        const u64 y = shfl_up_u64(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    u64 pre = 0, tot = 0;
    for (int k = 0; k < NT / 64; ++k) {
        const u64 v = sh[k];
        if (k < w) pre += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

__device__ __forceinline__ void scan_reduce_body(const u64* __restrict__ in, u64 n, u64* __restrict__ bsum, unsigned bx) {
    __shared__ u64 sh[SCAN_BLOCK / 64];
    const u64 base = (u64)bx * SCAN_TILE;
    u64 s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const u64 i = base + (u64)k * SCAN_BLOCK + threadIdx.x;
        if (i < n) s += in[i];
    }
    for (int off = 32; off >= 1; off >>= 1) s += shfl_xor_u64(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int k = 0; k < SCAN_BLOCK / 64; ++k) t += sh[k];
        bsum[bx] = t;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const u64* __restrict__ in, u64 n, u64* __restrict__ bsum) {
    scan_reduce_body(in, n, bsum, blockIdx.x);
}

// Single block: exclusive scan of nb block sums in place, total to *total.
__device__ __forceinline__ void scan_top_body(u64* __restrict__ bsum, u64 nb, u64* __restrict__ total) {
    __shared__ u64 sh[TOP_BLOCK / 64];
    u64 carry = 0;
    for (u64 base = 0; base < nb; base += TOP_BLOCK) {
        const u64 i = base + threadIdx.x;
        const u64 x = (i < nb) ? bsum[i] : 0;
        u64 tot;
        const u64 ex = block_excl_scan<TOP_BLOCK>(x, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(TOP_BLOCK) void k_scan_top(u64* __restrict__ bsum, u64 nb, u64* __restrict__ total) {
    scan_top_body(bsum, nb, total);
}

// Each thread scans SCAN_ITEMS consecutive counts.  in and out may be the
// same array (every thread reads its own counts before writing them).
__device__ __forceinline__ void scan_down_body(const u64* in, u64 n, const u64* __restrict__ boff, u64* out,
                                               unsigned bx) {
    __shared__ u64 sh[SCAN_BLOCK / 64];
    const u64 first = (u64)bx * SCAN_TILE + (u64)threadIdx.x * SCAN_ITEMS;
    const bool full = (u64)(bx + 1) * SCAN_TILE <= n;
    u64 v[SCAN_ITEMS];
    u64 s = 0;
    if (full) {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = in[first + k];
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = (first + k < n) ? in[first + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    u64 tot;
    u64 run = boff[bx] + block_excl_scan<SCAN_BLOCK>(s, sh, &tot);
    if (full) {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            out[first + k] = run;
            run += v[k];
        }
    } else {
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (first + k < n) out[first + k] = run;
            run += v[k];
        }
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(const u64* in, u64 n, const u64* __restrict__ boff,
                                                          u64* out) {
    scan_down_body(in, n, boff, out, blockIdx.x);
}

// One scan per job (blockIdx.y); blocks past a job's own size return at once.
__global__ __launch_bounds__(SCAN_BLOCK) void k_bscan_reduce(const BScanJob* __restrict__ jobs) {
    const BScanJob J = jobs[blockIdx.y];
    if ((u64)blockIdx.x * SCAN_TILE >= (J.n ? J.n : 1)) return;  // n = 0: block 0 writes a zero sum
    scan_reduce_body(J.in, J.n, J.bsum, blockIdx.x);
}

__global__ __launch_bounds__(TOP_BLOCK) void k_bscan_top(const BScanJob* __restrict__ jobs) {
    const BScanJob J = jobs[blockIdx.y];
    scan_top_body(J.bsum, (J.n + SCAN_TILE - 1) / SCAN_TILE, J.total);
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_bscan_down(const BScanJob* __restrict__ jobs) {
    const BScanJob J = jobs[blockIdx.y];
    if ((u64)blockIdx.x * SCAN_TILE >= J.n) return;
    scan_down_body(J.in, J.n, J.bsum, J.out, blockIdx.x);
}

unsigned grid1d(u64 n, u64 per, u64 cap = 65536) {
    u64 g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

void launch_fill_f64(double* p, u64 n, double val, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid1d(n, 256 * 16, 1u << 20)), dim3(256), 0, s, p, n, val);
    SFCI_CHECK_HIP(hipGetLastError());
}

void launch_fill_u64(u64* p, u64 n, u64 val, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1d(n, 256 * 16, 1u << 20)), dim3(256), 0, s, p, n, val);
    SFCI_CHECK_HIP(hipGetLastError());
}

u64 scan_block_sums(u64 n) { return std::max<u64>(1, (n + SCAN_TILE - 1) / SCAN_TILE); }

void exclusive_scan_u64(sfci_problem* P, const u64* in, u64* out, u64 n, u64* total_dev, u64* bsum_ws) {
    const u64 nb = scan_block_sums(n);
    u64* bsum = bsum_ws ? bsum_ws : (u64*)P->ws_scan.get(nb * sizeof(u64));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, P->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TOP_BLOCK), 0, P->stream, bsum, nb, total_dev);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, P->stream, in, n, bsum, out);
    SFCI_CHECK_HIP(hipGetLastError());
}

void bscan_u64(hipStream_t st, const BScanJob* d_jobs, int n_jobs, u64 max_n) {
    const u64 nb = scan_block_sums(max_n);
    hipLaunchKernelGGL(k_bscan_reduce, dim3((unsigned)nb, (unsigned)n_jobs), dim3(SCAN_BLOCK), 0, st, d_jobs);
    hipLaunchKernelGGL(k_bscan_top, dim3(1, (unsigned)n_jobs), dim3(TOP_BLOCK), 0, st, d_jobs);
    hipLaunchKernelGGL(k_bscan_down, dim3((unsigned)nb, (unsigned)n_jobs), dim3(SCAN_BLOCK), 0, st, d_jobs);
    SFCI_CHECK_HIP(hipGetLastError());
}
