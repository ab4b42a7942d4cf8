// Small device utilities: fills and a three-phase exclusive scan of u64 counts.
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

// Block-wide inclusive scan of one value per thread (256 threads).
__device__ u64 block_incl_scan(u64 x, u64* sh) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        u64 y = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    u64 r = sh[t];
    __syncthreads();
    return r;
}

__global__ void k_scan_reduce(const u64* __restrict__ in, u64 n, u64* __restrict__ bsum) {
    __shared__ u64 sh[SCAN_BLOCK];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    u64 s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) s += in[i];
    }
    u64 inc = block_incl_scan(s, sh);
    if (threadIdx.x == SCAN_BLOCK - 1) bsum[blockIdx.x] = inc;
}

// Single block: exclusive scan of nb block sums in place, total to *total.
__global__ void k_scan_top(u64* __restrict__ bsum, u64 nb, u64* __restrict__ total) {
    __shared__ u64 sh[SCAN_BLOCK];
    __shared__ u64 tot;
    u64 carry = 0;
    for (u64 base = 0; base < nb; base += SCAN_BLOCK) {
        u64 i = base + threadIdx.x;
        u64 x = (i < nb) ? bsum[i] : 0;
        u64 inc = block_incl_scan(x, sh);
        if (i < nb) bsum[i] = carry + inc - x;
        if (threadIdx.x == SCAN_BLOCK - 1) tot = inc;
        __syncthreads();
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_down(const u64* __restrict__ in, u64 n, const u64* __restrict__ boff, u64* __restrict__ out) {
    __shared__ u64 sh[SCAN_BLOCK];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    u64 v[SCAN_ITEMS];
    u64 s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    u64 inc = block_incl_scan(s, sh);
    u64 run = boff[blockIdx.x] + inc - s;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
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

void exclusive_scan_u64(sfci_problem* P, const u64* in, u64* out, u64 n, u64* total_dev) {
    u64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    u64* bsum = (u64*)P->ws_scan.get(nb * sizeof(u64));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, P->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCK), 0, P->stream, bsum, nb, total_dev);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, P->stream, in, n, bsum, out);
    SFCI_CHECK_HIP(hipGetLastError());
}
