// Device ceilings of the memory operations sigma is built from: streaming
// copy, random 8-byte gathers, random FP64 atomic adds into HBM, and FP64
// atomic adds / random reads in LDS.  These are the roofs the benchmark
// reports a sigma launch against (the method itself is in the other files).
// Every index is a hash of the thread and iteration, scaled into the array
// by a 64-bit high multiply, so every access stays inside its buffer.
#include <algorithm>
#include <string>

#include "../../include/sfci_roof.h"
#include "sfci_internal.h"

namespace {

constexpr int PB = 256;            // threads per block
constexpr int LDS_SLOTS = 8192;    // 64 KiB of doubles per block

__device__ __forceinline__ u64 mix64(u64 x) {
    // splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ __launch_bounds__(PB) void k_copy(const double2* __restrict__ a, double2* __restrict__ b, u64 n) {
    for (u64 i = (u64)blockIdx.x * PB + threadIdx.x; i < n; i += (u64)gridDim.x * PB) b[i] = a[i];
}

__global__ __launch_bounds__(PB) void k_gather(const double* __restrict__ a, u64 slots, unsigned per,
                                               double* __restrict__ sink) {
    const u64 tid = (u64)blockIdx.x * PB + threadIdx.x;
    double s = 0.0;
    for (unsigned i = 0; i < per; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = a[__umul64hi(mix64(tid * per + i + u), slots)];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    sink[tid] = s;
}

__global__ __launch_bounds__(PB) void k_atomic(double* __restrict__ a, u64 slots, unsigned per) {
    const u64 tid = (u64)blockIdx.x * PB + threadIdx.x;
    for (unsigned i = 0; i < per; ++i) atomicAdd(a + __umul64hi(mix64(tid * per + i), slots), 1.0);
}

template <int PATTERN>
__global__ __launch_bounds__(PB) void k_lds_atomic(double* __restrict__ sink, unsigned per) {
    __shared__ double acc[LDS_SLOTS];
    for (int t = threadIdx.x; t < LDS_SLOTS; t += PB) acc[t] = 0.0;
    __syncthreads();
    const unsigned lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 tid = (u64)blockIdx.x * PB + threadIdx.x;
    for (unsigned i = 0; i < per; ++i) {
        unsigned idx;
        if (PATTERN == 0) idx = (lane + 64u * ((i * 4u + wave) & (LDS_SLOTS / 64 - 1)));
        else idx = (unsigned)(mix64(tid * per + i) & (LDS_SLOTS - 1));
        atomicAdd(&acc[idx], 1.0);
    }
    __syncthreads();
    sink[tid] = acc[threadIdx.x];
}

__global__ __launch_bounds__(PB) void k_lds_read(double* __restrict__ sink, unsigned per) {
    __shared__ double acc[LDS_SLOTS];
    for (int t = threadIdx.x; t < LDS_SLOTS; t += PB) acc[t] = (double)t;
    __syncthreads();
    const u64 tid = (u64)blockIdx.x * PB + threadIdx.x;
    double s = 0.0;
    for (unsigned i = 0; i < per; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = acc[mix64(tid * per + i + u) & (LDS_SLOTS - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    sink[tid] = s;
}

struct Timer {
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    explicit Timer(hipStream_t st) : s(st) {
        SFCI_CHECK_HIP(hipEventCreate(&a));
        SFCI_CHECK_HIP(hipEventCreate(&b));
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    // best of three runs of f, in milliseconds
    template <class F>
    double best(F&& f) {
        double m = 1e300;
        for (int r = 0; r < 3; ++r) {
            SFCI_CHECK_HIP(hipEventRecord(a, s));
            f();
            SFCI_CHECK_HIP(hipEventRecord(b, s));
            SFCI_CHECK_HIP(hipEventSynchronize(b));
            float ms = 0.f;
            SFCI_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
            m = std::min(m, (double)ms);
        }
        SFCI_CHECK_HIP(hipGetLastError());
        return m;
    }
};

struct Buf {
    void* p = nullptr;
    explicit Buf(size_t bytes) {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw sfci_error(SFCI_E_NOMEM, "probe buffer of " + std::to_string(bytes) + " bytes");
        }
    }
    ~Buf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" sfci_status sfci_roof_probe(uint64_t big_bytes, void* stream, sfci_roof* out) {
    try {
        if (!out || big_bytes < (128ull << 20)) return (sfci_status)sfci_set_error(SFCI_E_ARG, "bad argument");
        hipStream_t st = (hipStream_t)stream;
        int dev = 0, ncu = 0;
        SFCI_CHECK_HIP(hipGetDevice(&dev));
        SFCI_CHECK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if (ncu < 1) ncu = 256;
        const unsigned grid = (unsigned)ncu * 8;
        const u64 threads = (u64)grid * PB;
        Timer T(st);
        *out = sfci_roof{};
        out->big_bytes = big_bytes;
        Buf sink(threads * sizeof(double));
        {
            const u64 cb = 1ull << 30;
            Buf a(cb), b(cb);
            launch_fill_f64((double*)a.p, cb / 8, 1.0, st);
            const double ms = T.best([&] {
                hipLaunchKernelGGL(k_copy, dim3(grid), dim3(PB), 0, st, (const double2*)a.p, (double2*)b.p, cb / 16);
            });
            out->copy_GBps = 2.0 * (double)cb / (ms * 1e-3) / 1e9;
        }
        Buf big(big_bytes);
        launch_fill_f64((double*)big.p, big_bytes / 8, 0.0, st);
        const u64 sizes[3] = {2ull << 20, 128ull << 20, big_bytes};
        const unsigned per = 256;
        for (int k = 0; k < 3; ++k) {
            const u64 slots = sizes[k] / 8;
            const double mg = T.best([&] {
                hipLaunchKernelGGL(k_gather, dim3(grid), dim3(PB), 0, st, (const double*)big.p, slots, per,
                                   (double*)sink.p);
            });
            out->gather_Gops[k] = (double)threads * per / (mg * 1e-3) / 1e9;
            const double ma = T.best([&] {
                hipLaunchKernelGGL(k_atomic, dim3(grid), dim3(PB), 0, st, (double*)big.p, slots, per);
            });
            out->atomic_Gops[k] = (double)threads * per / (ma * 1e-3) / 1e9;
        }
        const unsigned lper = 1024;
        const double l0 = T.best([&] {
            hipLaunchKernelGGL(k_lds_atomic<0>, dim3(grid), dim3(PB), 0, st, (double*)sink.p, lper);
        });
        const double l1 = T.best([&] {
            hipLaunchKernelGGL(k_lds_atomic<1>, dim3(grid), dim3(PB), 0, st, (double*)sink.p, lper);
        });
        const double lr = T.best([&] {
            hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(PB), 0, st, (double*)sink.p, lper);
        });
        out->lds_atomic_Gops[0] = (double)threads * lper / (l0 * 1e-3) / 1e9;
        out->lds_atomic_Gops[1] = (double)threads * lper / (l1 * 1e-3) / 1e9;
        out->lds_read_Gops = (double)threads * lper / (lr * 1e-3) / 1e9;
        SFCI_CHECK_HIP(hipStreamSynchronize(st));
        return SFCI_OK;
    } catch (const sfci_error& e) {
        return (sfci_status)sfci_set_error(e.code, e.msg);
    }
}
