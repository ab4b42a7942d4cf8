// sfci_topm_noalloc: the truncation of sfci_topm for callers that cannot
// allocate device memory.  Every piece of working memory -- the radix-select
// state, the per-chunk counts and their scan sums, the norm's partial sums,
// the validation flags and the device-side counts -- lives in one file-scope
// device array.  Host code never passes that array's name to a kernel (in
// host code it is a stand-in, not a device address): its device address is
// looked up once per device with hipGetSymbolAddress and kept.
#include <mutex>
#include <string>

#include "../../include/sfci_noalloc.h"
#include "sfci_internal.h"

namespace {

constexpr u64 kMaxNnz = SFCI_TOPM_NOALLOC_MAX_NNZ;
constexpr u64 kChunk = 4096;  // candidates per selection chunk (select_chunks)
constexpr u64 kMaxChunks = kMaxNnz / kChunk;
constexpr u64 kMaxBsum = 64;  // >= scan_block_sums(kMaxChunks)

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffSt = 0;
constexpr size_t kOffCnt = kOffSt + up256(sizeof(SelState));
constexpr size_t kOffBsum = kOffCnt + up256(kMaxChunks * sizeof(u64));
constexpr size_t kOffRed = kOffBsum + up256(kMaxBsum * sizeof(u64));
constexpr size_t kRedDoubles = 1024 + 8;  // >= normalise_ws_doubles()
constexpr size_t kOffScal = kOffRed + up256(kRedDoubles * sizeof(double));
constexpr size_t kScalWords = 8;  // [0] nnz(v) [1] kept count [2] bad rank flag [3] order flag
constexpr size_t kScratchBytes = kOffScal + up256(kScalWords * sizeof(u64));

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev` (the current device), looked up
// on the first call there.
void* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw sfci_error(SFCI_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw sfci_error(SFCI_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

__global__ void k_check_ranks(const u64* __restrict__ r, u64 n, u64 ndet, u64* __restrict__ flags) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        if (r[i] >= ndet) flags[0] = 1;
        if (i > 0 && r[i] <= r[i - 1]) flags[1] = 1;
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        SFCI_CHECK_HIP(hipGetDevice(&prev));
        if (prev != dev) SFCI_CHECK_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" sfci_status sfci_topm_noalloc(sfci_problem* P, const sfci_svec* v, uint64_t M, int32_t normalise,
                                         int32_t tie_band, sfci_svec* out) {
    try {
        if (!P || !v || !out) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
        if (v->nnz > kMaxNnz)
            return (sfci_status)sfci_set_error(SFCI_E_ARG, "input has " + std::to_string(v->nnz) +
                                                               " entries; sfci_topm_noalloc takes at most " +
                                                               std::to_string(kMaxNnz));
        if (v->nnz && (!v->rank || !v->amp)) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL input arrays");
        DeviceGuard dg(P->device);
        unsigned char* base = (unsigned char*)scratch_on(P->device);
        SelWs ws{(SelState*)(base + kOffSt), (u64*)(base + kOffCnt), (u64*)(base + kOffBsum)};
        double* red = (double*)(base + kOffRed);
        u64* scal = (u64*)(base + kOffScal);
        const u64 n = v->nnz;
        if (select_chunks(n) > kMaxChunks || scan_block_sums(select_chunks(n)) > kMaxBsum ||
            normalise_ws_doubles() > kRedDoubles)
            throw sfci_error(SFCI_E_DEVICE, "scratch layout too small");
        // the previous call's contents are still there: clear what must start at zero
        launch_fill_u64(scal, kScalWords, 0, P->stream);
        launch_fill_u64(scal, 1, n, P->stream);
        if (n) {
            const unsigned g = (unsigned)std::min<u64>(16384, (n + 255) / 256);
            hipLaunchKernelGGL(k_check_ranks, dim3(g), dim3(256), 0, P->stream, v->rank, n, P->Ndet, scal + 2);
            SFCI_CHECK_HIP(hipGetLastError());
        }
        P->tie_band = tie_band ? 1 : 0;
        CandSrc src{};
        src.lrank = v->rank;
        src.lval = v->amp;
        src.lcount = scal;
        src.lcap = std::max<u64>(1, n);
        select_prepare_ws(P, src, M, scal + 1, ws);
        u64 h[4] = {0, 0, 0, 0};
        SFCI_CHECK_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, P->stream));
        SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
        if (h[2]) return (sfci_status)sfci_set_error(SFCI_E_RANGE, "input rank >= N_det");
        if (h[3]) return (sfci_status)sfci_set_error(SFCI_E_DUP, "input ranks not strictly ascending");
        const u64 need = h[1];
        if (need > out->capacity || (need && (!out->rank || !out->amp))) {
            out->nnz = need;
            return (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "output capacity too small");
        }
        if (need) select_write_ws(P, src, out->rank, out->amp, ws);
        if (normalise && need) launch_normalise(P, out->amp, scal + 1, need, true, red);
        out->nnz = need;
        SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
        return SFCI_OK;
    } catch (const sfci_error& e) {
        return (sfci_status)sfci_set_error(e.code, e.msg);
    }
}
