// C ABI of libsfci: problem lifecycle, sigma, truncation and the SFCI
// iteration driver (Sec. 2.1).  All device work goes to the problem's stream.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/sfci.h"
#include "sfci_internal.h"

static thread_local std::string g_last_error;

int sfci_set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

static std::atomic<u64> g_free_epoch{0};

u64 device_free_epoch() { return g_free_epoch.load(); }

void note_device_free() { g_free_epoch.fetch_add(1); }

void DevBuf::release() {
    if (p) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p);
        note_device_free();
    }
    p = nullptr;
    bytes = 0;
}

void* DevBuf::get(size_t need) {
    if (need == 0) need = 8;
    if (need <= bytes) return p;
    release();
    size_t nb = need + need / 4;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        bytes = 0;
        throw sfci_error(SFCI_E_NOMEM, "device allocation of " + std::to_string(nb) + " bytes failed");
    }
    bytes = nb;
    return p;
}

namespace {

#define SFCI_GUARD_BEGIN try {
#define SFCI_GUARD_END                                                   \
    }                                                                    \
    catch (const sfci_error& e) {                                        \
        return (sfci_status)sfci_set_error(e.code, e.msg);               \
    }                                                                    \
    catch (const std::exception& e) {                                    \
        return (sfci_status)sfci_set_error(SFCI_E_DEVICE, e.what());     \
    }

u64 binom_host(int a, int b) {
    if (b < 0 || a < b) return 0;
    u64 r = 1;
    for (int i = 1; i <= b; ++i) r = r * (u64)(a - b + i) / (u64)i;  // exact at every step
    return r;
}

int bits_for(u64 maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b < 1 ? 1 : b;
}

__global__ void k_validate(const u64* __restrict__ r, u64 n, u64 ndet, int* __restrict__ flags) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        if (r[i] >= ndet) flags[0] = 1;
        if (i > 0 && r[i] <= r[i - 1]) flags[1] = 1;
    }
}

// The fast-mode reductions keep their partial sums at the front of ws_red.
constexpr u64 RAW_PAD = 2048;

__global__ void k_set_u64(u64* p, u64 v) {
    if (threadIdx.x == 0) *p = v;
}

unsigned g1(u64 n) {
    u64 g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

}  // namespace

void sfci_sync(sfci_problem* P) { SFCI_CHECK_HIP(hipStreamSynchronize(P->stream)); }
static void sync(sfci_problem* P) { sfci_sync(P); }

void launch_set_u64(sfci_problem* P, u64* p, u64 v) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, p, v);
    SFCI_CHECK_HIP(hipGetLastError());
}

namespace {

u64 read_u64(sfci_problem* P, const u64* d) {
    u64 h = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&h, d, sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    return h;
}

}  // namespace

void validate_vec(sfci_problem* P, const u64* r, u64 n) {
    if (n == 0) return;
    int* flags = (int*)P->ws_scalar.get(64);
    SFCI_CHECK_HIP(hipMemsetAsync(flags, 0, 2 * sizeof(int), P->stream));
    hipLaunchKernelGGL(k_validate, dim3(g1(n)), dim3(256), 0, P->stream, r, n, P->Ndet, flags);
    int hf[2] = {0, 0};
    SFCI_CHECK_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    if (hf[0]) throw sfci_error(SFCI_E_RANGE, "input rank >= N_det");
    if (hf[1]) throw sfci_error(SFCI_E_DUP, "input ranks not strictly ascending");
}

bool ensure_dense(sfci_problem* P) {
    if (P->dense_state == 0) {
        size_t freeb = 0, totb = 0;
        SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
        const double need = (double)P->Ndet * 8.0;
        const double margin = 4.0 * 1024 * 1024 * 1024;
        if (need + margin > (double)freeb) {
            P->dense_state = -1;
        } else {
            hipError_t e = hipMalloc(&P->d_D, (size_t)P->Ndet * 8);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                P->dense_state = -1;
            } else {
                launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
                P->dense_state = 1;
            }
        }
    }
    return P->dense_state == 1;
}

// Dense-mode sigma into P->d_D: the target-owned tile kernel unless the
// caller asks for the one-atomic-per-term kernel (or the tiles do not fit).
void dense_sigma(sfci_problem* P, const SigmaLaunch& sl, int dedup, unsigned long long* emitted, double eps) {
    if (dedup != SFCI_DEDUP_DENSE_ATOMIC && rowtile_available(P)) {
        launch_sigma_rowtile(P, sl, P->d_D, emitted, eps);
    } else {
        launch_sigma_dense(P, sl, P->d_D, emitted);
        if (eps > 0.0) launch_screen(P, P->d_D, P->Ndet, eps);
    }
}

bool halt_after_block(sfci_problem* P, const sfci_lanczos_opts* o, const double* energies_d, int b) {
    if (!(o->conv_eps > 0.0) || b < 1) return false;
    double e[2];
    SFCI_CHECK_HIP(hipMemcpyAsync(e, energies_d + b - 1, sizeof(e), hipMemcpyDeviceToHost, P->stream));
    sfci_sync(P);
    return e[0] - e[1] < o->conv_eps;
}

extern "C" {

const char* sfci_last_error(void) { return g_last_error.c_str(); }

sfci_status sfci_space_size(const sfci_space* sp, uint64_t* n_det) {
    if (!sp || !n_det) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    if (sp->n_orb < 1 || sp->n_orb > 32) return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "n_orb must be 1..32");
    if (sp->n_alpha < 0 || sp->n_beta < 0 || sp->n_alpha > sp->n_orb || sp->n_beta > sp->n_orb)
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "electron count outside 0..n_orb");
    unsigned __int128 p = (unsigned __int128)binom_host(sp->n_orb, sp->n_alpha) * binom_host(sp->n_orb, sp->n_beta);
    if (p >> 64) return (sfci_status)sfci_set_error(SFCI_E_RANGE, "N_det does not fit in 64 bits");
    *n_det = (uint64_t)p;
    return SFCI_OK;
}

sfci_status sfci_problem_create(const sfci_space* sp, const double* h, const double* eri, void* stream,
                                sfci_problem** out) {
    SFCI_GUARD_BEGIN
    if (!sp || !h || !eri || !out) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    u64 ndet = 0;
    sfci_status st = sfci_space_size(sp, &ndet);
    if (st != SFCI_OK) return st;
    const int n = sp->n_orb;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (h[p * n + q] != h[q * n + p]) return (sfci_status)sfci_set_error(SFCI_E_NOTSYM, "h not symmetric");
    auto G = [&](int p, int q, int r, int s) { return eri[((size_t)(p * n + q) * n + r) * n + s]; };
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double v = G(p, q, r, s);
                    if (v != G(q, p, r, s) || v != G(p, q, s, r) || v != G(r, s, p, q))
                        return (sfci_status)sfci_set_error(SFCI_E_NOTSYM, "eri not 8-fold symmetric");
                }
    sfci_problem* P = new sfci_problem();
    P->n = n;
    P->na = sp->n_alpha;
    P->nb = sp->n_beta;
    P->Na = binom_host(n, P->na);
    P->Nb = binom_host(n, P->nb);
    P->Ndet = ndet;
    P->kg.rank_bits = bits_for(ndet - 1);
    P->kg.ndig = (63 + P->kg.rank_bits + 10) / 11;
    P->kg.pad_bits = 0;
    P->kg.ndet_m1 = ndet - 1;
    P->stream = (hipStream_t)stream;
    try {
        SFCI_CHECK_HIP(hipGetDevice(&P->device));
        int ncu = 0;
        SFCI_CHECK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device));
        P->num_cu = ncu > 0 ? ncu : 256;
        SFCI_CHECK_HIP(hipMalloc(&P->d_h, sizeof(double) * n * n));
        SFCI_CHECK_HIP(hipMalloc(&P->d_g, sizeof(double) * (size_t)n * n * n * n));
        SFCI_CHECK_HIP(hipMalloc(&P->d_binom, sizeof(u64) * 33 * 33));
        std::vector<u64> tab(33 * 33);
        for (int a = 0; a <= 32; ++a)
            for (int b = 0; b <= 32; ++b) tab[a * 33 + b] = binom_host(a, b);
        SFCI_CHECK_HIP(hipMemcpy(P->d_h, h, sizeof(double) * n * n, hipMemcpyHostToDevice));
        SFCI_CHECK_HIP(hipMemcpy(P->d_g, eri, sizeof(double) * (size_t)n * n * n * n, hipMemcpyHostToDevice));
        SFCI_CHECK_HIP(hipMemcpy(P->d_binom, tab.data(), sizeof(u64) * 33 * 33, hipMemcpyHostToDevice));
    } catch (...) {
        sfci_problem_destroy(P);
        throw;
    }
    *out = P;
    return SFCI_OK;
    SFCI_GUARD_END
}

sfci_status sfci_problem_destroy(sfci_problem* P) {
    if (!P) return SFCI_OK;
    (void)hipStreamSynchronize(P->stream);
    note_device_free();
    if (P->swapped) sfci_problem_destroy(P->swapped);
    if (!P->borrowed) {
        if (P->d_h) (void)hipFree(P->d_h);
        if (P->d_g) (void)hipFree(P->d_g);
        if (P->d_binom) (void)hipFree(P->d_binom);
        if (P->d_D) (void)hipFree(P->d_D);
    }
    rowtile_release(P);
    DevBuf* bufs[] = {&P->ws_sel,   &P->ws_cnt,   &P->ws_scan,  &P->ws_scan2,  &P->ws_scalar, &P->ws_red,
                      &P->ws_tup_k, &P->ws_tup_v, &P->ws_tup_k2, &P->ws_tup_v2, &P->ws_seg_v, &P->ws_seg_f,
                      &P->ws_src_cnt, &P->ws_src_off, &P->ws_hist, &P->ws_list_r, &P->ws_list_a, &P->ws_prod,
                      &P->ws_sel2,    &P->ws_cand_r, &P->ws_cand_a};
    for (DevBuf* b : bufs) b->release();
    for (auto& b : P->ws_lz) b.release();
    P->ws_rt_rows.release();
    P->ws_rt_beta.release();
    P->ws_rt_nbr.release();
    P->ws_rt_desc.release();
    for (DevBuf* b : {&P->ws_ab_rc, &P->ws_ab_cr, &P->ws_ab_off, &P->ws_ab_it, &P->ws_rt_phase})
        b->release();
    P->grad_ws.release();
    P->list_ws.release();
    for (int i = 0; i < SFCI_MAX_ROOTS; ++i) {
        P->ws_hroot_r[i].release();
        P->ws_hroot_a[i].release();
    }
    P->ws_roots_sc.release();
    P->ws_roots_cnt.release();
    P->rowpass_ws.release();
    delete P;
    return SFCI_OK;
}

sfci_status sfci_rank(sfci_problem* P, const uint64_t* a, const uint64_t* b, uint64_t cnt, uint64_t* rank) {
    SFCI_GUARD_BEGIN
    if (!P || (cnt && (!a || !b || !rank))) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    int* bad = (int*)P->ws_scalar.get(64);
    SFCI_CHECK_HIP(hipMemsetAsync(bad, 0, sizeof(int), P->stream));
    launch_rank(P, a, b, cnt, rank, bad);
    int hb = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    if (hb) return (sfci_status)sfci_set_error(SFCI_E_ARG, "string with wrong electron count or bits >= n");
    return SFCI_OK;
    SFCI_GUARD_END
}

sfci_status sfci_unrank(sfci_problem* P, const uint64_t* rank, uint64_t cnt, uint64_t* a, uint64_t* b) {
    SFCI_GUARD_BEGIN
    if (!P || (cnt && (!a || !b || !rank))) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    int* bad = (int*)P->ws_scalar.get(64);
    SFCI_CHECK_HIP(hipMemsetAsync(bad, 0, sizeof(int), P->stream));
    launch_unrank(P, rank, cnt, a, b, bad);
    int hb = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    if (hb) return (sfci_status)sfci_set_error(SFCI_E_RANGE, "rank >= N_det");
    return SFCI_OK;
    SFCI_GUARD_END
}

sfci_status sfci_sigma(sfci_problem* P, const sfci_svec* v, const sfci_sigma_opts* opts, sfci_svec* out,
                       sfci_sigma_stats* stats) {
    SFCI_GUARD_BEGIN
    if (!P || !v || !opts || !out) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    if (v->nnz && (!v->rank || !v->amp)) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL input arrays");
    if (opts->dedup < 0 || opts->dedup > 3) return (sfci_status)sfci_set_error(SFCI_E_ARG, "bad dedup mode");
    if (!(opts->screen_eps >= 0.0) || !(opts->excite_eps >= 0.0))
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "screen_eps and excite_eps must be >= 0");
    validate_vec(P, v->rank, v->nnz);
    P->tie_band = opts->tie_band ? 1 : 0;
    P->excite_eps = opts->excite_eps;
    hipEvent_t e0, e1;
    SFCI_CHECK_HIP(hipEventCreate(&e0));
    SFCI_CHECK_HIP(hipEventCreate(&e1));
    SFCI_CHECK_HIP(hipEventRecord(e0, P->stream));
    u64* scal = (u64*)P->ws_lz[0].get(8 * sizeof(u64));  // [0] nnz(v) [1] emitted [2] count [3] list count
    launch_fill_u64(scal, 8, 0, P->stream);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, scal, (u64)v->nnz);
    SigmaLaunch sl{v->rank, v->amp, scal, v->nnz};
    const u64 tps = terms_per_source(P->n, P->na, P->nb);
    bool use_sort = opts->deterministic || opts->dedup == SFCI_DEDUP_SORT;
    bool list_tiles = false;  // no N_det array, fast: the tile kernel's slices may serve
    if (!use_sort && !ensure_dense(P)) {
        if (opts->dedup == SFCI_DEDUP_DENSE || opts->dedup == SFCI_DEDUP_DENSE_ATOMIC)
            return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "dense accumulator does not fit on the device");
        use_sort = true;
        list_tiles = true;
    }
    if (use_sort) {
        // alpha-range passes (sort path, or tile-kernel slices in fast mode)
        // into a running top-M candidate list, no N_det array and no
        // full-length sigma list
        u64 distinct = 0;
        const u64 need = sigma_list_topm(P, sl, opts->M, out->rank, out->amp,
                                         (out->rank && out->amp) ? out->capacity : 0, &scal[1], &distinct,
                                         list_tiles, opts->screen_eps);
        SFCI_CHECK_HIP(hipEventRecord(e1, P->stream));
        const u64 emitted = read_u64(P, &scal[1]);
        out->nnz = need;
        sfci_status rc = SFCI_OK;
        if (need > out->capacity || (need && (!out->rank || !out->amp)))
            rc = (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "output capacity " + std::to_string(out->capacity) +
                                                                   " < " + std::to_string(need));
        if (stats) {
            float ms = 0.f;
            SFCI_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            stats->ms = ms;
            stats->terms_enumerated = v->nnz * tps;
            stats->terms_emitted = emitted;
            stats->candidates = distinct;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
    }
    CandSrc src{};
    dense_sigma(P, sl, opts->dedup, (unsigned long long*)&scal[1], opts->screen_eps);
    src.dense = P->d_D;
    select_prepare(P, src, opts->M, &scal[2]);
    u64 hs[4];
    SFCI_CHECK_HIP(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    const u64 need = hs[2];
    sfci_status rc = SFCI_OK;
    if (need > out->capacity || (need && (!out->rank || !out->amp))) {
        launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
        out->nnz = need;
        rc = (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "output capacity " + std::to_string(out->capacity) +
                                                               " < " + std::to_string(need));
    } else {
        select_write(P, src, out->rank, out->amp, true);
        out->nnz = need;
    }
    SFCI_CHECK_HIP(hipEventRecord(e1, P->stream));
    sync(P);
    if (stats) {
        float ms = 0.f;
        SFCI_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        stats->ms = ms;
        stats->terms_enumerated = v->nnz * tps;
        stats->terms_emitted = hs[1];
        SelState sst;
        SFCI_CHECK_HIP(hipMemcpy(&sst, P->ws_sel.p, sizeof(SelState) - sizeof(sst.hist), hipMemcpyDeviceToHost));
        stats->candidates = sst.take_all ? sst.count_out : sst.total;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
    SFCI_GUARD_END
}

sfci_status sfci_topm(sfci_problem* P, const sfci_svec* v, uint64_t M, int32_t normalise, int32_t tie_band,
                      sfci_svec* out) {
    SFCI_GUARD_BEGIN
    if (!P || !v || !out) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    validate_vec(P, v->rank, v->nnz);
    P->tie_band = tie_band ? 1 : 0;
    u64* scal = (u64*)P->ws_lz[0].get(8 * sizeof(u64));
    launch_fill_u64(scal, 8, 0, P->stream);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, scal, (u64)v->nnz);
    CandSrc src{};
    src.lrank = v->rank;
    src.lval = v->amp;
    src.lcount = scal;
    src.lcap = v->nnz;
    select_prepare(P, src, M, &scal[1]);
    u64 need = read_u64(P, &scal[1]);
    if (need > out->capacity) {
        out->nnz = need;
        return (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "output capacity too small");
    }
    if (need) select_write(P, src, out->rank, out->amp, false);
    if (normalise && need) launch_normalise(P, out->amp, &scal[1], need, true);
    out->nnz = need;
    sync(P);
    return SFCI_OK;
    SFCI_GUARD_END
}

sfci_status sfci_lanczos(sfci_problem* P, const sfci_svec* v0, const sfci_lanczos_opts* o, double* energies,
                         sfci_svec* psi_out, double* T_out, double* S_out, sfci_lanczos_stats* stats) {
    return sfci_lanczos_roots(P, v0, o, nullptr, 0, energies, psi_out, T_out, S_out, stats);
}

namespace {
__global__ void k_div_scalar(const double* __restrict__ num, const double* __restrict__ den, double* __restrict__ out) {
    if (threadIdx.x == 0) *out = *num / *den;
}
}  // namespace

sfci_status sfci_lanczos_roots(sfci_problem* P, const sfci_svec* v0, const sfci_lanczos_opts* o,
                               const sfci_svec* roots, int32_t n_roots, double* energies, sfci_svec* psi_out,
                               double* T_out, double* S_out, sfci_lanczos_stats* stats) {
    SFCI_GUARD_BEGIN
    if (!P || !v0 || !o || !energies) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    if (n_roots < 0 || n_roots > SFCI_MAX_ROOTS || (n_roots > 0 && !roots))
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "need 0 <= n_roots <= SFCI_MAX_ROOTS root vectors");
    for (int i = 0; i < n_roots; ++i) {
        if (roots[i].nnz == 0 || !roots[i].rank || !roots[i].amp)
            return (sfci_status)sfci_set_error(SFCI_E_ARG, "empty root vector");
        validate_vec(P, roots[i].rank, roots[i].nnz);
    }
    if (o->n_L < 1 || o->n_L > 32 || o->n_iter < o->n_L)
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "need 1 <= n_L <= 32 and n_iter >= n_L");
    if (v0->nnz == 0) return (sfci_status)sfci_set_error(SFCI_E_ARG, "empty start vector");
    if (!(o->screen_eps >= 0.0) || !(o->conv_eps >= 0.0) || !(o->excite_eps >= 0.0))
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "screen_eps, conv_eps and excite_eps must be >= 0");
    validate_vec(P, v0->rank, v0->nnz);
    P->tie_band = o->tie_band ? 1 : 0;
    P->excite_eps = o->excite_eps;
    const int nL = o->n_L;
    const int nblk = o->n_iter / nL;
    const bool det = o->deterministic != 0;
    const bool list_mode = o->no_dense != 0 || !ensure_dense(P);
    if (list_mode && n_roots > 0)
        return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "projected roots need the dense accumulator");
    // a truncated vector holds at most M entries (M + SFCI_TIE_SLACK with the tie band)
    const u64 cap = (o->M >= P->Ndet) ? P->Ndet
                                      : std::min<u64>(std::max<u64>(o->M + tie_extra(P), v0->nnz), P->Ndet);
    const u64 tps = terms_per_source(P->n, P->na, P->nb);
    // basis storage
    u64* Wr = (u64*)P->ws_lz[1].get((size_t)nL * cap * sizeof(u64));
    double* Wa = (double*)P->ws_lz[2].get((size_t)nL * cap * sizeof(double));
    const int nsc = 64 + 2 * nL;
    u64* sc = (u64*)P->ws_lz[3].get(nsc * sizeof(u64));  // [0..nL) nnz, [32] emitted, [33] list count, [34] psi count
    double* Td = (double*)P->ws_lz[4].get((size_t)(nblk * 2 + 1) * nL * nL * sizeof(double) + 64 * sizeof(double));
    double* Sd = Td + (size_t)nblk * nL * nL;
    double* xd = Sd + (size_t)nblk * nL * nL;
    double* lam = xd + 32;
    double* en = lam + 1;
    (void)en;
    double* energies_d = (double*)P->ws_lz[5].get((size_t)(nblk + 1) * sizeof(double));
    int* status = (int*)P->ws_lz[6].get(64);
    launch_fill_u64(sc, nsc, 0, P->stream);
    launch_fill_f64(Td, (size_t)nblk * 2 * nL * nL, 0.0, P->stream);
    SFCI_CHECK_HIP(hipMemsetAsync(status, 0, sizeof(int), P->stream));
    u64 lcap = 0;
    u64 *lr = nullptr;
    double* la = nullptr;
    if (det && !list_mode) {
        lcap = std::min<u64>(P->Ndet, cap * tps);
        lr = (u64*)P->ws_list_r.get(lcap * sizeof(u64));
        la = (double*)P->ws_list_a.get(lcap * sizeof(double));
    }
    auto W = [&](int j) { return DVec{Wr + (size_t)j * cap, Wa + (size_t)j * cap, sc + j, cap}; };
    EventTimer tsig;
    tsig.on = (stats != nullptr);
    hipEvent_t e0, e1;
    SFCI_CHECK_HIP(hipEventCreate(&e0));
    SFCI_CHECK_HIP(hipEventCreate(&e1));
    SFCI_CHECK_HIP(hipEventRecord(e0, P->stream));
    // Projected roots (excited states, Sec. 4): <Psi_i|Psi_i> and H Psi_i once;
    // per root scalars: [0] q, [1] c or d numerator, [2] c or d.
    double* rsc = (double*)P->ws_roots_sc.get((size_t)(3 * SFCI_MAX_ROOTS + 8) * sizeof(double));
    u64* rcnt = (u64*)P->ws_roots_cnt.get((size_t)(2 * SFCI_MAX_ROOTS + 8) * sizeof(u64));
    std::vector<u64> hcap(n_roots, 0);
    for (int i = 0; i < n_roots; ++i) {
        launch_set_u64(P, rcnt + i, roots[i].nnz);
        launch_sumsq(P, roots[i].amp, rcnt + i, roots[i].nnz, rsc + 3 * i, det);
        u64 *yr;
        double* ya;
        const SigmaLaunch rl{roots[i].rank, roots[i].amp, rcnt + i, roots[i].nnz};
        P->excite_eps = 0.0;  // H Psi_i in full
        const u64 ny = sigma_full_list(P, rl, det, sc + 40, &yr, &ya, rcnt + SFCI_MAX_ROOTS + i);
        P->excite_eps = o->excite_eps;
        hcap[i] = std::max<u64>(1, ny);
        u64* hr = (u64*)P->ws_hroot_r[i].get(hcap[i] * sizeof(u64));
        double* ha = (double*)P->ws_hroot_a[i].get(hcap[i] * sizeof(double));
        if (ny) {
            SFCI_CHECK_HIP(hipMemcpyAsync(hr, yr, ny * sizeof(u64), hipMemcpyDeviceToDevice, P->stream));
            SFCI_CHECK_HIP(hipMemcpyAsync(ha, ya, ny * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
        }
    }
    // D <- P D: D -= (<Psi_i|D>/q_i) Psi_i, roots in order
    auto project_dense = [&]() {
        for (int i = 0; i < n_roots; ++i) {
            launch_dot_dense(P, roots[i].rank, roots[i].amp, rcnt + i, roots[i].nnz, P->d_D, rsc + 3 * i + 1,
                             nullptr, det);
            hipLaunchKernelGGL(k_div_scalar, dim3(1), dim3(64), 0, P->stream, rsc + 3 * i + 1, rsc + 3 * i,
                               rsc + 3 * i + 2);
            launch_axpy_scatter(P, P->d_D, roots[i].rank, roots[i].amp, rcnt + i, roots[i].nnz, rsc + 3 * i + 2,
                                -1.0);
        }
    };
    // w_0 = v0 / |v0| (with roots: the projected start, truncated to M)
    if (n_roots == 0) {
        DVec w = W(0);
        SFCI_CHECK_HIP(hipMemcpyAsync(w.r, v0->rank, v0->nnz * sizeof(u64), hipMemcpyDeviceToDevice, P->stream));
        SFCI_CHECK_HIP(hipMemcpyAsync(w.a, v0->amp, v0->nnz * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, w.nnz, (u64)v0->nnz);
        launch_normalise(P, w.a, w.nnz, cap, det);
    } else {
        DVec w = W(0);
        launch_set_u64(P, rcnt + 2 * SFCI_MAX_ROOTS, v0->nnz);
        launch_scatter_set(P, P->d_D, v0->rank, v0->amp, rcnt + 2 * SFCI_MAX_ROOTS, v0->nnz);
        project_dense();
        CandSrc src{};
        src.dense = P->d_D;
        select_topm(P, src, o->M, w.r, w.a, w.nnz, true);
        launch_normalise(P, w.a, w.nnz, cap, det);
    }
    u64 sigma_calls = 0;
    u64* nnz_hist = (u64*)P->ws_lz[7].get((size_t)(nblk * nL + 1) * sizeof(u64));
    u64 psi_n = 0;
    int blocks_run = 0;
    if (list_mode) {
        ListBasis LB{cap, Wr, Wa, sc, Td, Sd, xd, lam, energies_d, status, nnz_hist};
        lanczos_list(P, o, LB, psi_out, &psi_n, &sigma_calls, tsig, &blocks_run);
    }
    for (int b = 0; b < (list_mode ? 0 : nblk); ++b) {
        double* T = Td + (size_t)b * nL * nL;
        double* S = Sd + (size_t)b * nL * nL;
        for (int j = 0; j < nL; ++j) {
            DVec wj = W(j);
            SFCI_CHECK_HIP(hipMemcpyAsync(nnz_hist + (size_t)b * nL + j, wj.nnz, sizeof(u64), hipMemcpyDeviceToDevice,
                                          P->stream));
            SigmaLaunch sl{wj.r, wj.a, wj.nnz, cap};
            tsig.begin(P->stream);
            if (det) {
                sigma_sorted(P, sl, lcap, lr, la, sc + 33, sc + 32);
                tsig.end(P->stream);
                launch_scatter_set(P, P->d_D, lr, la, sc + 33, lcap);
                if (o->screen_eps > 0.0) launch_screen(P, P->d_D, P->Ndet, o->screen_eps);
            } else {
                dense_sigma(P, sl, o->dedup, (unsigned long long*)(sc + 32), o->screen_eps);
                tsig.end(P->stream);
            }
            if (n_roots > 0) {
                // H P w_j = H w_j - sum_i c_i H Psi_i, c_i = <Psi_i|w_j>/q_i; then P
                for (int i = 0; i < n_roots; ++i) {
                    launch_dot_sparse(P, roots[i].rank, roots[i].amp, rcnt + i, roots[i].nnz, wj.r, wj.a, wj.nnz,
                                      rsc + 3 * i + 1, nullptr, det);
                    hipLaunchKernelGGL(k_div_scalar, dim3(1), dim3(64), 0, P->stream, rsc + 3 * i + 1, rsc + 3 * i,
                                       rsc + 3 * i + 2);
                    launch_axpy_scatter(P, P->d_D, (const u64*)P->ws_hroot_r[i].p, (const double*)P->ws_hroot_a[i].p,
                                        rcnt + SFCI_MAX_ROOTS + i, hcap[i], rsc + 3 * i + 2, -1.0);
                }
                project_dense();
            }
            ++sigma_calls;
            for (int l = 0; l <= j; ++l) {
                DVec wl = W(l);
                launch_dot_dense(P, wl.r, wl.a, wl.nnz, cap, P->d_D, T + l * nL + j, T + j * nL + l, det);
                launch_dot_sparse(P, wl.r, wl.a, wl.nnz, cap, wj.r, wj.a, wj.nnz, S + l * nL + j, S + j * nL + l, det);
            }
            if (j + 1 < nL) {
                launch_axpy_scatter(P, P->d_D, wj.r, wj.a, wj.nnz, cap, T + j * nL + j, -1.0);
                if (j >= 1) {
                    DVec wm = W(j - 1);
                    launch_axpy_scatter(P, P->d_D, wm.r, wm.a, wm.nnz, cap, T + (j - 1) * nL + j, -1.0);
                }
                DVec wn = W(j + 1);
                CandSrc src{};
                src.dense = P->d_D;
                select_topm(P, src, o->M == UINT64_MAX ? UINT64_MAX : o->M, wn.r, wn.a, wn.nnz, true);
                launch_normalise(P, wn.a, wn.nnz, cap, det);
            } else {
                launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
            }
        }
        launch_geneig_full(P, nL, T, S, lam, xd, energies_d + b, status);
        for (int j = 0; j < nL; ++j) {
            DVec wj = W(j);
            launch_axpy_scatter(P, P->d_D, wj.r, wj.a, wj.nnz, cap, xd + j, +1.0);
        }
        if (n_roots > 0) project_dense();
        CandSrc src{};
        src.dense = P->d_D;
        blocks_run = b + 1;
        if (b + 1 < nblk && !halt_after_block(P, o, energies_d, b)) {
            DVec w0 = W(0);
            select_topm(P, src, o->M, w0.r, w0.a, w0.nnz, true);
            launch_normalise(P, w0.a, w0.nnz, cap, det);
        } else {
            select_prepare(P, src, UINT64_MAX, sc + 34);
            break;
        }
    }
    // Final Psi (untruncated) into psi_out when it fits.
    sfci_status rc = SFCI_OK;
    if (list_mode) {
        if (psi_out) {
            if (psi_n > psi_out->capacity || (psi_n && (!psi_out->rank || !psi_out->amp)))
                rc = (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "psi_out capacity too small");
            psi_out->nnz = psi_n;
        }
    } else {
    psi_n = read_u64(P, sc + 34);
    CandSrc src{};
    src.dense = P->d_D;
    if (psi_out) {
        if (psi_n <= psi_out->capacity && psi_out->rank && psi_out->amp) {
            select_write(P, src, psi_out->rank, psi_out->amp, true);
            psi_out->nnz = psi_n;
        } else {
            launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
            psi_out->nnz = psi_n;
            rc = (sfci_status)sfci_set_error(SFCI_E_CAPACITY, "psi_out capacity too small");
        }
    } else {
        launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
    }
    }
    SFCI_CHECK_HIP(hipEventRecord(e1, P->stream));
    for (int b = 0; b < nblk; ++b) energies[b] = std::numeric_limits<double>::quiet_NaN();
    SFCI_CHECK_HIP(hipMemcpyAsync(energies, energies_d, blocks_run * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    int hstat = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&hstat, status, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    if (T_out)
        SFCI_CHECK_HIP(hipMemcpyAsync(T_out, Td, (size_t)nblk * nL * nL * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    if (S_out)
        SFCI_CHECK_HIP(hipMemcpyAsync(S_out, Sd, (size_t)nblk * nL * nL * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    std::vector<u64> nh((size_t)blocks_run * nL);
    SFCI_CHECK_HIP(hipMemcpyAsync(nh.data(), nnz_hist, nh.size() * sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    u64 emitted = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&emitted, sc + 32, sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    sync(P);
    if (stats) {
        float ms = 0.f;
        SFCI_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        stats->total_ms = ms;
        stats->sigma_ms = tsig.total_ms();
        stats->sigma_calls = sigma_calls;
        u64 en_terms = 0;
        for (u64 x : nh) en_terms += x * tps;
        stats->terms_enumerated = en_terms;
        stats->terms_emitted = emitted;
        stats->blocks_run = blocks_run;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hstat) return (sfci_status)sfci_set_error(SFCI_E_DEVICE, "generalized eigenproblem: S has no positive direction");
    return rc;
    SFCI_GUARD_END
}

sfci_status sfci_sigma_backward(sfci_problem* P, const sfci_svec* v, const sfci_svec* sbar, double* v_bar, double* dh,
                                double* deri) {
    SFCI_GUARD_BEGIN
    if (!P || !v || !sbar) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    if ((v->nnz && (!v->rank || !v->amp)) || (sbar->nnz && (!sbar->rank || !sbar->amp)))
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL input arrays");
    validate_vec(P, v->rank, v->nnz);
    validate_vec(P, sbar->rank, sbar->nnz);
    if (!ensure_dense(P))
        return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "backward needs the dense array (N_det doubles)");
    const int n = P->n;
    const u64 n2 = (u64)n * n, n4 = n2 * n2;
    u64* scal = (u64*)P->ws_lz[0].get(8 * sizeof(u64));
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, scal, (u64)v->nnz);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, P->stream, scal + 1, (u64)sbar->nnz);
    double* raw = (double*)P->ws_red.get((RAW_PAD + n2 + n4) * sizeof(double));
    SigmaLaunch sl{v->rank, v->amp, scal, v->nnz};
    if (!v_bar && v->nnz && sbar->nnz && rowtile_grad_available(P)) {
        // integral gradients only: the target-owned tile passes
        GradJob J{};
        J.P = P;
        J.v = sl;
        J.s_rank = sbar->rank;
        J.s_amp = sbar->amp;
        J.s_nnz = scal + 1;
        J.s_cap = sbar->nnz;
        J.Rh = raw + RAW_PAD;
        J.Rg = raw + RAW_PAD + n2;
        J.dh = dh;
        J.dg = deri;
        J.vt_rank = (u64*)P->ws_list_r.get(v->nnz * sizeof(u64));
        J.vt_amp = (double*)P->ws_list_a.get(v->nnz * sizeof(double));
        J.vt_nnz = scal + 2;
        rowtile_gradients(P->stream, 1, &J, P->grad_ws);
        sync(P);
        return SFCI_OK;
    }
    launch_scatter_set(P, P->d_D, sbar->rank, sbar->amp, scal + 1, std::max<u64>(1, sbar->nnz));
    launch_backward_dense(P, sl, P->d_D, v_bar, dh, deri, raw + RAW_PAD, raw + RAW_PAD + n2);
    launch_scatter_zero(P, P->d_D, sbar->rank, scal + 1, std::max<u64>(1, sbar->nnz));
    sync(P);
    return SFCI_OK;
    SFCI_GUARD_END
}

}  // extern "C"
