// Second-order Epstein-Nesbet correction of a variational vector Psi: the
// perturbative correction the paper leaves for future work (its comparison
// of the F2 result with ASCI and that method's Epstein-Nesbet correction).
// Standard partitioning with the diagonal of H as the zeroth-order operator:
//   E0 = <Psi|H|Psi> / <Psi|Psi>,
//   E2 = [ sum over k outside supp(Psi) of (H Psi)_k^2 / (E0 - H_kk) ] / <Psi|Psi>.
// The same sigma machinery produces H Psi as a rank-sorted list; one pass
// forms E0's products over supp(Psi) (each Psi rank searched in H Psi), one
// the external terms (each H Psi rank searched in Psi) with H_kk in the
// diagonal element's fixed addition order.  The
// deterministic option (sort-path sigma, every sum strictly in rank order)
// gives the bits of a sequential evaluation; otherwise the dense tile kernel
// and tree reductions.
#include <algorithm>

#include "sfci_internal.h"

namespace {

constexpr int PB = 256;

__device__ __forceinline__ bool find_rank(const u64* __restrict__ r, u64 n, u64 key, u64* pos) {
    u64 lo = 0, hi = n;
    while (lo < hi) {
        const u64 mid = lo + ((hi - lo) >> 1);
        if (r[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    *pos = lo;
    return lo < n && r[lo] == key;
}

// prod[t] = Psi_t * y(rank of Psi_t) (0 where H Psi has no entry): the
// products of <Psi|H Psi> in ascending rank (skipping the zero products of
// entries outside supp(Psi) leaves the ordered sum's bits unchanged)
__global__ __launch_bounds__(PB) void k_pt2_inner(const u64* __restrict__ yr, const double* __restrict__ ya,
                                                  const u64* __restrict__ ny, const u64* __restrict__ pr,
                                                  const double* __restrict__ pa, u64 np, double* __restrict__ prod) {
    const u64 n = *ny;
    for (u64 t = (u64)blockIdx.x * PB + threadIdx.x; t < np; t += (u64)gridDim.x * PB) {
        u64 pos;
        prod[t] = find_rank(yr, n, pr[t], &pos) ? pa[t] * ya[pos] : 0.0;
    }
}

__global__ void k_pt2_e0(const double* __restrict__ num, const double* __restrict__ den, double* __restrict__ e0) {
    if (threadIdx.x == 0) *e0 = *num / *den;
}

// prod[i] = y_i^2 / (E0 - H_kk) outside supp(Psi), else 0; counts the external entries
__global__ __launch_bounds__(PB) void k_pt2_outer(SpaceDev sp, Ints I, const u64* __restrict__ binom,
                                                  const u64* __restrict__ yr, const double* __restrict__ ya,
                                                  const u64* __restrict__ ny, const u64* __restrict__ pr, u64 np,
                                                  const double* __restrict__ e0p, double* __restrict__ prod,
                                                  unsigned long long* __restrict__ n_ext) {
    __shared__ BinomLds B;
    load_binom(B, binom);
    __syncthreads();
    const u64 n = *ny;
    const double E0 = *e0p;
    unsigned long long cnt = 0;
    for (u64 i = (u64)blockIdx.x * PB + threadIdx.x; i < n; i += (u64)gridDim.x * PB) {
        u64 pos;
        const double y = ya[i];
        double t = 0.0;
        if (y != 0.0 && !find_rank(pr, np, yr[i], &pos)) {
            const u64 ra = yr[i] / sp.Nb;
            const u32 A = str_unrank(ra, sp.na, sp.n, B);
            const u32 Bs = str_unrank(yr[i] - ra * sp.Nb, sp.nb, sp.n, B);
            const double hkk = diag_element(I, A, Bs);
            t = (y * y) / (E0 - hkk);
            ++cnt;
        }
        prod[i] = t;
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(n_ext, cnt);
}

unsigned grid_of(u64 n) {
    u64 g = (n + PB - 1) / PB;
    return (unsigned)std::max<u64>(1, std::min<u64>(g, 16384));
}

}  // namespace

// H Psi as a rank-sorted list: the sort path (deterministic, or when the
// N_det array does not fit) or the dense tile kernel compacted in rank order.
u64 sigma_full_list(sfci_problem* P, const SigmaLaunch& sl, bool det, u64* emitted, u64** yr, double** ya,
                    u64* cnt_dev) {
    if (det || !ensure_dense(P)) {
        const u64 n = sigma_list_full(P, sl, emitted, yr, ya);
        launch_set_u64(P, cnt_dev, n);
        return n;
    }
    dense_sigma(P, sl, SFCI_DEDUP_DENSE, (unsigned long long*)emitted);
    CandSrc src{};
    src.dense = P->d_D;
    select_prepare(P, src, UINT64_MAX, cnt_dev);
    u64 n = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&n, cnt_dev, sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    *yr = (u64*)P->ws_list_r.get(std::max<u64>(1, n) * sizeof(u64));
    *ya = (double*)P->ws_list_a.get(std::max<u64>(1, n) * sizeof(double));
    select_write(P, src, *yr, *ya, true);  // rank order; zeroes the accumulator
    return n;
}

// Gradients of E = <Psi|H|Psi>/<Psi|Psi> at fixed Psi (Hellmann-Feynman form):
// the backward of sigma with v = Psi and cotangent Psi/<Psi|Psi>.  sc[0] holds
// nnz(Psi) on the device; sc[5] is scratch for the transposed vector's count.
void energy_gradients_at(sfci_problem* P, const sfci_svec* psi, u64* sc, double* dh, double* deri) {
    const int n = P->n;
    const u64 n2 = (u64)n * n, n4 = n2 * n2;
    double* sbar = (double*)P->ws_cand_a.get(psi->nnz * sizeof(double));
    launch_div_by_sumsq(P, psi->amp, sc, psi->nnz, sbar);
    double* raw = (double*)P->ws_red.get((2048 + n2 + n4) * sizeof(double));
    const SigmaLaunch sl{psi->rank, psi->amp, sc, psi->nnz};
    if (rowtile_grad_available(P)) {
        GradJob J{};
        J.P = P;
        J.v = sl;
        J.s_rank = psi->rank;
        J.s_amp = sbar;
        J.s_nnz = sc;
        J.s_cap = psi->nnz;
        J.Rh = raw + 2048;
        J.Rg = raw + 2048 + n2;
        J.dh = dh;
        J.dg = deri;
        J.vt_rank = (u64*)P->ws_list_r.get(psi->nnz * sizeof(u64));
        J.vt_amp = (double*)P->ws_list_a.get(psi->nnz * sizeof(double));
        J.vt_nnz = sc + 5;
        J.pair_sym = true;  // sbar = Psi / <Psi|Psi>
        rowtile_gradients(P->stream, 1, &J, P->grad_ws);
    } else {
        launch_scatter_set(P, P->d_D, psi->rank, sbar, sc, psi->nnz);
        launch_backward_dense(P, sl, P->d_D, nullptr, dh, deri, raw + 2048, raw + 2048 + n2);
        launch_scatter_zero(P, P->d_D, psi->rank, sc, psi->nnz);
    }
}

extern "C" sfci_status sfci_energy_gradients(sfci_problem* P, const sfci_svec* psi, int32_t deterministic,
                                             double* energy, double* dh, double* deri) {
    try {
        if (!P || !psi || !energy) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
        if (psi->nnz == 0 || !psi->rank || !psi->amp)
            return (sfci_status)sfci_set_error(SFCI_E_ARG, "empty vector");
        validate_vec(P, psi->rank, psi->nnz);
        P->excite_eps = 0.0;  // the energy of the full H
        if ((dh || deri) && !ensure_dense(P))
            return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "gradients need the dense array (N_det doubles)");
        const bool det = deterministic != 0;
        u64* sc = (u64*)P->ws_lz[0].get(16 * sizeof(u64));  // [0] nnz(Psi) [1] emitted [2] |y| [5] scratch
        double* sd = (double*)(sc + 8);                     // [0] num [1] den [2] E
        launch_fill_u64(sc, 16, 0, P->stream);
        launch_set_u64(P, sc, psi->nnz);
        const SigmaLaunch sl{psi->rank, psi->amp, sc, psi->nnz};
        u64* yr;
        double* ya;
        sigma_full_list(P, sl, det, sc + 1, &yr, &ya, sc + 2);
        double* prod = (double*)P->ws_prod.get(std::max<u64>(1, psi->nnz) * sizeof(double));
        hipLaunchKernelGGL(k_pt2_inner, dim3(grid_of(psi->nnz)), dim3(PB), 0, P->stream, yr, ya, sc + 2, psi->rank,
                           psi->amp, (u64)psi->nnz, prod);
        launch_sum(P, prod, sc, psi->nnz, sd + 0, det);
        launch_sumsq(P, psi->amp, sc, psi->nnz, sd + 1, det);
        hipLaunchKernelGGL(k_pt2_e0, dim3(1), dim3(64), 0, P->stream, sd + 0, sd + 1, sd + 2);
        SFCI_CHECK_HIP(hipGetLastError());
        if (dh || deri) energy_gradients_at(P, psi, sc, dh, deri);
        double hd[3];
        SFCI_CHECK_HIP(hipMemcpyAsync(hd, sd, sizeof(hd), hipMemcpyDeviceToHost, P->stream));
        SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
        if (!(hd[1] > 0.0)) return (sfci_status)sfci_set_error(SFCI_E_ARG, "Psi has zero norm");
        *energy = hd[2];
        return SFCI_OK;
    } catch (const sfci_error& e) {
        return (sfci_status)sfci_set_error(e.code, e.msg);
    }
}

extern "C" sfci_status sfci_pt2(sfci_problem* P, const sfci_svec* psi, int32_t deterministic, double* e0,
                                double* e2, uint64_t* n_external) {
    try {
        if (!P || !psi || !e0 || !e2) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
        if (psi->nnz == 0 || !psi->rank || !psi->amp)
            return (sfci_status)sfci_set_error(SFCI_E_ARG, "empty vector");
        validate_vec(P, psi->rank, psi->nnz);
        P->excite_eps = 0.0;  // the correction of the full H
        const bool det = deterministic != 0;
        u64* sc = (u64*)P->ws_lz[0].get(16 * sizeof(u64));  // [0] nnz(Psi) [1] emitted [2] |y| [3] n_ext
        double* sd = (double*)(sc + 8);                     // [0] num [1] den [2] E0 [3] sum
        launch_fill_u64(sc, 16, 0, P->stream);
        launch_set_u64(P, sc, psi->nnz);
        const SigmaLaunch sl{psi->rank, psi->amp, sc, psi->nnz};
        u64* yr;
        double* ya;
        const u64 ny = sigma_full_list(P, sl, det, sc + 1, &yr, &ya, sc + 2);
        double* prod = (double*)P->ws_prod.get(std::max<u64>(std::max<u64>(1, ny), psi->nnz) * sizeof(double));
        hipLaunchKernelGGL(k_pt2_inner, dim3(grid_of(psi->nnz)), dim3(PB), 0, P->stream, yr, ya, sc + 2, psi->rank,
                           psi->amp, (u64)psi->nnz, prod);
        launch_sum(P, prod, sc, psi->nnz, sd + 0, det);
        launch_sumsq(P, psi->amp, sc, psi->nnz, sd + 1, det);
        hipLaunchKernelGGL(k_pt2_e0, dim3(1), dim3(64), 0, P->stream, sd + 0, sd + 1, sd + 2);
        hipLaunchKernelGGL(k_pt2_outer, dim3(grid_of(ny)), dim3(PB), 0, P->stream,
                           SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb}, Ints{P->d_h, P->d_g, P->n}, P->d_binom, yr,
                           ya, sc + 2, psi->rank, (u64)psi->nnz, sd + 2, prod, (unsigned long long*)(sc + 3));
        launch_sum(P, prod, sc + 2, std::max<u64>(1, ny), sd + 3, det);
        SFCI_CHECK_HIP(hipGetLastError());
        double hd[4];
        u64 hc[4];
        SFCI_CHECK_HIP(hipMemcpyAsync(hd, sd, sizeof(hd), hipMemcpyDeviceToHost, P->stream));
        SFCI_CHECK_HIP(hipMemcpyAsync(hc, sc, sizeof(hc), hipMemcpyDeviceToHost, P->stream));
        SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
        if (!(hd[1] > 0.0)) return (sfci_status)sfci_set_error(SFCI_E_ARG, "Psi has zero norm");
        *e0 = hd[2];
        *e2 = hd[3] / hd[1];
        if (n_external) *n_external = hc[3];
        return SFCI_OK;
    } catch (const sfci_error& e) {
        return (sfci_status)sfci_set_error(e.code, e.msg);
    }
}
