// The SFCI iteration (Sec. 2.1) without a dense N_det array: every vector is
// a rank-sorted (rank, amplitude) list and sigma = H w_j comes one alpha-rank
// range at a time (Sec. 2.2's buckets, restricted to the spin-up string as in
// Sec. 3) from the sort path, or in fast mode from the tile kernel in row
// slices when the input is large enough (list_sigma_tiles).  This is what runs
// when 8 N_det bytes do not fit the device (12 electrons in 28 orbitals:
// 1.14 TB).
//
// Per sigma application, each pass's reduced entries y (ascending ranks of
// one alpha range) are consumed at once:
//   * T: y is gathered at the entries of every w_l (l <= j) that fall in the
//     range; T_lj is then the same ordered (or tree) dot as with a dense y;
//   * Eq. 10 touches y only on supp(w_j) and supp(w_{j-1}); every other entry
//     of u equals y, is final, and goes to a running candidate list.  Once
//     that list holds more than 2K entries (K = M, or M + SFCI_TIE_SLACK + 1
//     with the tie band) it is cut back to its K best (by |c|, then rank);
//     later entries must beat the K-th |c| to join, since their ranks are
//     larger.  The global K best are always among the kept ones, which is all
//     the truncation needs;
//   * after the last pass, u on supp(w_j) U supp(w_{j-1}) is formed from the
//     gathered y (the same two subtractions, in the same order, as the dense
//     scatters), appended, and the top-M of the whole list is w_{j+1}.
// Psi = sum_j x_j w_j is a stable sort of the concatenated, scaled basis and
// an in-order segmented sum, which adds x_0 w_0, x_1 w_1, ... per rank in the
// order the dense scatters do.  The deterministic option therefore gives the
// dense deterministic iteration's numbers bit for bit.
#include <algorithm>
#include <cstring>
#include <vector>

#include "sfci_internal.h"

namespace {

constexpr int LB = 256;

__device__ __forceinline__ u64 lower_bound_u64(const u64* __restrict__ r, u64 n, u64 key) {
    u64 lo = 0, hi = n;
    while (lo < hi) {
        u64 mid = lo + ((hi - lo) >> 1);
        if (r[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// bounds[2l], bounds[2l+1]: the entries of w_l with rlo <= rank < rhi.
__global__ void k_range_bounds(const u64* __restrict__ Wr, u64 cap, const u64* __restrict__ nnz, int nl, u64 rlo,
                               u64 rhi, u64* __restrict__ bounds) {
    const int l = threadIdx.x;
    if (l >= nl) return;
    const u64* r = Wr + (u64)l * cap;
    const u64 n = nnz[l];
    bounds[2 * l] = lower_bound_u64(r, n, rlo);
    bounds[2 * l + 1] = lower_bound_u64(r, n, rhi);
}

// rowptr[r] = the first entry of a rank-sorted list with rank >= r N_beta,
// r = 0..N_alpha: the entries of alpha row r are [rowptr[r], rowptr[r + 1]).
__global__ void k_row_ptrs(const u64* __restrict__ r, const u64* __restrict__ nnz, u64 Na, u64 Nb,
                           u64* __restrict__ rowptr) {
    const u64 n = *nnz;
    for (u64 row = (u64)blockIdx.x * blockDim.x + threadIdx.x; row <= Na; row += (u64)gridDim.x * blockDim.x)
        rowptr[row] = lower_bound_u64(r, n, row * Nb);
}

// Y[l][i] = y(rank of w_l[i]) for the entries of w_l inside this pass; the
// pass entries hit from w_j and w_{j-1} (l >= mark_from) are marked.
__global__ __launch_bounds__(LB) void k_gather_pass(const u64* __restrict__ Wr, u64 cap, const u64* __restrict__ bounds,
                                                    int mark_from, const u64* __restrict__ pr,
                                                    const double* __restrict__ pa, const u64* __restrict__ pn,
                                                    double* __restrict__ Y, unsigned char* __restrict__ mark) {
    const int l = blockIdx.y;
    const u64 s = bounds[2 * l], e = bounds[2 * l + 1], n = *pn;
    const u64* r = Wr + (u64)l * cap;
    for (u64 i = s + (u64)blockIdx.x * LB + threadIdx.x; i < e; i += (u64)gridDim.x * LB) {
        const u64 key = r[i];
        const u64 pos = lower_bound_u64(pr, n, key);
        if (pos < n && pr[pos] == key) {
            Y[(u64)l * cap + i] = pa[pos];
            if (l >= mark_from) mark[pos] = 1;
        }
    }
}

// Unmarked pass entries with |c| above the running bound join the candidate
// list (positions by wave-aggregated atomics: the list's order is irrelevant,
// selection keys on (|c|, rank) and its output is sorted afterwards).
__global__ __launch_bounds__(LB) void k_append_cands(const u64* __restrict__ pr, const double* __restrict__ pa,
                                                     const u64* __restrict__ pn, const unsigned char* __restrict__ mark,
                                                     const u64* __restrict__ bound_bits, u64* __restrict__ Rr,
                                                     double* __restrict__ Ra, u64* __restrict__ Rn, u64 Rcap,
                                                     int* __restrict__ overflow) {
    const u64 n = *pn, tb = *bound_bits;
    const int lane = threadIdx.x & 63;
    for (u64 base = (u64)blockIdx.x * LB; base < n; base += (u64)gridDim.x * LB) {
        const u64 i = base + threadIdx.x;
        bool p = false;
        double c = 0.0;
        if (i < n) {
            c = pa[i];
            p = !mark[i] && (u64)(__double_as_longlong(c) & 0x7fffffffffffffffll) > tb;
        }
        const u64 m = __ballot(p);
        if (m == 0) continue;
        u64 at0 = 0;
        if (lane == 0) at0 = atomicAdd((unsigned long long*)Rn, (unsigned long long)__popcll(m));
        at0 = (u64)__shfl((long long)at0, 0);
        if (p) {
            const u64 at = at0 + (u64)__popcll(m & ((1ull << lane) - 1ull));
            if (at < Rcap) {
                Rr[at] = pr[i];
                Ra[at] = c;
            } else {
                *overflow = 1;
            }
        }
    }
}

// Eq. 10 on supp(w_{j-1}) (and on the entries of w_j it shares):
//   u = (y - T_jj w_j) - T_{j-1,j} w_{j-1},
// each subtraction rounded as the dense scatters round it.
__global__ __launch_bounds__(LB) void k_fix_prev(const u64* __restrict__ jr, const double* __restrict__ ja,
                                                 const u64* __restrict__ jn, const double* __restrict__ Yj,
                                                 const u64* __restrict__ mr, const double* __restrict__ ma,
                                                 const u64* __restrict__ mn, const double* __restrict__ Ym,
                                                 const double* __restrict__ Tjj, const double* __restrict__ Tmj,
                                                 unsigned char* __restrict__ taken, u64* __restrict__ Rr,
                                                 double* __restrict__ Ra, const u64* __restrict__ Rn, u64 Rcap,
                                                 int* __restrict__ overflow) {
    const u64 nj = *jn, nm = *mn, base = *Rn;
    const double a = *Tjj, b = *Tmj;
    for (u64 i = (u64)blockIdx.x * LB + threadIdx.x; i < nm; i += (u64)gridDim.x * LB) {
        const u64 key = mr[i];
        const u64 pos = lower_bound_u64(jr, nj, key);
        double y;
        if (pos < nj && jr[pos] == key) {
            const double prod = a * ja[pos];
            y = Yj[pos] - prod;
            taken[pos] = 1;
        } else {
            y = Ym[i];
        }
        const double prod = b * ma[i];
        const double u = y - prod;
        if (base + i < Rcap) {
            Rr[base + i] = key;
            Ra[base + i] = u;
        } else {
            *overflow = 1;
        }
    }
}

// ... and on the rest of supp(w_j): u = y - T_jj w_j (entries taken above are
// written as zero, which selection never keeps).
__global__ __launch_bounds__(LB) void k_fix_cur(const u64* __restrict__ jr, const double* __restrict__ ja,
                                                const u64* __restrict__ jn, const double* __restrict__ Yj,
                                                const double* __restrict__ Tjj, const unsigned char* __restrict__ taken,
                                                const u64* __restrict__ mn, u64* __restrict__ Rr,
                                                double* __restrict__ Ra, const u64* __restrict__ Rn, u64 Rcap,
                                                int* __restrict__ overflow) {
    const u64 nj = *jn, base = *Rn + *mn;
    const double a = *Tjj;
    for (u64 i = (u64)blockIdx.x * LB + threadIdx.x; i < nj; i += (u64)gridDim.x * LB) {
        double u = 0.0;
        if (!taken[i]) {
            const double prod = a * ja[i];
            u = Yj[i] - prod;
        }
        if (base + i < Rcap) {
            Rr[base + i] = jr[i];
            Ra[base + i] = u;
        } else {
            *overflow = 1;
        }
    }
}

__global__ void k_add_two(u64* __restrict__ Rn, const u64* __restrict__ a, const u64* __restrict__ b) {
    if (threadIdx.x == 0) *Rn += *a + *b;
}

// After cutting the candidate list back: its length, and the bound a later
// entry must beat (the smallest |c| among the K selected).
__global__ void k_after_cut(const SelState* __restrict__ st, u64* __restrict__ Rn, u64* __restrict__ bound_bits) {
    if (threadIdx.x == 0) {
        *Rn = st->count_out;
        if (!st->take_all && st->cmin != ~0ull) *bound_bits = st->cmin;
    }
}

// offs[j] = nnz[0] + ... + nnz[j-1], offs[nl] = total.
__global__ void k_concat_offsets(const u64* __restrict__ nnz, int nl, u64* __restrict__ offs) {
    if (threadIdx.x == 0) {
        u64 s = 0;
        for (int j = 0; j < nl; ++j) {
            offs[j] = s;
            s += nnz[j];
        }
        offs[nl] = s;
    }
}

// keys/vals[offs[j] + i] = (rank, x_j * a) of w_j's entries, j = blockIdx.y.
__global__ __launch_bounds__(LB) void k_scaled_concat(const u64* __restrict__ Wr, const double* __restrict__ Wa,
                                                      u64 cap, const u64* __restrict__ nnz, const double* __restrict__ x,
                                                      const u64* __restrict__ offs, u64* __restrict__ keys,
                                                      double* __restrict__ vals) {
    const int j = blockIdx.y;
    const u64 n = nnz[j], o = offs[j];
    const double c = x[j];
    for (u64 i = (u64)blockIdx.x * LB + threadIdx.x; i < n; i += (u64)gridDim.x * LB) {
        keys[o + i] = Wr[(u64)j * cap + i];
        vals[o + i] = c * Wa[(u64)j * cap + i];
    }
}

// Order-preserving compaction of a dense slice: block b counts the nonzero
// entries of its DC_CHUNK slots, then writes them (rank = rank_base + slot)
// at out[*out_base + off[b] + ...] in slot order and zeroes the slots read.
constexpr int DC_ITEMS = 16;
constexpr u64 DC_CHUNK = (u64)LB * DC_ITEMS;

__global__ __launch_bounds__(LB) void k_dense_count(const double* __restrict__ D, u64 n, u64* __restrict__ cnt) {
    __shared__ unsigned wsum[LB / 64];
    const u64 base = (u64)blockIdx.x * DC_CHUNK;
    unsigned c = 0;
    for (int k = 0; k < DC_ITEMS; ++k) {
        const u64 i = base + (u64)k * LB + threadIdx.x;
        c += (i < n && D[i] != 0.0) ? 1u : 0u;
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int w = 0; w < LB / 64; ++w) t += wsum[w];
        cnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(LB) void k_dense_write(double* __restrict__ D, u64 n, const u64* __restrict__ off,
                                                    u64 rank_base, const u64* __restrict__ out_base,
                                                    u64* __restrict__ out_r, double* __restrict__ out_a) {
    __shared__ unsigned wtot[LB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 base = (u64)blockIdx.x * DC_CHUNK;
    u64 run = *out_base + off[blockIdx.x];
    for (int k = 0; k < DC_ITEMS; ++k) {
        const u64 i = base + (u64)k * LB + threadIdx.x;
        double v = 0.0;
        if (i < n) v = D[i];
        const bool p = v != 0.0;
        if (p) D[i] = 0.0;
        const u64 m = __ballot(p);
        if (lane == 0) wtot[wave] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned wbase = 0, all = 0;
        for (int w = 0; w < LB / 64; ++w) {
            if (w < wave) wbase += wtot[w];
            all += wtot[w];
        }
        if (p) {
            const u64 at = run + wbase + (u64)__popcll(m & ((1ull << lane) - 1ull));
            out_r[at] = rank_base + i;
            out_a[at] = v;
        }
        run += all;
        __syncthreads();
    }
}

unsigned grid_for(u64 n, unsigned max_blocks = 4096) {
    u64 g = (n + LB - 1) / LB;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (unsigned)g;
}

u64 read_dev(sfci_problem* P, const u64* d) {
    u64 h = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&h, d, sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    return h;
}

// Grow a buffer to hold need bytes, keeping its first keep bytes.
void grow_keep(sfci_problem* P, DevBuf& b, size_t need, size_t keep) {
    if (need <= b.bytes) return;
    DevBuf nb;
    nb.get(std::max(need, b.bytes * 2));
    if (keep && b.p) SFCI_CHECK_HIP(hipMemcpyAsync(nb.p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    b.release();
    b = nb;
}

void check_overflow(sfci_problem* P, const int* flag) {
    int ovf = 0;
    SFCI_CHECK_HIP(hipMemcpyAsync(&ovf, flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    if (ovf) throw sfci_error(-5, "list path: candidate list overflow");
}

// Running top-K candidate list fed by the sort path's passes (also used by a
// single truncated sigma: no basis, nothing excluded).
struct ListCands {
    sfci_problem* P;
    ListWs& ws;
    u64 K;          // keep the K best (UINT64_MAX: keep everything)
    u64 reserve;    // room kept free at the end for the Eq. 10 entries
    u64 n_upper;    // host upper bound on the list length
    u64* Rn;        // device: list length
    u64* bound;     // device: |c| bits a new entry must exceed
    int* overflow;  // device flag

    u64* Rr() { return (u64*)ws.Rr.p; }
    double* Ra() { return (double*)ws.Ra.p; }
    u64 cap() const { return std::min(ws.Rr.bytes / sizeof(u64), ws.Ra.bytes / sizeof(double)); }

    void reset() {
        launch_fill_u64(Rn, 1, 0, P->stream);
        launch_fill_u64(bound, 1, 0, P->stream);
        n_upper = 0;
    }
    void ensure(u64 more) {
        const u64 need = n_upper + more + reserve;
        if (need > cap()) {
            grow_keep(P, ws.Rr, need * sizeof(u64), n_upper * sizeof(u64));
            grow_keep(P, ws.Ra, need * sizeof(double), n_upper * sizeof(double));
        }
    }
    // Cut the list back to its K best once it has grown past 2K.
    void maybe_cut() {
        check_overflow(P, overflow);
        const u64 n = read_dev(P, Rn);
        n_upper = n;  // the actual length (the appends' bound counts every pass entry)
        if (K == UINT64_MAX) return;
        if (n <= 2 * K + SFCI_TIE_SLACK) return;
        u64* r2 = (u64*)ws.R2r.get(n * sizeof(u64));
        double* a2 = (double*)ws.R2a.get(n * sizeof(double));
        CandSrc src{};
        src.lrank = Rr();
        src.lval = Ra();
        src.lcount = Rn;
        src.lcap = n;
        select_prepare(P, src, K, nullptr);
        select_write(P, src, r2, a2, false);
        hipLaunchKernelGGL(k_after_cut, dim3(1), dim3(64), 0, P->stream, (const SelState*)P->ws_sel.p, Rn, bound);
        n_upper = read_dev(P, Rn);
        SFCI_CHECK_HIP(hipMemcpyAsync(Rr(), r2, n_upper * sizeof(u64), hipMemcpyDeviceToDevice, P->stream));
        SFCI_CHECK_HIP(hipMemcpyAsync(Ra(), a2, n_upper * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    }
};

// The sort-path sink: gathers for T, marks, candidate appends.
struct ListPassSink : SortPassSink {
    sfci_problem* P = nullptr;
    ListCands* cands = nullptr;
    bool collect = true;     // append candidates (false: last sigma of a block)
    const u64* Wr = nullptr;
    u64 cap = 0;
    const u64* nnz = nullptr;  // nnz[l] of the basis
    int nl = 0;                // gather for l < nl (= j + 1)
    int mark_from = 0;         // mark hits of w_l, l >= mark_from
    double* Y = nullptr;       // Y[l * cap + i]
    u64* bounds = nullptr;     // 2 * 32 scratch
    u64* pcount = nullptr;     // pass entry count (device)
    u64* distinct = nullptr;   // optional device sum of pass counts
    u64 tuples = 0;

    SortPassOut begin(u64, u64, u64 t) override {
        tuples = t;
        ListWs& ws = P->list_ws;
        ws.pr.get(t * sizeof(u64));
        ws.pa.get(t * sizeof(double));
        launch_fill_u64(pcount, 1, 0, P->stream);
        if (collect) cands->ensure(t);
        return SortPassOut{(u64*)ws.pr.p, (double*)ws.pa.p, t, pcount};
    }
    void end(u64 alo, u64 ahi) override {
        ListWs& ws = P->list_ws;
        unsigned char* mark = (unsigned char*)ws.mark.get(tuples);
        SFCI_CHECK_HIP(hipMemsetAsync(mark, 0, tuples, P->stream));
        if (distinct) launch_add_u64(P, distinct, pcount);
        if (nl > 0) {
            hipLaunchKernelGGL(k_range_bounds, dim3(1), dim3(64), 0, P->stream, Wr, cap, nnz, nl, alo * P->Nb,
                               ahi * P->Nb, bounds);
            hipLaunchKernelGGL(k_gather_pass, dim3(grid_for(cap, 1024), nl), dim3(LB), 0, P->stream, Wr, cap, bounds,
                               mark_from, (const u64*)ws.pr.p, (const double*)ws.pa.p, pcount, Y, mark);
        }
        if (collect) {
            hipLaunchKernelGGL(k_append_cands, dim3(grid_for(tuples)), dim3(LB), 0, P->stream, (const u64*)ws.pr.p,
                               (const double*)ws.pa.p, pcount, mark, cands->bound, cands->Rr(), cands->Ra(),
                               cands->Rn, cands->cap(), cands->overflow);
            cands->n_upper += tuples;
            cands->maybe_cut();
        }
        SFCI_CHECK_HIP(hipGetLastError());
    }
};

// How many of the best entries the running candidate list must keep so that
// the final selection sees all it needs: M (at least 1), and with the tie
// band its reach plus one more, which tells whether the band overflows.
u64 list_keep(const sfci_problem* P, u64 M) {
    if (M == UINT64_MAX) return UINT64_MAX;
    return P->tie_band ? M + SFCI_TIE_SLACK + 1 : std::max<u64>(M, 1);
}

// Selected entries come out in the candidate list's order: sort them by rank.
void sort_by_rank(sfci_problem* P, u64* r, double* a, u64 n) {
    if (n < 2) return;
    ListWs& ws = P->list_ws;
    u64* k2 = (u64*)ws.R2r.get(n * sizeof(u64));
    double* v2 = (double*)ws.R2a.get(n * sizeof(double));
    u64* ko;
    double* vo;
    radix_sort_pairs(P, r, a, k2, v2, n, key_bits(P->Ndet - 1), &ko, &vo);
    if (ko != r) {
        SFCI_CHECK_HIP(hipMemcpyAsync(r, ko, n * sizeof(u64), hipMemcpyDeviceToDevice, P->stream));
        SFCI_CHECK_HIP(hipMemcpyAsync(a, vo, n * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    }
}

}  // namespace

u64 sigma_dense_passes(sfci_problem* P, const SigmaLaunch& v, ListPassSink& sink, u64* emitted_dev, double eps);

u64 sigma_list_topm(sfci_problem* P, const SigmaLaunch& v, u64 M, u64* out_rank, double* out_amp, u64 out_cap,
                    u64* emitted_dev, u64* distinct_host, bool tiles_ok, double eps) {
    ListWs& ws = P->list_ws;
    u64* ls = (u64*)ws.scal.get(128 * sizeof(u64));  // [0] Rn [1] bound [2] pass count [3] overflow [4] distinct [8..) bounds
    launch_fill_u64(ls, 128, 0, P->stream);
    ListCands C{P, ws, list_keep(P, M), 0, 0, ls, ls + 1, (int*)(ls + 3)};
    C.reset();
    ListPassSink sink;
    sink.P = P;
    sink.cands = &C;
    sink.bounds = ls + 8;
    sink.pcount = ls + 2;
    sink.distinct = ls + 4;
    if (tiles_ok && list_sigma_tiles(P, read_dev(P, v.v_nnz)))
        sigma_dense_passes(P, v, sink, emitted_dev, eps);
    else
        sigma_sorted_passes(P, v, sink, emitted_dev, 0, eps);
    check_overflow(P, (const int*)(ls + 3));
    C.n_upper = read_dev(P, C.Rn);
    CandSrc src{};
    src.lrank = C.Rr();
    src.lval = C.Ra();
    src.lcount = C.Rn;
    src.lcap = std::max<u64>(1, C.n_upper);
    u64* cnt = ls + 5;
    select_prepare(P, src, M, cnt);
    const u64 need = read_dev(P, cnt);
    if (distinct_host) *distinct_host = read_dev(P, ls + 4);
    if (need <= out_cap && need > 0) {
        select_write(P, src, out_rank, out_amp, false);
        sort_by_rank(P, out_rank, out_amp, need);
    }
    return need;
}

// Which passes sigma takes in fast mode.  The tile kernel pays a fixed cost
// per (target row, tile) item (its neighbour records) plus ~2.2e-11 s per term;
// the sort path ~4.2e-11 s per term and nothing per item (measured at 28
// orbitals, M = 1e6 and 1e7: the item cost is ~1.2e-7 s).  The tile kernel is
// taken once terms exceed ~5 700 per item.  SFCI_LIST_SIGMA=tile|sort forces
// one kind.
constexpr double kSortTermsPerTileItem = 5700.0;

bool list_sigma_tiles(sfci_problem* P, u64 nnz) {
    if (!rowtile_available(P)) return false;
    if (const char* env = getenv("SFCI_LIST_SIGMA")) {
        if (!strcmp(env, "tile")) return true;
        if (!strcmp(env, "sort")) return false;
    }
    const double terms = (double)nnz * (double)terms_per_source(P->n, P->na, P->nb);
    return terms > kSortTermsPerTileItem * (double)P->Na * (double)rowtile_ntiles(P);
}

// Dense passes: sigma through the target-owned tile kernel, a range of
// target alpha rows at a time.  Fused (the default): every finished tile is
// consumed in the kernel itself (FusedOut: the T gathers, the marks of
// supp(w_j) U supp(w_{j-1}), the candidate appends above the running bound),
// so no N_beta-wide slice is written or re-read; a pass whose appends overflow
// the candidate list is run again after the list has grown.  The first pass
// is small, so that the bound is set before most rows append.
// SFCI_LIST_FUSED=0: each pass fills a zeroed slice of rows x N_beta doubles,
// compacted (rank order, zeroing it) into the sink.
u64 sigma_dense_passes(sfci_problem* P, const SigmaLaunch& v, ListPassSink& sink, u64* emitted_dev, double eps) {
    ListWs& ws = P->list_ws;
    const char* fenv = getenv("SFCI_LIST_FUSED");
    if (!(fenv && fenv[0] == '0')) {
        const RowTileDesc all = rowtile_prepare(P, v, nullptr, (unsigned long long*)emitted_dev, eps, true);
        ListCands& C = *sink.cands;
        const int nl = sink.nl;
        u64* rowptr = (u64*)ws.rowptr.get((size_t)std::max(1, nl) * (P->Na + 1) * sizeof(u64));
        const unsigned gr = (unsigned)std::min<u64>((P->Na + 256) / 256, 16384);
        for (int l = 0; l < nl; ++l)
            hipLaunchKernelGGL(k_row_ptrs, dim3(gr), dim3(256), 0, P->stream, sink.Wr + (size_t)l * sink.cap,
                               sink.nnz + l, P->Na, P->Nb, rowptr + (size_t)l * (P->Na + 1));
        SFCI_CHECK_HIP(hipGetLastError());
        FusedOut h{};
        h.Wr = sink.Wr;
        h.rowptr = rowptr;
        h.Y = sink.Y;
        h.cap = sink.cap;
        h.na_rows = P->Na;
        h.nl = nl;
        h.mark_from = sink.mark_from;
        h.collect = sink.collect ? 1 : 0;
        h.bound = C.bound;
        h.Rn = C.Rn;
        h.overflow = C.overflow;
        h.distinct = sink.distinct;
        FusedOut* d_fo = (FusedOut*)ws.fo.get(sizeof(FusedOut));
        const u64 room = std::max<u64>(1ull << 24, 4 * std::min<u64>(C.K, 1ull << 26));
        u64 lo = 0, passes = 0, extra = 0;
        while (lo < P->Na) {
            const u64 rows = std::max<u64>(1, passes == 0 ? P->Na / 64 : P->Na / 8);
            const u64 hi = std::min<u64>(P->Na, lo + rows);
            if (sink.collect) C.ensure(room + extra);
            h.Rr = C.Rr();
            h.Ra = C.Ra();
            h.Rcap = C.cap();
            const u64 n_before = C.n_upper;
            const u64 dist_before = sink.distinct ? read_dev(P, sink.distinct) : 0;
            SFCI_CHECK_HIP(hipMemcpyAsync(d_fo, &h, sizeof(h), hipMemcpyHostToDevice, P->stream));
            launch_sigma_rowtile_rows_fused(P, all, lo, hi, d_fo);  // synchronises the stream
            if (sink.collect) {
                int ovf = 0;
                SFCI_CHECK_HIP(hipMemcpyAsync(&ovf, C.overflow, sizeof(int), hipMemcpyDeviceToHost, P->stream));
                SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
                if (ovf) {
                    // run the pass again with room for what it appends
                    const u64 need = read_dev(P, C.Rn) - n_before;
                    launch_fill_u64(C.Rn, 1, n_before, P->stream);
                    launch_fill_u64((u64*)C.overflow, 1, 0, P->stream);
                    if (sink.distinct) launch_fill_u64(sink.distinct, 1, dist_before, P->stream);
                    extra = need + need / 4;
                    continue;
                }
                C.n_upper = read_dev(P, C.Rn);
                C.maybe_cut();
            }
            extra = 0;
            ++passes;
            lo = hi;
        }
        return passes;
    }
    size_t freeb = 0, totb = 0;
    SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
    const u64 slice_bytes = std::min<u64>((u64)(freeb + ws.dpass.bytes) / 4, 32ull << 30);
    u64 rows = std::max<u64>(1, std::min<u64>(P->Na, slice_bytes / (8 * P->Nb)));
    if (const char* env = getenv("SFCI_LIST_PASS_ROWS")) {
        long long e = atoll(env);
        if (e > 0) rows = std::min<u64>(rows, (u64)e);
    }
    const u64 slots = rows * P->Nb;
    if (ws.dpass.bytes < slots * sizeof(double)) {
        ws.dpass.get(slots * sizeof(double));
        launch_fill_f64((double*)ws.dpass.p, ws.dpass.bytes / sizeof(double), 0.0, P->stream);
    }
    double* Dp = (double*)ws.dpass.p;
    u64* sc = (u64*)ws.scal2.get(8 * sizeof(u64));  // [0] pass count
    const RowTileDesc all = rowtile_prepare(P, v, Dp, (unsigned long long*)emitted_dev, eps, true);
    u64 passes = 0;
    for (u64 lo = 0; lo < P->Na; lo += rows) {
        const u64 hi = std::min<u64>(P->Na, lo + rows);
        const u64 n = (hi - lo) * P->Nb;
        launch_sigma_rowtile_rows(P, all, lo, hi, Dp);
        const u64 nblk = (n + DC_CHUNK - 1) / DC_CHUNK;
        u64* cnt = (u64*)ws.dcnt.get(nblk * sizeof(u64));
        hipLaunchKernelGGL(k_dense_count, dim3((unsigned)nblk), dim3(LB), 0, P->stream, (const double*)Dp, n, cnt);
        exclusive_scan_u64(P, cnt, cnt, nblk, &sc[0]);
        const u64 total = read_dev(P, &sc[0]);
        ++passes;
        SortPassOut out = sink.begin(lo, hi, std::max<u64>(1, total));
        if (total > out.cap) throw sfci_error(-5, "dense pass: output buffer too small");
        hipLaunchKernelGGL(k_dense_write, dim3((unsigned)nblk), dim3(LB), 0, P->stream, Dp, n, (const u64*)cnt,
                           lo * P->Nb, (const u64*)out.base_dev, out.r, out.a);
        launch_add_u64(P, out.base_dev, &sc[0]);
        SFCI_CHECK_HIP(hipGetLastError());
        sink.end(lo, hi);
    }
    return passes;
}

u64 sigma_list_full(sfci_problem* P, const SigmaLaunch& v, u64* emitted_dev, u64** r, double** a) {
    ListWs& ws = P->list_ws;
    u64* ls = (u64*)ws.scal.get(128 * sizeof(u64));
    launch_fill_u64(ls, 128, 0, P->stream);
    ListCands C{P, ws, UINT64_MAX, 0, 0, ls, ls + 1, (int*)(ls + 3)};
    C.reset();
    ListPassSink sink;
    sink.P = P;
    sink.cands = &C;
    sink.bounds = ls + 8;
    sink.pcount = ls + 2;
    sigma_sorted_passes(P, v, sink, emitted_dev, 0, 0.0);
    check_overflow(P, (const int*)(ls + 3));
    const u64 n = read_dev(P, C.Rn);
    sort_by_rank(P, C.Rr(), C.Ra(), n);
    *r = C.Rr();
    *a = C.Ra();
    return n;
}

void lanczos_list(sfci_problem* P, const sfci_lanczos_opts* o, const ListBasis& Bs, sfci_svec* psi_out,
                  u64* psi_n_out, u64* sigma_calls, EventTimer& tsig, int* blocks_run) {
    const int nL = o->n_L;
    const int nblk = o->n_iter / nL;
    const bool det = o->deterministic != 0;
    const u64 cap = Bs.cap;
    u64* Wr = Bs.Wr;
    double* Wa = Bs.Wa;
    u64* sc = Bs.sc;
    ListWs& ws = P->list_ws;
    u64* ls = (u64*)ws.scal.get(128 * sizeof(u64));
    // ls: [0] Rn [1] bound [2] pass count [3] overflow [8..72) bounds [80] psi count [81] zero [88..) offsets
    launch_fill_u64(ls, 128, 0, P->stream);
    const u64 K = list_keep(P, o->M);
    ListCands C{P, ws, K, 2 * cap, 0, ls, ls + 1, (int*)(ls + 3)};
    double* Y = (double*)ws.yg.get((size_t)nL * cap * sizeof(double));
    unsigned char* taken = (unsigned char*)ws.taken.get(cap);
    auto Wn = [&](int j) { return sc + j; };
    auto Wrj = [&](int j) { return Wr + (size_t)j * cap; };
    auto Waj = [&](int j) { return Wa + (size_t)j * cap; };
    const u64 tup_cap = sort_tuple_cap(P);
    // without the ordered-sum requirement, sigma may go through the tile kernel in row passes
    const bool tiles_ok = !det && rowtile_available(P);

    // Top-M of a candidate list into w_dst (rank order, normalised).
    auto select_into = [&](const CandSrc& src, int dst, bool sorted_src) {
        select_prepare(P, src, o->M, Wn(dst));
        const u64 n = read_dev(P, Wn(dst));
        if (n > cap) throw sfci_error(-4, "list iteration: truncated vector exceeds its capacity");
        select_write(P, src, Wrj(dst), Waj(dst), false);
        if (!sorted_src) sort_by_rank(P, Wrj(dst), Waj(dst), n);
        launch_normalise(P, Waj(dst), Wn(dst), cap, det);
    };

    for (int b = 0; b < nblk; ++b) {
        double* T = Bs.Td + (size_t)b * nL * nL;
        double* S = Bs.Sd + (size_t)b * nL * nL;
        for (int j = 0; j < nL; ++j) {
            SFCI_CHECK_HIP(hipMemcpyAsync(Bs.nnz_hist + (size_t)b * nL + j, Wn(j), sizeof(u64),
                                          hipMemcpyDeviceToDevice, P->stream));
            SigmaLaunch sl{Wrj(j), Waj(j), Wn(j), cap};
            launch_fill_f64(Y, (size_t)(j + 1) * cap, 0.0, P->stream);
            C.reset();
            ListPassSink sink;
            sink.P = P;
            sink.cands = &C;
            sink.collect = (j + 1 < nL);
            sink.Wr = Wr;
            sink.cap = cap;
            sink.nnz = sc;
            sink.nl = j + 1;
            sink.mark_from = std::max(0, j - 1);
            sink.Y = Y;
            sink.bounds = ls + 8;
            sink.pcount = ls + 2;
            const bool dense_passes = tiles_ok && list_sigma_tiles(P, read_dev(P, Wn(j)));
            tsig.begin(P->stream);
            if (dense_passes)
                sigma_dense_passes(P, sl, sink, sc + 32, o->screen_eps);
            else
                sigma_sorted_passes(P, sl, sink, sc + 32, tup_cap, o->screen_eps);
            tsig.end(P->stream);
            ++*sigma_calls;
            for (int l = 0; l <= j; ++l) {
                launch_dot_gathered(P, Waj(l), Wn(l), cap, Y + (size_t)l * cap, T + l * nL + j, T + j * nL + l, det);
                launch_dot_sparse(P, Wrj(l), Waj(l), Wn(l), cap, Wrj(j), Waj(j), Wn(j), S + l * nL + j,
                                  S + j * nL + l, det);
            }
            if (j + 1 < nL) {
                // Eq. 10 on supp(w_j) U supp(w_{j-1}), then the top-M of all candidates
                C.ensure(0);
                SFCI_CHECK_HIP(hipMemsetAsync(taken, 0, cap, P->stream));
                const u64* mn = (j >= 1) ? Wn(j - 1) : ls + 81;
                if (j >= 1)
                    hipLaunchKernelGGL(k_fix_prev, dim3(grid_for(cap)), dim3(LB), 0, P->stream, Wrj(j), Waj(j), Wn(j),
                                       Y + (size_t)j * cap, Wrj(j - 1), Waj(j - 1), Wn(j - 1),
                                       Y + (size_t)(j - 1) * cap, T + j * nL + j, T + (j - 1) * nL + j, taken, C.Rr(),
                                       C.Ra(), C.Rn, C.cap(), C.overflow);
                hipLaunchKernelGGL(k_fix_cur, dim3(grid_for(cap)), dim3(LB), 0, P->stream, Wrj(j), Waj(j), Wn(j),
                                   Y + (size_t)j * cap, T + j * nL + j, taken, mn, C.Rr(), C.Ra(), C.Rn, C.cap(),
                                   C.overflow);
                hipLaunchKernelGGL(k_add_two, dim3(1), dim3(64), 0, P->stream, C.Rn, Wn(j), mn);
                SFCI_CHECK_HIP(hipGetLastError());
                check_overflow(P, C.overflow);
                C.n_upper = read_dev(P, C.Rn);
                CandSrc src{};
                src.lrank = C.Rr();
                src.lval = C.Ra();
                src.lcount = C.Rn;
                src.lcap = std::max<u64>(1, C.n_upper);
                select_into(src, j + 1, false);
            }
        }
        launch_geneig_full(P, nL, T, S, Bs.lam, Bs.xd, Bs.energies_d + b, Bs.status_d);
        // Psi = sum_j x_j w_j: stable sort of the scaled concatenation, in-order sums
        u64* offs = ls + 88;
        hipLaunchKernelGGL(k_concat_offsets, dim3(1), dim3(64), 0, P->stream, sc, nL, offs);
        const u64 tot = read_dev(P, offs + nL);
        const u64 tb = std::max<u64>(1, tot);
        u64* k1 = (u64*)P->ws_tup_k.get(tb * sizeof(u64));
        double* v1 = (double*)P->ws_tup_v.get(tb * sizeof(double));
        u64* k2 = (u64*)P->ws_tup_k2.get(tb * sizeof(u64));
        double* v2 = (double*)P->ws_tup_v2.get(tb * sizeof(double));
        hipLaunchKernelGGL(k_scaled_concat, dim3(grid_for(cap, 1024), nL), dim3(LB), 0, P->stream, Wr, Wa, cap, sc,
                           Bs.xd, offs, k1, v1);
        u64* ks;
        double* vs;
        radix_sort_pairs(P, k1, v1, k2, v2, tot, key_bits(P->Ndet - 1), &ks, &vs);
        u64* pr = (u64*)ws.psi_r.get(tb * sizeof(u64));
        double* pa = (double*)ws.psi_a.get(tb * sizeof(double));
        u64* pn = ls + 80;
        launch_fill_u64(pn, 1, 0, P->stream);
        segmented_sum_append(P, ks, vs, tot, 0, 0.0, pn, tot, pr, pa);
        *blocks_run = b + 1;
        const bool last = (b + 1 == nblk) || halt_after_block(P, o, Bs.energies_d, b);
        if (!last) {
            CandSrc src{};
            src.lrank = pr;
            src.lval = pa;
            src.lcount = pn;
            src.lcap = tb;
            select_into(src, 0, true);
        } else {
            const u64 np = read_dev(P, pn);
            *psi_n_out = np;
            if (psi_out && np <= psi_out->capacity && psi_out->rank && psi_out->amp && np) {
                SFCI_CHECK_HIP(hipMemcpyAsync(psi_out->rank, pr, np * sizeof(u64), hipMemcpyDeviceToDevice, P->stream));
                SFCI_CHECK_HIP(hipMemcpyAsync(psi_out->amp, pa, np * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
            }
            break;
        }
    }
}
