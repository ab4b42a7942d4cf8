// Truncation to the M largest amplitudes (Sec. 2.1, Eqs. 10-11; the paper
// sorts the whole intermediate vector, Sec. 3).  Here: an MSD radix select
// over the 128-bit key K = bits(|c|) ++ (N_det - 1 - rank), which orders
// entries by |c| descending and breaks exact ties by rank ascending, followed
// by an order-preserving compaction that writes the kept entries by rank.
// Every pass is a streaming read of the candidates (dense N_det array or a
// rank-sorted list); no sort of the candidates is needed.  Exactly min(M,
// nonzero) entries are kept, unless the problem's tie_band extension is on
// (then entries within a relative 2^-36 of the M-th |c| stay too, at most
// SFCI_TIE_SLACK of them).
#include <algorithm>

#include "../../include/sfci.h"
#include "sfci_internal.h"

namespace {

typedef unsigned __int128 u128;

constexpr int DIG = 11;
constexpr int NBIN = 1 << DIG;
constexpr int CBLOCK = 256;
constexpr int CITEMS = 16;
constexpr u64 CCHUNK = (u64)CBLOCK * CITEMS;

struct Geo {
    int tb;    // total key bits = 63 + rank_bits
    int ndig;  // ceil(tb / 11)
    u64 ndet_m1;
    int rank_bits;
};

__device__ __forceinline__ u128 sel_key(u64 rank, double c, const Geo& g) {
    u64 P = (u64)__double_as_longlong(c) & 0x7FFFFFFFFFFFFFFFull;
    u64 Q = g.ndet_m1 - rank;
    return ((u128)P << g.rank_bits) | (u128)Q;
}

__device__ __forceinline__ int dig_lo(const Geo& g, int L) {
    int lo = g.tb - DIG * (L + 1);
    return lo < 0 ? 0 : lo;
}

struct DenseSrc {
    const double* D;
    u64 n;
    __device__ __forceinline__ u64 size() const { return n; }
    __device__ __forceinline__ void get(u64 i, u64& r, double& c) const { r = i; c = D[i]; }
};

struct ListSrc {
    const u64* r;
    const double* v;
    const u64* cnt;
    __device__ __forceinline__ u64 size() const { return *cnt; }
    __device__ __forceinline__ void get(u64 i, u64& rr, double& c) const { rr = r[i]; c = v[i]; }
};

__device__ __forceinline__ u64 abs_bits(double c) { return (u64)__double_as_longlong(c) & 0x7FFFFFFFFFFFFFFFull; }

__device__ __forceinline__ bool sel_pred(const SelState& st, const Geo& g, u64 r, double c) {
    if (c == 0.0) return false;
    if (st.cand) return abs_bits(c) >= st.cand_bits;
    if (st.take_all) return true;
    if (!st.done || st.level == 0) return false;  // M = 0: nothing is kept
    if (st.use_thr) return abs_bits(c) >= st.thr_bits;
    u128 K = sel_key(r, c, g);
    u128 pre = ((u128)st.pre_hi << 64) | st.pre_lo;
    int sh = dig_lo(g, st.level - 1);
    return (K >> sh) >= pre;
}

__device__ __forceinline__ void sel_init_body(SelState* st, u64 M, int take_all, int take_none) {
    for (int t = threadIdx.x; t < NBIN; t += blockDim.x) st->hist[t] = 0;
    if (threadIdx.x == 0) {
        st->need = M;
        st->pre_hi = 0;
        st->pre_lo = 0;
        st->level = 0;
        st->done = (take_all || take_none) ? 1 : 0;
        st->take_all = take_all;
        st->total = 0;
        st->count_out = 0;
        st->cmin = ~0ull;
        st->thr_bits = 0;
        st->count_thr = 0;
        st->use_thr = 0;
        st->cand = 0;
        st->cand_bits = 0;
        st->count_cand = 0;
    }
}

__global__ void k_sel_init(SelState* st, u64 M, int take_all, int take_none) { sel_init_body(st, M, take_all, take_none); }

// Dense sources: after the level-0 pick (the top key digit is the exponent
// field of |c|), every entry that can still be kept has |c| >= 2^e, e the
// binade of the M-th |c| (with the tie band: >= 2^e (1 - 2^-36)).  Those
// candidates are compacted into a list and the rest of the selection runs on
// the list.
__device__ __forceinline__ void sel_cand_bound_body(SelState* st, int band) {
    if (threadIdx.x != 0) return;
    u64 b;
    if (st->take_all) {
        b = 1;  // every nonzero entry
    } else if (st->level == 0) {
        b = ~0ull;  // M = 0: nothing
    } else {
        const u64 d0 = st->pre_lo & (u64)(NBIN - 1);
        if (d0 == 0) b = 1;
        else if (band) b = abs_bits(__longlong_as_double((long long)(d0 << 52)) * (1.0 - 1.0 / 68719476736.0));
        else b = d0 << 52;
    }
    st->cand_bits = b;
    st->cand = 1;
}

__global__ void k_sel_cand_bound(SelState* st, int band) { sel_cand_bound_body(st, band); }

// Ties at the cut: the smallest |c| among the M selected (exact rule) ...
template <class Src>
__device__ __forceinline__ void sel_min_body(const Src& src, SelState* __restrict__ st, const Geo& g, unsigned bx, unsigned gx) {
    const SelState s = *st;
    if (s.take_all || !s.done || s.level == 0) return;
    const u64 n = src.size();
    u64 m = ~0ull;
    for (u64 i = (u64)bx * blockDim.x + threadIdx.x; i < n; i += (u64)gx * blockDim.x) {
        u64 r;
        double c;
        src.get(i, r, c);
        if (sel_pred(s, g, r, c)) m = min(m, abs_bits(c));
    }
    // one atomic per workgroup: wavefront minima, then the workgroup's
    __shared__ u64 wmin[4];
    for (int off = 32; off >= 1; off >>= 1) m = min(m, (u64)__shfl_xor((long long)m, off));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = min(m, wmin[w]);
        if (m != ~0ull) atomicMin((unsigned long long*)&st->cmin, (unsigned long long)m);
    }
}

template <class Src>
__global__ __launch_bounds__(256) void k_sel_min(Src src, SelState* __restrict__ st, Geo g) {
    sel_min_body(src, st, g, blockIdx.x, gridDim.x);
}

// ... the threshold cmin * (1 - 2^-36) ...
__device__ __forceinline__ void sel_thr_body(SelState* st) {
    if (threadIdx.x != 0 || st->take_all || !st->done || st->level == 0 || st->cmin == ~0ull) return;
    const double thr = __longlong_as_double((long long)st->cmin) * (1.0 - 1.0 / 68719476736.0);
    st->thr_bits = abs_bits(thr);
}

__global__ void k_sel_thr(SelState* st) { sel_thr_body(st); }

// ... how many nonzero candidates reach it ...
template <class Src>
__device__ __forceinline__ void sel_count_thr_body(const Src& src, SelState* __restrict__ st, unsigned bx, unsigned gx) {
    if (st->take_all || !st->done || st->level == 0 || st->cmin == ~0ull) return;
    const u64 thr = st->thr_bits;
    const u64 n = src.size();
    unsigned long long c_ = 0;
    for (u64 i = (u64)bx * blockDim.x + threadIdx.x; i < n; i += (u64)gx * blockDim.x) {
        u64 r;
        double c;
        src.get(i, r, c);
        c_ += (c != 0.0 && abs_bits(c) >= thr) ? 1ull : 0ull;
    }
    __shared__ unsigned long long wsum[4];
    for (int off = 32; off >= 1; off >>= 1) c_ += (unsigned long long)__shfl_xor((long long)c_, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c_;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) c_ += wsum[w];
        if (c_) atomicAdd((unsigned long long*)&st->count_thr, c_);
    }
}

template <class Src>
__global__ __launch_bounds__(256) void k_sel_count_thr(Src src, SelState* __restrict__ st) {
    sel_count_thr_body(src, st, blockIdx.x, gridDim.x);
}

// ... and whether they are kept (at most SFCI_TIE_SLACK beyond M).
__device__ __forceinline__ void sel_mode_body(SelState* st, u64 M) {
    if (threadIdx.x != 0 || st->take_all || !st->done || st->level == 0 || st->cmin == ~0ull) return;
    st->use_thr = (st->count_thr <= M + (u64)SFCI_TIE_SLACK) ? 1 : 0;
}

__global__ void k_sel_mode(SelState* st, u64 M) { sel_mode_body(st, M); }

template <class Src>
__device__ __forceinline__ void sel_hist_body(const Src& src, SelState* __restrict__ st, const Geo& g, int L, unsigned bx, unsigned gx) {
    if (st->done) return;
    __shared__ unsigned int h[NBIN];
    __shared__ unsigned long long blk_total;
    for (int t = threadIdx.x; t < NBIN; t += blockDim.x) h[t] = 0;
    if (threadIdx.x == 0) blk_total = 0;
    __syncthreads();
    const u128 pre = ((u128)st->pre_hi << 64) | st->pre_lo;
    const int lo = dig_lo(g, L);
    const int hi_sh = g.tb - DIG * L;  // bits above the current digit
    const u64 n = src.size();
    u64 my_total = 0;
    for (u64 i = (u64)bx * blockDim.x + threadIdx.x; i < n; i += (u64)gx * blockDim.x) {
        u64 r;
        double c;
        src.get(i, r, c);
        if (c == 0.0) continue;
        ++my_total;
        u128 K = sel_key(r, c, g);
        if (L > 0 && (K >> hi_sh) != pre) continue;
        unsigned d = (unsigned)((K >> lo) & (u128)(NBIN - 1));
        atomicAdd(&h[d], 1u);
    }
    if (L == 0 && my_total) atomicAdd(&blk_total, (unsigned long long)my_total);
    __syncthreads();
    for (int t = threadIdx.x; t < NBIN; t += blockDim.x)
        if (h[t]) atomicAdd((unsigned long long*)&st->hist[t], (unsigned long long)h[t]);
    if (L == 0 && threadIdx.x == 0 && blk_total) atomicAdd((unsigned long long*)&st->total, blk_total);
}

template <class Src>
__global__ __launch_bounds__(256) void k_sel_hist(Src src, SelState* __restrict__ st, Geo g, int L) {
    sel_hist_body(src, st, g, L, blockIdx.x, gridDim.x);
}

// Pick the digit of level L: the largest d >= 1 whose bins d.. hold at least
// `need` entries (else 0), as a block-wide suffix scan over the histogram.
constexpr int PICK_T = 256;
constexpr int PICK_PER = NBIN / PICK_T;
__device__ __forceinline__ void sel_pick_body(SelState* st, const Geo& g, int L, u64 M) {
    __shared__ int s_d;
    __shared__ u64 s_acc;
    const int t = threadIdx.x;
    if (st->done) return;  // uniform: nobody writes it before every thread has read it
    const u64 need = st->need;
    if (L == 0 && st->total <= M) {
        __syncthreads();
        for (int b = t; b < NBIN; b += PICK_T) st->hist[b] = 0;
        if (t == 0) {
            st->take_all = 1;
            st->done = 1;
        }
        return;
    }
    u64 h[PICK_PER];
    u64 mine = 0;
    for (int k = 0; k < PICK_PER; ++k) {
        h[k] = st->hist[t * PICK_PER + k];
        mine += h[k];
    }
    if (t == 0) {
        s_d = 0;
        s_acc = 0;
    }
    // exclusive suffix sum over threads (bins above this thread's block):
    // suffix scan within the wavefront, then the totals of later wavefronts
    __shared__ u64 wtot[PICK_T / 64];
    const int lane = t & 63;
    u64 suf = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const u64 y = (u64)__shfl_down((long long)suf, off);
        if (lane + off < 64) suf += y;
    }
    if (lane == 0) wtot[t >> 6] = suf;
    __syncthreads();
    u64 above = suf - mine;
    for (int w = (t >> 6) + 1; w < PICK_T / 64; ++w) above += wtot[w];
    u64 incl = above;  // entries in bins > current bin
    for (int k = PICK_PER - 1; k >= 0; --k) {
        const int b = t * PICK_PER + k;
        const u64 hi = incl;  // bins > b
        incl += h[k];         // bins >= b
        if (b >= 1 && incl >= need && hi < need) {
            s_d = b;
            s_acc = hi;
        }
    }
    __syncthreads();
    int d = s_d;
    u64 acc = s_acc;
    if (d == 0) {
        // no bin >= 1 reaches `need`: the digit is 0, with everything above it taken
        acc = 0;
        for (int w = 0; w < PICK_T / 64; ++w) acc += wtot[w];
        acc -= st->hist[0];
    }
    const u64 hd = st->hist[d];
    __syncthreads();
    for (int b = t; b < NBIN; b += PICK_T) st->hist[b] = 0;
    if (t == 0) {
        st->need = need - acc;
        const int lo = dig_lo(g, L);
        const int width = (g.tb - DIG * L) - lo;
        u128 pre = ((u128)st->pre_hi << 64) | st->pre_lo;
        pre = (pre << width) | (u128)(unsigned)d;
        st->pre_hi = (u64)(pre >> 64);
        st->pre_lo = (u64)pre;
        st->level = L + 1;
        if (hd == st->need || L == g.ndig - 1) st->done = 1;
    }
}

__global__ __launch_bounds__(PICK_T) void k_sel_pick(SelState* st, Geo g, int L, u64 M) { sel_pick_body(st, g, L, M); }

template <class Src>
__device__ __forceinline__ void compact_count_body(const Src& src, const SelState* __restrict__ st, const Geo& g,
                                                   u64* __restrict__ cnt, unsigned bx) {
    const u64 n = src.size();
    const u64 base = (u64)bx * CCHUNK;
    if (base >= n) {  // grid sized for capacity; chunk beyond the live size
        if (threadIdx.x == 0) cnt[bx] = 0;
        return;
    }
    const SelState s = *st;
    unsigned c = 0;
    for (int k = 0; k < CITEMS; ++k) {
        u64 i = base + (u64)k * CBLOCK + threadIdx.x;
        if (i < n) {
            u64 r;
            double v;
            src.get(i, r, v);
            c += sel_pred(s, g, r, v) ? 1u : 0u;
        }
    }
    __shared__ unsigned sh[CBLOCK / 64];
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int w = 0; w < CBLOCK / 64; ++w) t += sh[w];
        cnt[bx] = t;
    }
}

template <class Src>
__global__ __launch_bounds__(CBLOCK) void k_compact_count(Src src, const SelState* __restrict__ st, Geo g,
                                                          u64* __restrict__ cnt) {
    compact_count_body(src, st, g, cnt, blockIdx.x);
}

template <class Src, bool ZERO>
__device__ __forceinline__ void compact_write_body(const Src& src, const SelState* __restrict__ st, const Geo& g,
                                                   const u64* __restrict__ off, u64* __restrict__ out_r,
                                                   double* __restrict__ out_a, double* __restrict__ Dz, unsigned bx) {
    const u64 n = src.size();
    const u64 base = (u64)bx * CCHUNK;
    if (base >= n) return;
    const SelState s = *st;
    __shared__ unsigned wtot[CBLOCK / 64];
    u64 run = off[bx];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < CITEMS; ++k) {
        u64 i = base + (u64)k * CBLOCK + threadIdx.x;
        u64 r = 0;
        double v = 0.0;
        bool p = false;
        if (i < n) {
            src.get(i, r, v);
            p = sel_pred(s, g, r, v);
            if (ZERO && v != 0.0) Dz[i] = 0.0;
        }
        u64 m = __ballot(p);
        unsigned below = (unsigned)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wave] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned wbase = 0, all = 0;
        for (int w = 0; w < CBLOCK / 64; ++w) {
            if (w < wave) wbase += wtot[w];
            all += wtot[w];
        }
        if (p) {
            u64 at = run + wbase + below;
            out_r[at] = r;
            out_a[at] = v;
        }
        run += all;
        __syncthreads();
    }
}

template <class Src, bool ZERO>
__global__ __launch_bounds__(CBLOCK) void k_compact_write(Src src, const SelState* __restrict__ st, Geo g,
                                                          const u64* __restrict__ off, u64* __restrict__ out_r,
                                                          double* __restrict__ out_a, double* __restrict__ Dz) {
    compact_write_body<Src, ZERO>(src, st, g, off, out_r, out_a, Dz, blockIdx.x);
}

__global__ void k_copy_count(const u64* src, u64* dst) {
    if (threadIdx.x == 0) *dst = *src;
}

// ---- batched selection: each launch serves every instance of a batch
// (blockIdx.y), the same steps as select_topm on a dense source ----
__device__ __forceinline__ Geo bgeo(const BInst& b) {
    Geo g;
    g.rank_bits = b.rank_bits;
    g.tb = 63 + b.rank_bits;
    g.ndig = (g.tb + DIG - 1) / DIG;
    g.ndet_m1 = b.ndet_m1;
    return g;
}
__device__ __forceinline__ u64 bchunks(const BInst& b) { return b.Ndet ? (b.Ndet + CCHUNK - 1) / CCHUNK : 1; }
__device__ __forceinline__ ListSrc blist(const BInst& b) { return ListSrc{b.cr, b.ca, &b.st->count_cand}; }
__device__ __forceinline__ void bout_vec(const BInst& b, int kind, int j, u64*& r, double*& a, u64*& n) {
    if (kind == BOUT_PSI) {
        r = b.psi_r;
        a = b.psi_a;
        n = b.psi_n;
    } else {
        const u64 l = kind == BOUT_W0 ? 0 : (u64)j + 1;
        r = b.Wr + l * b.cap;
        a = b.Wa + l * b.cap;
        n = b.sc + l;
    }
}

// list = 0: the dense pass's state, 1: the candidate list's; M = UINT64_MAX
// keeps every nonzero entry, M = 0 none (the dense pass then lists all, or no,
// nonzero entries as candidates)
__global__ void k_bsel_init(const BInst* __restrict__ B, int list, int all) {
    const BInst& b = B[blockIdx.y];
    const u64 M = all ? UINT64_MAX : b.M;
    sel_init_body(list ? b.st2 : b.st, M, M == UINT64_MAX ? 1 : 0, M == 0 ? 1 : 0);
}

__global__ __launch_bounds__(256) void k_bsel_hist_dense(const BInst* __restrict__ B, int L) {
    const BInst& b = B[blockIdx.y];
    sel_hist_body(DenseSrc{b.D, b.Ndet}, b.st, bgeo(b), L, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_bsel_hist_list(const BInst* __restrict__ B, int L) {
    const BInst& b = B[blockIdx.y];
    sel_hist_body(blist(b), b.st2, bgeo(b), L, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(PICK_T) void k_bsel_pick(const BInst* __restrict__ B, int list, int L) {
    const BInst& b = B[blockIdx.y];
    sel_pick_body(list ? b.st2 : b.st, bgeo(b), L, b.M);
}

__global__ void k_bsel_cand_bound(const BInst* __restrict__ B, int band) { sel_cand_bound_body(B[blockIdx.y].st, band); }

__global__ __launch_bounds__(CBLOCK) void k_bcompact_count_dense(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    if (blockIdx.x >= bchunks(b)) return;  // past this instance's chunks (and its count array)
    compact_count_body(DenseSrc{b.D, b.Ndet}, b.st, bgeo(b), b.cnt, blockIdx.x);
}

template <bool ZERO>
__global__ __launch_bounds__(CBLOCK) void k_bcompact_write_dense(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    if (blockIdx.x >= bchunks(b)) return;
    compact_write_body<DenseSrc, ZERO>(DenseSrc{b.D, b.Ndet}, b.st, bgeo(b), b.cnt, b.cr, b.ca, b.D, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_bsel_min_list(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    sel_min_body(blist(b), b.st2, bgeo(b), blockIdx.x, gridDim.x);
}

__global__ void k_bsel_thr(const BInst* __restrict__ B) { sel_thr_body(B[blockIdx.y].st2); }

__global__ __launch_bounds__(256) void k_bsel_count_thr_list(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    sel_count_thr_body(blist(b), b.st2, blockIdx.x, gridDim.x);
}

__global__ void k_bsel_mode(const BInst* __restrict__ B) { sel_mode_body(B[blockIdx.y].st2, B[blockIdx.y].M); }

__global__ __launch_bounds__(CBLOCK) void k_bcompact_count_list(const BInst* __restrict__ B) {
    const BInst& b = B[blockIdx.y];
    if (blockIdx.x >= bchunks(b)) return;
    compact_count_body(blist(b), b.st2, bgeo(b), b.cnt, blockIdx.x);
}

__global__ void k_bcopy_count(const BInst* __restrict__ B, int kind, int j) {
    const BInst& b = B[blockIdx.y];
    u64* r;
    double* a;
    u64* n;
    bout_vec(b, kind, j, r, a, n);
    if (threadIdx.x == 0) *n = b.st2->count_out;
}

__global__ __launch_bounds__(CBLOCK) void k_bcompact_write_list(const BInst* __restrict__ B, int kind, int j) {
    const BInst& b = B[blockIdx.y];
    if (blockIdx.x >= bchunks(b)) return;
    u64* r;
    double* a;
    u64* n;
    bout_vec(b, kind, j, r, a, n);
    compact_write_body<ListSrc, false>(blist(b), b.st2, bgeo(b), b.cnt, r, a, nullptr, blockIdx.x);
}

Geo make_geo(sfci_problem* P) {
    Geo g;
    g.rank_bits = P->kg.rank_bits;
    g.tb = 63 + g.rank_bits;
    g.ndig = (g.tb + DIG - 1) / DIG;
    g.ndet_m1 = P->kg.ndet_m1;
    return g;
}

template <class Src>
void run_prepare(sfci_problem* P, const Src& src, u64 n_upper, u64 M, u64* out_count_dev, SelState* st = nullptr,
                 u64* cnt_ws = nullptr, u64* bsum_ws = nullptr) {
    // k_sel_min always runs: its cmin (the smallest kept |c|) bounds the list
    // iteration's running candidate list.  The band's three steps only with
    // the extension on.
    Geo g = make_geo(P);
    if (!st) st = (SelState*)P->ws_sel.get(sizeof(SelState));
    int take_all = (M == UINT64_MAX) ? 1 : 0;
    int take_none = (M == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, P->stream, st, M, take_all, take_none);
    unsigned hgrid = (unsigned)std::min<u64>((n_upper + 255) / 256, (u64)P->num_cu * 8);
    if (hgrid < 1) hgrid = 1;
    if (!take_all && !take_none) {
        for (int L = 0; L < g.ndig; ++L) {
            hipLaunchKernelGGL(k_sel_hist<Src>, dim3(hgrid), dim3(256), 0, P->stream, src, st, g, L);
            hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(PICK_T), 0, P->stream, st, g, L, M);
        }
        hipLaunchKernelGGL(k_sel_min<Src>, dim3(hgrid), dim3(256), 0, P->stream, src, st, g);
        if (P->tie_band) {
            hipLaunchKernelGGL(k_sel_thr, dim3(1), dim3(64), 0, P->stream, st);
            hipLaunchKernelGGL(k_sel_count_thr<Src>, dim3(hgrid), dim3(256), 0, P->stream, src, st);
            hipLaunchKernelGGL(k_sel_mode, dim3(1), dim3(64), 0, P->stream, st, M);
        }
    }
    u64 nblk = (n_upper + CCHUNK - 1) / CCHUNK;
    if (nblk < 1) nblk = 1;
    u64* cnt = cnt_ws ? cnt_ws : (u64*)P->ws_cnt.get(nblk * sizeof(u64));
    hipLaunchKernelGGL(k_compact_count<Src>, dim3((unsigned)nblk), dim3(CBLOCK), 0, P->stream, src, st, g, cnt);
    exclusive_scan_u64(P, cnt, cnt, nblk, &st->count_out, bsum_ws);
    if (out_count_dev) hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, P->stream, &st->count_out, out_count_dev);
    SFCI_CHECK_HIP(hipGetLastError());
}

template <class Src>
void run_write(sfci_problem* P, const Src& src, u64 n_upper, u64* out_rank, double* out_amp, bool zero_dense,
               double* Dz, SelState* st = nullptr, u64* cnt_ws = nullptr) {
    Geo g = make_geo(P);
    if (!st) st = (SelState*)P->ws_sel.p;
    u64 nblk = (n_upper + CCHUNK - 1) / CCHUNK;
    if (nblk < 1) nblk = 1;
    u64* cnt = cnt_ws ? cnt_ws : (u64*)P->ws_cnt.p;
    if (zero_dense)
        hipLaunchKernelGGL((k_compact_write<Src, true>), dim3((unsigned)nblk), dim3(CBLOCK), 0, P->stream, src, st, g,
                           cnt, out_rank, out_amp, Dz);
    else
        hipLaunchKernelGGL((k_compact_write<Src, false>), dim3((unsigned)nblk), dim3(CBLOCK), 0, P->stream, src, st,
                           g, cnt, out_rank, out_amp, Dz);
    SFCI_CHECK_HIP(hipGetLastError());
}

}  // namespace

void select_prepare(sfci_problem* P, const CandSrc& src, u64 M, u64* count_dev) {
    if (src.dense) {
        DenseSrc s{src.dense, P->Ndet};
        run_prepare(P, s, P->Ndet, M, count_dev);
    } else {
        ListSrc s{src.lrank, src.lval, src.lcount};
        run_prepare(P, s, src.lcap, M, count_dev);
    }
}

void select_write(sfci_problem* P, const CandSrc& src, u64* out_rank, double* out_amp, bool zero_dense) {
    if (src.dense) {
        DenseSrc s{src.dense, P->Ndet};
        run_write(P, s, P->Ndet, out_rank, out_amp, zero_dense, (double*)src.dense);
    } else {
        ListSrc s{src.lrank, src.lval, src.lcount};
        run_write(P, s, src.lcap, out_rank, out_amp, false, nullptr);
    }
}

u64 select_chunks(u64 n_upper) { return std::max<u64>(1, (n_upper + CCHUNK - 1) / CCHUNK); }

void select_prepare_ws(sfci_problem* P, const CandSrc& src, u64 M, u64* count_dev, const SelWs& ws) {
    ListSrc s{src.lrank, src.lval, src.lcount};
    run_prepare(P, s, src.lcap, M, count_dev, ws.st, ws.cnt, ws.bsum);
}

void select_write_ws(sfci_problem* P, const CandSrc& src, u64* out_rank, double* out_amp, const SelWs& ws) {
    ListSrc s{src.lrank, src.lval, src.lcount};
    run_write(P, s, src.lcap, out_rank, out_amp, false, nullptr, ws.st, ws.cnt);
}

void select_topm(sfci_problem* P, const CandSrc& src, u64 M, u64* out_rank, double* out_amp, u64* out_count_dev,
                 bool zero_dense) {
    if (!src.dense || !zero_dense || M == UINT64_MAX || M == 0) {
        select_prepare(P, src, M, out_count_dev);
        select_write(P, src, out_rank, out_amp, zero_dense);
        return;
    }
    // Dense source, truncation to M: one histogram pass for the binade of the
    // M-th |c|, one pass to count and one to compact the candidates into a
    // rank-ordered list (zeroing the dense array), then the full selection on
    // the list.
    Geo g = make_geo(P);
    SelState* st = (SelState*)P->ws_sel.get(sizeof(SelState));
    SelState* st2 = (SelState*)P->ws_sel2.get(sizeof(SelState));
    u64* cr = (u64*)P->ws_cand_r.get(P->Ndet * sizeof(u64));
    double* ca = (double*)P->ws_cand_a.get(P->Ndet * sizeof(double));
    DenseSrc ds{src.dense, P->Ndet};
    const unsigned hgrid = (unsigned)std::max<u64>(1, std::min<u64>((P->Ndet + 255) / 256, (u64)P->num_cu * 8));
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, P->stream, st, M, 0, 0);
    hipLaunchKernelGGL(k_sel_hist<DenseSrc>, dim3(hgrid), dim3(256), 0, P->stream, ds, st, g, 0);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(PICK_T), 0, P->stream, st, g, 0, M);
    hipLaunchKernelGGL(k_sel_cand_bound, dim3(1), dim3(64), 0, P->stream, st, P->tie_band ? 1 : 0);
    const u64 nblk = std::max<u64>(1, (P->Ndet + CCHUNK - 1) / CCHUNK);
    u64* cnt = (u64*)P->ws_cnt.get(nblk * sizeof(u64));
    hipLaunchKernelGGL(k_compact_count<DenseSrc>, dim3((unsigned)nblk), dim3(CBLOCK), 0, P->stream, ds, st, g, cnt);
    exclusive_scan_u64(P, cnt, cnt, nblk, &st->count_cand);
    hipLaunchKernelGGL((k_compact_write<DenseSrc, true>), dim3((unsigned)nblk), dim3(CBLOCK), 0, P->stream, ds, st, g,
                       cnt, cr, ca, (double*)src.dense);
    SFCI_CHECK_HIP(hipGetLastError());
    ListSrc ls{cr, ca, &st->count_cand};
    run_prepare(P, ls, P->Ndet, M, out_count_dev, st2);
    run_write(P, ls, P->Ndet, out_rank, out_amp, false, nullptr, st2);
}

void bstep_select(hipStream_t st, const BInst* d, int n, int out_kind, int j, u64 max_ndet, int num_cu, int band,
                  int max_ndig, const BScanJob* d_scan_dense, const BScanJob* d_scan_list, int all, bool zero) {
    const unsigned N = (unsigned)n;
    const unsigned hgrid = (unsigned)std::max<u64>(1, std::min<u64>((max_ndet + 255) / 256, (u64)num_cu * 8));
    const u64 nch = select_chunks(max_ndet);
    // the dense pass: the binade of the M-th |c|, then every entry at or above
    // it compacted into the candidate list by rank (the accumulator zeroed)
    hipLaunchKernelGGL(k_bsel_init, dim3(1, N), dim3(256), 0, st, d, 0, all);
    hipLaunchKernelGGL(k_bsel_hist_dense, dim3(hgrid, N), dim3(256), 0, st, d, 0);
    hipLaunchKernelGGL(k_bsel_pick, dim3(1, N), dim3(PICK_T), 0, st, d, 0, 0);
    hipLaunchKernelGGL(k_bsel_cand_bound, dim3(1, N), dim3(64), 0, st, d, band);
    hipLaunchKernelGGL(k_bcompact_count_dense, dim3((unsigned)nch, N), dim3(CBLOCK), 0, st, d);
    bscan_u64(st, d_scan_dense, n, nch);
    if (zero) hipLaunchKernelGGL(k_bcompact_write_dense<true>, dim3((unsigned)nch, N), dim3(CBLOCK), 0, st, d);
    else hipLaunchKernelGGL(k_bcompact_write_dense<false>, dim3((unsigned)nch, N), dim3(CBLOCK), 0, st, d);
    // the full selection on the candidate list
    hipLaunchKernelGGL(k_bsel_init, dim3(1, N), dim3(256), 0, st, d, 1, all);
    for (int L = 0; L < max_ndig; ++L) {
        hipLaunchKernelGGL(k_bsel_hist_list, dim3(hgrid, N), dim3(256), 0, st, d, L);
        hipLaunchKernelGGL(k_bsel_pick, dim3(1, N), dim3(PICK_T), 0, st, d, 1, L);
    }
    hipLaunchKernelGGL(k_bsel_min_list, dim3(hgrid, N), dim3(256), 0, st, d);
    if (band) {
        hipLaunchKernelGGL(k_bsel_thr, dim3(1, N), dim3(64), 0, st, d);
        hipLaunchKernelGGL(k_bsel_count_thr_list, dim3(hgrid, N), dim3(256), 0, st, d);
        hipLaunchKernelGGL(k_bsel_mode, dim3(1, N), dim3(64), 0, st, d);
    }
    hipLaunchKernelGGL(k_bcompact_count_list, dim3((unsigned)nch, N), dim3(CBLOCK), 0, st, d);
    bscan_u64(st, d_scan_list, n, nch);
    hipLaunchKernelGGL(k_bcopy_count, dim3(1, N), dim3(64), 0, st, d, out_kind, j);
    hipLaunchKernelGGL(k_bcompact_write_list, dim3((unsigned)nch, N), dim3(CBLOCK), 0, st, d, out_kind, j);
    SFCI_CHECK_HIP(hipGetLastError());
}
