// sigma = H v, dense mode, target-owned: one workgroup owns a tile of one
// target alpha row (a contiguous rank range) in LDS and pulls every term that
// lands in it, so no term goes through a global atomic.
//
// For a target alpha string A' the contributing source rows are A' itself,
// its single and its double alpha excitations (Sec. 3: H couples determinants
// up to double excitations).  With the alpha-major rank, a source row is a
// contiguous slice of the sorted input vector, found through per-alpha-rank
// row pointers.  Per source row and tile:
//   * alpha double:   target (A', beta), one term per entry, element constant;
//   * alpha single:   target (A', beta) plus (A', beta') for the beta singles
//                     of each entry -- the alpha-beta doubles, most of the work;
//   * identity:       diagonal, beta singles, beta-beta doubles of each entry.
// The beta singles of every beta string are tabulated once per problem,
// sorted by target rank with per-tile offsets, so a tile visits exactly the
// singles that land in it.  Elements and phases are the same expressions as in
// the source-side enumeration (same integrals, same order of additions).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sfci_internal.h"

namespace {

constexpr int RT_WAVES = 16;
constexpr int RT_BLOCK = 64 * RT_WAVES;
constexpr int RT_PH = 10;  // phase-timing bins

struct RTParams {
    SpaceDev sp;
    Ints I;
    const u64* binom;
    const u64* v_rank;
    const double* v_amp;
    const u32* v_beta;     // beta string of every input entry
    const u32* v_rb;       // beta rank of every input entry (the rank within its alpha row)
    const u64* rowbeg;     // per alpha rank: first input entry of that row
    const u64* rowend;     // per alpha rank: one past the last (== rowbeg when empty)
    const u32* rtb;        // tile-major: rtb[t N_alpha + r], t = 0..ntiles, the first entry of alpha row r
                           // with beta rank >= tile_lo[t]
    const u32* T1;         // beta singles per beta rank, sorted by target: rank | (j n + b) << 21 | par << 31
    const uint16_t* toff;  // per beta rank, ntiles + 1 offsets into its T1 slice
    const u64* tile_lo;    // ntiles + 1 rank boundaries
    int ntiles;
    int sB;                // beta singles per string
    double* D;                   // sigma: the output; gradient passes: the dense cotangent
    unsigned long long* emitted;
    double* Rh;                  // gradient passes: raw dL/dh (n*n) and dL/d(pq|rs) (n^4)
    double* Rg;
    const double* K2;            // n^2: (pp|qq) - (pq|qp)
    const double* TS;            // per T1 entry: h_jb + sum_{k in beta\j} [(jb|kk) - (jk|kb)]
    const double* K4;            // [(i<j), (a<b)] pair-indexed (ia|jb) - (ib|ja), pair (x<y) -> y(y-1)/2 + x
    const u32* T2r;              // per beta rank, its beta-beta doubles: target beta rank
    const double* T2e;           //   and element with both phases, (ia|jb) - (ib|ja) signed,
                                 // grouped by target tile (pair order within a tile); nullptr
                                 // when the table is not built (too large)
    const uint16_t* toff2;       // per beta rank, ntiles + 1 offsets of the tile groups in its T2 slice
    double eps;                  // sigma: screening threshold (Sec. 3), 0 = off
    double eps_x;                // sigma: excitation screen of the doubles' terms, 0 = off
    u64 item_base;               // items of this description start at this global item
    u64 row_base;                // D holds target rows from this alpha rank on
    u32 tile_chunk;              // consecutive tiles of one row per work unit
    u32 short_dbl;               // sigma: alpha doubles with at most this many entries in the tile are added
                                 // while the records are built, longer ones by wavefront in the direct phase
    u32 pair_half;               // gradient passes with sbar a multiple of v: a pair of distinct rows is
                                 // visited once, from the lower source rank, and counted twice
    u32 full_rows;               // sigma into D: rows no term reaches are written as zeros too, so D
                                 // need not be zero before the launch
    u32 gs_min;                  // sigma, alpha-beta doubles: a source row's (ia|jb) slab is staged in LDS
                                 // when it has more than this many entries (else elements are read globally)
    u32 pad_gs;
    // Rows of several tiles (sigma): the alpha-beta doubles' items of every
    // input chunk (up to AB_CHUNK consecutive entries of one alpha row), by
    // target tile: the items of (chunk c, tile t) are ab_it[ab_off[c ntiles
    // + t] .. ab_off[c ntiles + t + 1]), each a beta single of one of the
    // chunk's entries packed as ab_item below.  ab_rowchunk[r]: first chunk of
    // alpha row r.  nullptr where the lists were not built.
    const u32* ab_it;
    const u64* ab_off;
    const u64* ab_rowchunk;
    // sigma: optional per-phase wavefront time (wall clock ticks), RT_PH bins
    // summed over wavefronts: neighbour records, direct targets, alpha-beta
    // units, identity beta-single units, beta-beta units, barrier wait and
    // tile write, other units, work fetch, tile clearing, the wait at the end
    // of the records.  nullptr = off.
    unsigned long long* phase_ns;
    const FusedOut* fo;  // sigma: finished tiles go here instead of D (nullptr: written to D)
};

// One contributing source row of the current (target row, tile).
struct NbrRec {
    u32 As;       // source alpha string
    u32 rAs;      // its rank
    u32 rowb, rowe;
    u32 e0, e1;   // its entries whose beta lies in the tile
    double cst;   // alpha double: the element; alpha single: its alpha part
    uint8_t type, i, a, j, b, par, pad0, pad1;
};

struct WaveScratch {
    uint8_t occ[32], vir[32];
};

// Packed beta single (T1 entry): target beta rank (bits 0..20), j n + b for
// the annihilated j and created b (bits 21..30: the index of (xx|jb) within
// an n x n slab of the integrals), phase (bit 31).
__device__ __forceinline__ u32 t1_rank(u32 t) { return t & 0x1FFFFFu; }
__device__ __forceinline__ u32 t1_jb(u32 t) { return (t >> 21) & 1023u; }
__device__ __forceinline__ int t1_par(u32 t) { return (int)(t >> 31); }

// Input entries per chunk of the alpha-beta item lists (one wavefront's lanes).
constexpr unsigned AB_CHUNK = 64;

// An alpha-beta item: target beta rank within its tile (bits 0..13, tiles
// hold at most 16 384 ranks), j n + b of the beta single (bits 14..23), the
// entry within its chunk (bits 24..29), beta phase (bit 31, as in T1).
__device__ __forceinline__ u32 ab_item(u32 rank_in_tile, u32 te, u32 entry) {
    return rank_in_tile | (((te >> 21) & 1023u) << 14) | (entry << 24) | (te & 0x80000000u);
}

// Entries of the identity row per beta-beta-double and per beta-single work unit.
// Default work per unit of the identity row's beta-beta doubles and beta
// singles (entries per unit); a launch may choose others (autotuning).
constexpr unsigned RT_BB_CHUNK = 4;
constexpr unsigned RT_B1_CHUNK = 16;
// Input entries whose table reads are issued together in the beta-single loop.
constexpr int RT_UNROLL = 4;
// Groups of 64 alpha-beta items whose loads are in flight together (rows of
// several tiles; measured at 26 orbitals, M = 1e7: 4, 6, 8 groups -> 0.346,
// 0.328, 0.330 s per sigma launch).
constexpr int AB_UNROLL = 6;

// Global-memory view of a device pointer (plain global loads, not flat ones).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gl(const T* q) {
    return (const __attribute__((address_space(1))) T*)q;
}

__device__ __forceinline__ u32 rl32(u32 v, int l) { return (u32)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ u64 rl64(u64 v, int l) { return ((u64)rl32((u32)(v >> 32), l) << 32) | rl32((u32)v, l); }
__device__ __forceinline__ double rlf64(double v, int l) { return __longlong_as_double((long long)rl64((u64)__double_as_longlong(v), l)); }

// Direct target (beta unchanged) of entry k of source row r: alpha double
// (constant element), alpha single (alpha part + beta part), or the diagonal.
// itab (LDS): K2[n^2] = (pp|qq) - (pq|qp) and J[n^2] = (pp|qq), hd[32] = h_pp
// (per instance), then EA = sum of h_pp over the item's target alpha string.
// The diagonal is summed in the same order as the reference formula (alpha
// h_pp, beta h_pp, alpha pairs, beta pairs, alpha-beta), so its bits match.
// gq: this wavefront's (ia|qq), q = 0..n-1, for its alpha-single row (or NULL).
__device__ __forceinline__ double direct_element(const RTParams& p, const NbrRec& r, u32 beta, const double* itab,
                                                 const double* gq) {
    if (r.type == 2) return r.cst;
    const int n = p.sp.n;
    if (r.type == 1) {
        double e = r.cst;
        for (u32 m = beta; m; m &= m - 1u) {
            int q = __builtin_ctz(m);
            e += gq ? gq[q] : p.I.G(r.i, r.a, q, q);
        }
        return r.par ? -e : e;
    }
    const double* K2 = itab;
    const double* J = itab + n * n;
    const double* hd = J + n * n;
    const u32 A = r.As;
    double e = hd[32];
    for (u32 m = beta; m; m &= m - 1u) e += hd[__builtin_ctz(m)];
    for (u32 m = A; m; m &= m - 1u) {
        const int q = __builtin_ctz(m);
        for (u32 m2 = m & (m - 1u); m2; m2 &= m2 - 1u) e += K2[q * n + __builtin_ctz(m2)];
    }
    for (u32 m = beta; m; m &= m - 1u) {
        const int q = __builtin_ctz(m);
        for (u32 m2 = m & (m - 1u); m2; m2 &= m2 - 1u) e += K2[q * n + __builtin_ctz(m2)];
    }
    for (u32 m = A; m; m &= m - 1u) {
        const double* Jq = J + __builtin_ctz(m) * n;
        for (u32 m2 = beta; m2; m2 &= m2 - 1u) e += Jq[__builtin_ctz(m2)];
    }
    return e;
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Work modes of the row-tile kernel.
//   RT_SIGMA: sigma = H v into the zero tile, written to D.
//   RT_GRAD_A: gradient of L = sbar^T H v along the integrals for the terms
//     that leave beta unchanged or are alpha-beta doubles: the diagonal, alpha
//     singles, alpha-alpha doubles and alpha-beta doubles.  The tile holds sbar.
//   RT_GRAD_B: the same for the rest (beta singles, beta-beta doubles), run on
//     the spin-exchanged problem with the transposed vectors, where they are
//     alpha singles and alpha-alpha doubles (identity row skipped).
// A beta excitation's phase and element do not involve the alpha string
// beyond its occupations, so exchanging the spins maps those terms exactly.
enum { RT_SIGMA = 0, RT_GRAD_A = 1, RT_GRAD_B = 2 };

// One launch serves one or many problem instances: item i belongs to the
// instance whose [item_prefix[k], item_prefix[k+1]) holds it; a workgroup
// reloads the instance description when consecutive items change instance.
template <int MODE, bool TIMED = false, bool WHOLE = false>
__device__ __forceinline__ void rowtile_body(const RTParams* __restrict__ descs, const u64* __restrict__ item_prefix,
                                             int n_inst, unsigned* __restrict__ counter, void* nbr_scratch,
                                             u64 nbr_cap, unsigned slab_off, unsigned slab_n2, unsigned itab_off,
                                             unsigned b1_chunk, unsigned bb_chunk, unsigned ja_off) {
    constexpr bool GRAD = MODE != RT_SIGMA;
    extern __shared__ double acc[];
    double* const itab = acc + itab_off;  // sigma: per-item element tables
    // sigma, when it fits (ja_off != 0): per item, (jb|kk) for each occupied
    // alpha orbital k of the target string (in ascending order) and every
    // j n + b: the alpha part of the identity row's beta-single elements
    double* const ja = acc + ja_off;
    __shared__ BinomLds sB;
    __shared__ WaveScratch sw[RT_WAVES];
    __shared__ uint8_t occA[32], virA[32];
    __shared__ uint16_t pairNA[SFCI_MAX_PAIRS], pairVA[SFCI_MAX_PAIRS], pairNB[SFCI_MAX_PAIRS], pairVB[SFCI_MAX_PAIRS];
    // the item's records: alpha-single source rows at list[0, s_nlist), the
    // others at list[nbr_cap - s_nlist2, nbr_cap) (phase 3 visits only the former)
    __shared__ unsigned s_nbr, s_nlist, s_nlist2, s_next, s_next2, s_touched, s_idb, s_ide;
    __shared__ u64 s_item, s_left;  // current item (row * ntiles + tile); tiles of its row still to do
    __shared__ int s_inst, s_cur;
    __shared__ u64 s_pfx0, s_pfx1;  // the loaded instance's items [s_pfx0, s_pfx1)
    // sigma with several tiles per row: the row's neighbour records, kept
    // across its tiles (tile-independent parts; entry ranges refreshed per tile)
    __shared__ u64 s_cache_row;
    __shared__ int s_cache_inst;
    // rows of several tiles: the row's records, alpha singles at rowlist[0,
    // s_nrow), the others at rowlist[nbr_cap - s_nrow2, nbr_cap); entry
    // ranges per tile are read when a record is used; the identity row's entries
    __shared__ unsigned s_nrow, s_nrow2;
    __shared__ u32 s_row_idb, s_row_ide;
    __shared__ RTParams p;
    // phase timing (timed build only): per wavefront, RT_PH bins
    __shared__ unsigned long long s_ph[TIMED ? RT_WAVES : 1][TIMED ? RT_PH : 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (TIMED && threadIdx.x < RT_WAVES * RT_PH) s_ph[threadIdx.x / RT_PH][threadIdx.x % RT_PH] = 0;
    u64 t_mark = 0;  // phase timing: the last timestamp of this wavefront
    auto ph_add = [&](bool on, int bin) {
        if (on) {
            const u64 now = wall_clock64();
            if (TIMED && lane == 0 && t_mark) s_ph[TIMED ? wave : 0][TIMED ? bin : 0] += now - t_mark;
            t_mark = now;
        }
    };
    WaveScratch& W = sw[wave];
    NbrRec* list = (NbrRec*)nbr_scratch + (u64)blockIdx.x * 2 * nbr_cap;
    NbrRec* rowlist = list + nbr_cap;
    // append the kept records of a wavefront: alpha singles at the front, the rest from the back
    auto push = [&](const NbrRec& r, bool keep) {
        const bool k1 = keep && r.type == 1;
        const bool k2 = keep && r.type != 1;
        const u64 m1 = __ballot(k1), m2 = __ballot(k2);
        unsigned s1 = 0, s2 = 0;
        if (lane_id() == 0) {
            if (m1) s1 = atomicAdd(&s_nlist, (unsigned)__popcll(m1));
            if (m2) s2 = atomicAdd(&s_nlist2, (unsigned)__popcll(m2));
        }
        s1 = __shfl(s1, 0);
        s2 = __shfl(s2, 0);
        const u64 lt = (1ull << lane_id()) - 1ull;
        if (k1) list[s1 + __popcll(m1 & lt)] = r;
        if (k2) list[nbr_cap - 1 - (s2 + __popcll(m2 & lt))] = r;
    };
    const u64 total_items = item_prefix[n_inst];
    load_binom(sB, descs[0].binom);  // the binomial table is the same for every instance
    // gradient passes: per wavefront, an n^2 slab of (j, b) weights (first
    // pass only) and 32 per-orbital weights, after the tile; zero between uses
    double* const wslab = acc + slab_off + (u32)wave * (slab_n2 + 32);
    double* const wo = wslab + slab_n2;
    if (GRAD)
        for (u32 t = threadIdx.x; t < (u32)RT_WAVES * (slab_n2 + 32); t += RT_BLOCK) acc[slab_off + t] = 0.0;
    if (threadIdx.x == 0) {
        s_cur = -1;
        s_left = 0;
        s_cache_row = ~0ull;
        s_cache_inst = -1;
        s_nrow = 0;
    }
    u64 my_terms = 0;
    u32 wterms = 0;  // terms counted per wavefront (ballot), folded into lane 0's my_terms
    // sigma: an alpha double's entries in the tile, added by the calling
    // thread (element constant); true when it took them (ranges of at most 32)
    auto take_double = [&](const NbrRec& r, u32 tlo_, const RTParams& pp) -> bool {
        if (r.e1 - r.e0 > pp.short_dbl) return false;
        for (u32 k0 = r.e0; k0 < r.e1; k0 += RT_UNROLL) {
            u32 rb[RT_UNROLL];
            double c[RT_UNROLL];
#pragma unroll
            for (int u = 0; u < RT_UNROLL; ++u) {
                const u32 k = min(k0 + (u32)u, r.e1 - 1u);
                rb[u] = pp.v_rb[k];
                c[u] = pp.v_amp[k];
            }
#pragma unroll
            for (int u = 0; u < RT_UNROLL; ++u) {
                if (k0 + (u32)u >= r.e1) continue;
                const double t = r.cst * c[u];
                if (!xscreened(t, pp.eps_x)) {
                    atomicAdd(&acc[rb[u] - tlo_], t);
                    ++my_terms;
                }
            }
        }
        if (r.e1 > r.e0) s_touched = 1;  // terms landed (the item is not skipped)
        return true;
    };

    // The counter hands out target rows (item_prefix counts rows per
    // instance); a workgroup then takes the row's tiles one after another.
    // A workgroup's units come in increasing order, so its instance index
    // never decreases: the search starts at the current one.
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_left > 0) {
                s_item += 1;
                s_left -= 1;
            } else {
                const u64 it = atomicAdd(counter, 1u);
                // a unit of the loaded instance needs no global reads
                const bool cur = s_cur >= 0 && it >= s_pfx0 && it < s_pfx1;
                int k = s_cur > 0 ? s_cur : 0;
                if (!cur && it < total_items)
                    while (k + 1 < n_inst && item_prefix[k + 1] <= it) ++k;
                s_item = ~0ull;
                s_left = 0;
                if (it < total_items) {
                    // unit -> (row, chunk of tile_chunk tiles), chunk-major: units
                    // running together share their tiles (and the tiles' entry
                    // boundaries, rtb's rows for those tiles, stay in cache)
                    const u64 nt = cur ? (u64)p.ntiles : (u64)descs[k].ntiles;
                    const u64 C = cur ? (u64)p.tile_chunk : (u64)descs[k].tile_chunk;
                    const u64 lo = cur ? s_pfx0 : item_prefix[k], hi = cur ? s_pfx1 : item_prefix[k + 1];
                    const u64 nch = (nt + C - 1) / C;
                    const u64 u = it - lo;
                    const u64 rows = (hi - lo) / nch;
                    const u64 ch = u / rows, row = u - ch * rows;
                    s_item = row * nt + ch * C;
                    s_left = min(C, nt - ch * C) - 1;
                }
                s_inst = k;
                s_nrow = 0;  // a new row: its records are built afresh
                s_nrow2 = 0;
                s_row_idb = 0;
                s_row_ide = 0;
                s_cache_row = ~0ull;
            }
            s_nbr = 0;
            s_nlist = 0;
            s_nlist2 = 0;
            s_next = 0;
            s_next2 = 0;
            s_touched = 0;
            s_idb = 0;
            s_ide = 0;
        }
        __syncthreads();
        if (s_item == ~0ull) break;
        if (s_inst != s_cur) {
            // new instance: flush the term count of the previous one, load the description
            if (lane == 0) my_terms += wterms;
            wterms = 0;
            for (int off = 32; off >= 1; off >>= 1) my_terms += __shfl_xor(my_terms, off);
            if (lane == 0 && s_cur >= 0 && p.emitted && my_terms) atomicAdd(p.emitted, (unsigned long long)my_terms);
            my_terms = 0;
            __syncthreads();
            const int words = (int)(sizeof(RTParams) / sizeof(u32));
            for (int t = threadIdx.x; t < words; t += RT_BLOCK) ((u32*)&p)[t] = ((const u32*)&descs[s_inst])[t];
            __syncthreads();
            const int na_ = p.sp.na, nb_ = p.sp.nb, nva_ = p.sp.n - na_, nvb_ = p.sp.n - nb_;
            for (int t = threadIdx.x; t < na_ * (na_ - 1) / 2; t += RT_BLOCK) pairNA[t] = decode_pair(t, na_);
            for (int t = threadIdx.x; t < nva_ * (nva_ - 1) / 2; t += RT_BLOCK) pairVA[t] = decode_pair(t, nva_);
            for (int t = threadIdx.x; t < nb_ * (nb_ - 1) / 2; t += RT_BLOCK) pairNB[t] = decode_pair(t, nb_);
            for (int t = threadIdx.x; t < nvb_ * (nvb_ - 1) / 2; t += RT_BLOCK) pairVB[t] = decode_pair(t, nvb_);
            if (!GRAD) {
                const int n_ = p.sp.n, n2_ = n_ * n_;
                for (int t = threadIdx.x; t < n2_; t += RT_BLOCK) {
                    const int q = t / n_, q2 = t - q * n_;
                    itab[t] = p.K2[t];
                    itab[n2_ + t] = p.I.G(q, q, q2, q2);
                }
                for (int t = threadIdx.x; t < n_; t += RT_BLOCK) itab[2 * n2_ + t] = p.I.H(t, t);
            }
            if (threadIdx.x == 0) {
                s_cur = s_inst;
                s_pfx0 = item_prefix[s_inst];
                s_pfx1 = item_prefix[s_inst + 1];
            }
            __syncthreads();
        }
        const bool timing = TIMED && !GRAD && p.phase_ns != nullptr;
        ph_add(timing, 7);
        const int n = p.sp.n, na = p.sp.na, nb = p.sp.nb;
        const int nva = n - na, nvb = n - nb;
        const u64 Nb = p.sp.Nb;
        const int PA = na * (na - 1) / 2, QA = nva * (nva - 1) / 2;
        const int PB = nb * (nb - 1) / 2, QB = nvb * (nvb - 1) / 2;
        const int sA = na * nva, sBn = p.sB;
        const u64 n_nbr = 1 + (u64)sA + (u64)PA * QA;
        const bool whole_rows = WHOLE || p.ntiles == 1;
        const u64 item = s_item + p.item_base;
        const u64 rAt = WHOLE ? item : item / (u64)p.ntiles;
        const int tile = WHOLE ? 0 : (int)(item - rAt * (u64)p.ntiles);
        const u64 tlo = whole_rows ? 0 : p.tile_lo[tile], thi = whole_rows ? Nb : p.tile_lo[tile + 1];
        const int tsz = (int)(thi - tlo);
        const u32 At = str_unrank_wave(rAt, na, n, sB);
        if (threadIdx.x < (unsigned)n) {
            int q = threadIdx.x;
            u32 below = (1u << q) - 1u;
            if ((At >> q) & 1u) occA[__popc(At & below)] = (uint8_t)q;
            else virA[q - __popc(At & below)] = (uint8_t)q;
        }
        if (GRAD) {
            const double* src = p.D + (rAt - p.row_base) * Nb + tlo;
            for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) acc[x] = src[x];
        } else {
            for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) acc[x] = 0.0;
        }
        __syncthreads();
        ph_add(timing, 8);
        if (!GRAD && ja_off) {
            // read in phase 3, after phase 1's barrier
            const u32 n2 = (u32)n * n;
            for (u32 t = threadIdx.x; t < (u32)na * n2; t += RT_BLOCK) {
                const u32 qi = t / n2, jb = t - qi * n2;
                const u32 kq = occA[qi];
                ja[t] = p.I.g[(jb * (u32)n + kq) * (u32)n + kq];
            }
        }

        // Phase 1: the nonempty source rows, with their entry range in this tile.
        const bool multi = !WHOLE && !GRAD && p.ntiles > 1;
        const bool cached = multi && s_cache_row == rAt && s_cache_inst == s_inst;
        if (cached) {
            // the row's records from its first tile: this tile's entry ranges
            // (alpha doubles with none here are left out)
            if (threadIdx.x == 0) {
                s_idb = s_row_idb;
                s_ide = s_row_ide;
            }
            const unsigned nrow = s_nrow + s_nrow2;
            for (unsigned b0 = 0; b0 < nrow; b0 += RT_BLOCK) {
                const unsigned t = b0 + threadIdx.x;
                NbrRec r;
                r.type = 255;
                if (t < nrow) {
                    r = rowlist[t < s_nrow ? t : nbr_cap - 1 - (t - s_nrow)];
                    const u32* tb = p.rtb + (u64)r.rAs;
                    r.e0 = tb[(u64)tile * p.sp.Na];
                    r.e1 = tb[(u64)(tile + 1) * p.sp.Na];
                    // an alpha double's few entries here are added at once (no list entry)
                    if (r.type == 2 && (r.e1 <= r.e0 || take_double(r, (u32)tlo, p))) r.type = 255;
                }
                push(r, r.type != 255);
            }
        }
        for (;;) {
            if (cached) break;
            unsigned base = 0;
            if (lane == 0) base = atomicAdd(&s_nbr, 64u);
            base = __shfl(base, 0);
            if ((u64)base >= n_nbr) break;
            const u64 idx = (u64)base + lane;
            NbrRec r;
            r.type = 255;
            bool row_ok = false;  // nonempty source row with a usable element (tile aside)
            if (idx < n_nbr) {
                int i = 0, a = 0, j = 0, b = 0, type;
                u32 As;
                if (idx == 0) {
                    type = 0;
                    As = At;
                } else if (idx <= (u64)sA) {
                    int s = (int)idx - 1;
                    a = occA[s / nva];  // created in the target
                    i = virA[s % nva];  // annihilated from the source
                    As = At ^ (1u << a) ^ (1u << i);
                    type = 1;
                } else {
                    u64 d = idx - 1 - sA;
                    int po = (int)(d / (u64)QA), pv = (int)(d - (u64)po * QA);
                    unsigned pa = pairNA[po], pvv = pairVA[pv];
                    a = occA[pa & 255];
                    b = occA[pa >> 8];
                    i = virA[pvv & 255];
                    j = virA[pvv >> 8];
                    As = At ^ (1u << a) ^ (1u << b) ^ (1u << i) ^ (1u << j);
                    type = 2;
                }
                const u64 rAs = str_rank(As, sB);
                // an alpha double's integrals are read together with the row bounds
                const double g2 = (!GRAD && type == 2) ? p.I.G(i, a, j, b) - p.I.G(i, b, j, a) : 0.0;
                // gradient with sbar proportional to v: sbar(J) v(I) = sbar(I) v(J), so of a pair of
                // rows only the visit from the lower source rank is made (and weighted twice)
                const bool mirror = GRAD && p.pair_half && type != 0 && rAs > rAt;
                u64 rb = 0, re = 0;
                if (!mirror) {
                    rb = p.rowbeg[rAs];
                    re = p.rowend[rAs];
                }
                if (type == 0) {
                    s_idb = (u32)rb;  // the identity row: all its entries feed the beta-beta doubles
                    s_ide = (u32)re;
                    s_row_idb = (u32)rb;
                    s_row_ide = (u32)re;
                }
                if (re > rb) {
                    row_ok = true;
                    r.As = As; r.rAs = (u32)rAs; r.rowb = (u32)rb; r.rowe = (u32)re;
                    if (whole_rows) {
                        r.e0 = (u32)rb;  // one tile: the whole row
                        r.e1 = (u32)re;
                    } else {
                        const u32* tb = p.rtb + (u64)rAs;
                        r.e0 = tb[(u64)tile * p.sp.Na];
                        r.e1 = tb[(u64)(tile + 1) * p.sp.Na];
                    }
                    r.i = (uint8_t)i; r.a = (uint8_t)a; r.j = (uint8_t)j; r.b = (uint8_t)b;
                    r.type = (uint8_t)type;
                    r.par = 0;
                    r.cst = 0.0;
                    if (type == 2) {
                        // alpha double, source-occupied i<j -> source-virtual a<b (pairing i->a, j->b)
                        const u32 mid = As ^ (1u << i) ^ (1u << a);
                        const int par = between_parity(As, i, a) ^ between_parity(mid, j, b);
                        r.par = (uint8_t)par;
                        if (!GRAD) {
                            double e = g2;
                            if (par) e = -e;
                            r.cst = e;
                            if (e == 0.0) {
                                r.type = 255;
                                row_ok = false;
                            }
                        }
                        // (a gradient pass keeps zero elements: their derivative need not vanish)
                        if (r.e1 <= r.e0) r.type = 255;
                        else if (!GRAD && r.type == 2 && take_double(r, (u32)tlo, p)) r.type = 255;
                    } else if (type == 1) {
                        if (!GRAD) {
                            double e = p.I.H(i, a);
                            for (u32 m = As & ~(1u << i); m; m &= m - 1u) {
                                int k = __builtin_ctz(m);
                                e += (p.I.G(i, a, k, k) - p.I.G(i, k, k, a));
                            }
                            r.cst = e;
                        }
                        r.par = (uint8_t)between_parity(As, i, a);
                        if (MODE == RT_GRAD_B && r.e1 <= r.e0) r.type = 255;  // direct targets only
                    } else if (GRAD) {
                        // identity row: the diagonal in the first pass, nothing in the second
                        if (MODE == RT_GRAD_B || r.e1 <= r.e0) r.type = 255;
                    }
                }
            }
            if (multi) {
                // keep every record that survives the row-level filters for all the row's
                // tiles: alpha singles at the front, the others from the back
                const bool k1 = row_ok && r.type == 1, k2 = row_ok && r.type != 1;
                const u64 m1 = __ballot(k1), m2 = __ballot(k2);
                unsigned s1 = 0, s2 = 0;
                if (lane == 0) {
                    if (m1) s1 = atomicAdd(&s_nrow, (unsigned)__popcll(m1));
                    if (m2) s2 = atomicAdd(&s_nrow2, (unsigned)__popcll(m2));
                }
                s1 = __shfl(s1, 0);
                s2 = __shfl(s2, 0);
                const u64 lt = (1ull << lane) - 1ull;
                NbrRec rr = r;
                if (rr.type == 255) rr.type = 2;  // an alpha double with no entries in this tile
                if (k1) rowlist[s1 + __popcll(m1 & lt)] = rr;
                if (k2) rowlist[nbr_cap - 1 - (s2 + __popcll(m2 & lt))] = rr;
            }
            push(r, r.type != 255);
        }
        if (multi && !cached) {
            __syncthreads();
            if (threadIdx.x == 0) {
                s_cache_row = rAt;
                s_cache_inst = s_inst;
            }
        }
        if (!GRAD && threadIdx.x == RT_BLOCK - 1) {
            // the alpha h_pp of the diagonal, summed from zero in ascending order
            double x = 0.0;
            for (u32 m = At; m; m &= m - 1u) x += p.I.H(__builtin_ctz(m), __builtin_ctz(m));
            itab[2 * n * n + 32] = x;
        }
        ph_add(timing, 0);
        __syncthreads();
        ph_add(timing, 9);
        const unsigned n1 = s_nlist, nlist = s_nlist + s_nlist2;
        auto rec = [&](unsigned li) -> const NbrRec& { return list[li < n1 ? li : nbr_cap - 1 - (li - n1)]; };
        if (nlist == 0 && !s_touched) {
            // nothing lands here: D keeps its zeros, or gets them (full_rows)
            if (!GRAD && p.full_rows && !p.fo) {
                double* dst = p.D + (rAt - p.row_base) * Nb + tlo;
                for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) dst[x] = 0.0;
            }
            continue;
        }
        if (threadIdx.x == 0) s_touched = 1;

        // Phase 2: direct targets (beta unchanged).  Short ranges: one thread
        // per source row; long ranges, and alpha-single rows of more than a
        // few entries (each entry's element adds (ia|qq) over its beta
        // orbitals, staged in LDS per wavefront there): one wavefront, lanes
        // over the entries.
        auto by_wave = [&](const NbrRec& r) {
            return r.e1 - r.e0 > (r.type == 1 ? 4u : (r.type == 2 ? p.short_dbl : 32u));
        };
        if (!GRAD) {
            for (unsigned li = threadIdx.x; li < nlist; li += RT_BLOCK) {
                const NbrRec r = rec(li);
                if (by_wave(r)) continue;
                // RT_UNROLL entries at a time, their loads in flight together
                for (u32 k0 = r.e0; k0 < r.e1; k0 += RT_UNROLL) {
                    u32 rb[RT_UNROLL], bt[RT_UNROLL];
                    double c[RT_UNROLL];
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        const u32 k = min(k0 + (u32)u, r.e1 - 1u);
                        rb[u] = p.v_rb[k];
                        c[u] = p.v_amp[k];
                        bt[u] = (r.type == 2) ? 0u : p.v_beta[k];
                    }
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        if (k0 + (u32)u >= r.e1) continue;
                        const double e = (r.type == 2) ? r.cst : direct_element(p, r, bt[u], itab, nullptr);
                        const double t = e * c[u];
                        if (e != 0.0 && !(r.type == 2 && xscreened(t, p.eps_x))) {
                            atomicAdd(&acc[rb[u] - tlo], t);
                            ++my_terms;
                        }
                    }
                }
            }
            // Long rows by wavefront, DB records at a time.  The alpha doubles
            // (constant element) of a batch are one stream of entries: lanes over
            // their concatenated entry ranges, RT_UNROLL groups of 64 loads in
            // flight across row boundaries.  The other long rows (the diagonal's,
            // alpha singles') one at a time, alpha singles with (ia|qq) staged.
            constexpr int DB = 8;
            // a batch's records are read while the previous batch streams
            auto claim = [&]() {
                unsigned b = 0;
                if (lane == 0) b = atomicAdd(&s_next2, (unsigned)DB);
                return (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl((int)b, 0));
            };
            unsigned nbase = claim();
            u32 n_e0 = 0, n_e1 = 0, n_type = 255;
            double n_cst = 0.0;
            auto fetch = [&]() {
                n_type = 255;
                if (lane < DB && nbase + (unsigned)lane < nlist) {
                    const NbrRec& r = rec(nbase + (unsigned)lane);
                    n_e0 = r.e0;
                    n_e1 = r.e1;
                    n_type = r.type;
                    n_cst = r.cst;
                }
            };
            if (nbase < nlist) fetch();
            for (;;) {
                const unsigned base = nbase;
                if (base >= nlist) break;
                u32 d_e0 = 0, d_len = 0;
                double d_cst = 0.0;
                bool other = false;
                if (n_type != 255) {
                    NbrRec r;
                    r.e0 = n_e0;
                    r.e1 = n_e1;
                    r.type = (uint8_t)n_type;
                    if (by_wave(r)) {
                        if (r.type == 2) {
                            d_e0 = n_e0;
                            d_len = n_e1 - n_e0;
                            d_cst = n_cst;
                        } else {
                            other = true;
                        }
                    }
                }
                nbase = claim();
                if (nbase < nlist) fetch();
                for (u64 om = __ballot(other); om; om &= om - 1) {
                    const unsigned j = (unsigned)(__ffsll((long long)om) - 1);
                    const NbrRec r = rec(base + j);
                    const double* gq = nullptr;
                    if (r.type == 1) {
                        // this row's (ia|qq), q = 0..n-1
                        wave_sync();
                        if (lane < n) wo[lane] = p.I.G(r.i, r.a, lane, lane);
                        wave_sync();
                        gq = wo;
                    }
                    // RT_UNROLL chunks of 64 entries at a time, their loads in flight together
                    for (u32 k0 = r.e0; k0 < r.e1; k0 += 64 * RT_UNROLL) {
                        u32 rb[RT_UNROLL], bt[RT_UNROLL];
                        double c[RT_UNROLL];
#pragma unroll
                        for (int u = 0; u < RT_UNROLL; ++u) {
                            const u32 k = k0 + (u32)u * 64 + lane;
                            rb[u] = 0;
                            bt[u] = 0;
                            c[u] = 0.0;
                            if (k < r.e1) {
                                rb[u] = p.v_rb[k];
                                c[u] = p.v_amp[k];
                                bt[u] = p.v_beta[k];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < RT_UNROLL; ++u) {
                            if (k0 + (u32)u * 64 + lane >= r.e1) continue;
                            const double e = direct_element(p, r, bt[u], itab, gq);
                            const double t = e * c[u];
                            if (e != 0.0) {
                                atomicAdd(&acc[rb[u] - tlo], t);
                                ++my_terms;
                            }
                        }
                    }
                }
                // exclusive prefix of the alpha doubles' lengths over lanes 0..DB-1
                u32 pfx = 0, total = 0;
                for (int j = 0; j < DB; ++j) {
                    const u32 lj = rl32(d_len, j);
                    if (lane == j) pfx = total;
                    total += lj;
                }
                for (u32 q0 = 0; q0 < total; q0 += 64 * RT_UNROLL) {
                    u32 rb[RT_UNROLL];
                    double c[RT_UNROLL], e[RT_UNROLL];
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        const u32 q = q0 + (u32)u * 64 + lane;
                        // the row of stream position q: the last of the batch starting at or before it
                        int j = 0;
                        for (int jj = 1; jj < DB; ++jj) j += (rl32(pfx, jj) <= q) ? 1 : 0;
                        const u32 k = (u32)__shfl((int)d_e0, j) + (q - (u32)__shfl((int)pfx, j));
                        e[u] = __shfl(d_cst, j);
                        rb[u] = 0;
                        c[u] = 0.0;
                        if (q < total) {
                            rb[u] = p.v_rb[k];
                            c[u] = p.v_amp[k];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        if (q0 + (u32)u * 64 + lane >= total) continue;
                        const double t = e[u] * c[u];
                        if (!xscreened(t, p.eps_x)) {
                            atomicAdd(&acc[rb[u] - tlo], t);
                            ++my_terms;
                        }
                    }
                }
            }
        } else {
            // Gradient: every direct term of a source row shares the row's
            // integrals up to the beta occupations, so the row reduces to
            //   W = sum_k sbar(target_k) v_k,  O_q = same over entries with q occupied,
            // and (identity row) P_pq over entries with p and q occupied.
            const u32 n2 = (u32)n * n;
            auto gi = [&](int a_, int b_, int c_, int d_) { return (((u32)a_ * n + b_) * n + c_) * n + d_; };
            for (unsigned li = threadIdx.x; li < nlist; li += RT_BLOCK) {
                const NbrRec r = rec(li);
                if (r.type != 2 || r.e1 - r.e0 > 32) continue;
                double w = 0.0;
                // RT_UNROLL entries' loads in flight together; the sum keeps entry order
                for (u32 k0 = r.e0; k0 < r.e1; k0 += RT_UNROLL) {
                    u32 rb[RT_UNROLL];
                    double c[RT_UNROLL];
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        const u32 k = min(k0 + (u32)u, r.e1 - 1u);
                        rb[u] = p.v_rb[k];
                        c[u] = p.v_amp[k];
                    }
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u)
                        if (k0 + (u32)u < r.e1) w += acc[rb[u] - tlo] * c[u];
                }
                if (w != 0.0) {
                    if (r.par) w = -w;
                    if (p.pair_half) w *= 2.0;
                    atomicAdd(p.Rg + gi(r.i, r.a, r.j, r.b), w);
                    atomicAdd(p.Rg + gi(r.i, r.b, r.j, r.a), -w);
                }
            }
            double* slab = wslab;
            for (;;) {
                unsigned li = 0;
                if (lane == 0) li = atomicAdd(&s_next2, 1u);
                li = __shfl(li, 0);
                if (li >= nlist) break;
                const NbrRec r = rec(li);
                const int T = r.type;
                if (T == 2 && r.e1 - r.e0 <= 32) continue;
                if (r.e1 <= r.e0) continue;
                double wl = 0.0;
                // RT_UNROLL chunks of 64 entries: their loads in flight together
                for (u32 k0 = r.e0; k0 < r.e1; k0 += 64 * RT_UNROLL) {
                    u32 rb[RT_UNROLL], bt[RT_UNROLL];
                    double c[RT_UNROLL];
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        const u32 k = k0 + (u32)u * 64 + lane;
                        rb[u] = 0;
                        bt[u] = 0;
                        c[u] = 0.0;
                        if (k < r.e1) {
                            rb[u] = p.v_rb[k];
                            c[u] = p.v_amp[k];
                            if (T != 2) bt[u] = p.v_beta[k];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < RT_UNROLL; ++u) {
                        if (k0 + (u32)u * 64 + lane >= r.e1) continue;
                        const double sb = acc[rb[u] - tlo];
                        if (sb == 0.0) continue;
                        const double w = sb * c[u];
                        wl += w;
                        if (T != 2) {
                            for (u32 m = bt[u]; m; m &= m - 1u) {
                                const int q = __builtin_ctz(m);
                                atomicAdd(&wo[q], w);
                                if (T == 0)
                                    for (u32 m2 = m & (m - 1u); m2; m2 &= m2 - 1u)
                                        atomicAdd(&slab[q * n + __builtin_ctz(m2)], w);
                            }
                        }
                    }
                }
                // a pair of distinct rows counted twice (pair_half); the identity row once
                const double pf = (p.pair_half && T != 0) ? 2.0 : 1.0;
                const double Wr = wave_sum(wl) * pf;
                wave_sync();
                if (T == 2) {
                    if (lane == 0 && Wr != 0.0) {
                        const double w = r.par ? -Wr : Wr;
                        atomicAdd(p.Rg + gi(r.i, r.a, r.j, r.b), w);
                        atomicAdd(p.Rg + gi(r.i, r.b, r.j, r.a), -w);
                    }
                } else if (T == 1) {
                    // alpha single i -> a: h_ia + sum_{k in As\i} [(ia|kk) - (ik|ka)] + sum_{q in beta} (ia|qq)
                    const int i = r.i, a = r.a;
                    const double sg = r.par ? -1.0 : 1.0;
                    if (lane < n) {
                        const int q = lane;
                        const bool spect = q != i && ((r.As >> q) & 1u);
                        const double add = sg * (wo[q] * pf + (spect ? Wr : 0.0));
                        wo[q] = 0.0;
                        if (add != 0.0) atomicAdd(p.Rg + gi(i, a, q, q), add);
                        if (spect && Wr != 0.0) atomicAdd(p.Rg + gi(i, q, q, a), -sg * Wr);
                    }
                    if (lane == 0 && Wr != 0.0) atomicAdd(p.Rh + i * n + a, sg * Wr);
                } else {
                    // diagonal: sum_{p in A, B} h_pp + same-spin pairs [(pp|qq) - (pq|qp)] + alpha-beta (pp|qq)
                    const u32 A = r.As;
                    if (lane < n) {
                        const int q = lane;
                        const double oq = wo[q];
                        wo[q] = 0.0;
                        const double dh = oq + (((A >> q) & 1u) ? Wr : 0.0);
                        if (dh != 0.0) atomicAdd(p.Rh + q * n + q, dh);
                        if (oq != 0.0)
                            for (u32 m = A; m; m &= m - 1u) atomicAdd(p.Rg + gi(__builtin_ctz(m), __builtin_ctz(m), q, q), oq);
                        if (((A >> q) & 1u) && Wr != 0.0)
                            for (u32 m = A & ~((2u << q) - 1u); m; m &= m - 1u) {
                                const int q2 = __builtin_ctz(m);
                                atomicAdd(p.Rg + gi(q, q, q2, q2), Wr);
                                atomicAdd(p.Rg + gi(q, q2, q2, q), -Wr);
                            }
                    }
                    for (u32 t = lane; t < n2; t += 64) {
                        const double v = slab[t];
                        if (v != 0.0) {
                            const int q = (int)(t / n), q2 = (int)(t - (u32)q * n);
                            atomicAdd(p.Rg + gi(q, q, q2, q2), v);
                            atomicAdd(p.Rg + gi(q, q2, q2, q), -v);
                            slab[t] = 0.0;
                        }
                    }
                }
                wave_sync();
            }
        }

        ph_add(timing, 1);
        // Phase 3: beta singles of the identity and alpha-single source rows
        // (the alpha-beta doubles), one list row per work unit; then the
        // identity row's beta-beta doubles, bb_chunk entries per unit, so
        // that every wavefront shares the largest single-row job.
        const u32 idb = s_idb, ide = s_ide;
        const unsigned n_b1 = (!GRAD && ide > idb) ? (ide - idb + b1_chunk - 1) / b1_chunk : 0u;
        const unsigned n_bb = (!GRAD && PB > 0 && QB > 0) ? (ide - idb + bb_chunk - 1) / bb_chunk : 0u;
        const unsigned n_units = (MODE == RT_GRAD_B) ? 0u : n1 + n_b1 + n_bb;
        const int top_lo = (nb > 0) ? 31 - __clz((int)str_unrank_wave(tlo, nb, n, sB)) : 0;
        const int top_hi = (nb > 0) ? 31 - __clz((int)str_unrank_wave(thi - 1, nb, n, sB)) : 0;
        int ph_bin = 6;
        for (;;) {
            unsigned li = 0;
            if (lane == 0) li = atomicAdd(&s_next, 1u);
            li = __shfl(li, 0);
            ph_add(timing, ph_bin);
            if (li >= n_units) break;
            if (timing) ph_bin = (li >= n1 + n_b1) ? 4 : (li >= n1) ? 3 : 2;
            if (!GRAD && li >= n1 + n_b1) {
                // beta-beta doubles of identity-row entries [k0, k1)
                const u32 k0 = idb + (li - n1 - n_b1) * bb_chunk;
                const u32 k1 = min(ide, k0 + bb_chunk);
                const auto K4g = gl(p.K4);
                const int np2 = n * (n - 1) / 2;
                if (p.T2r) {
                    // tabulated target rank and signed element per double, the
                    // entry's doubles that land in this tile only; RT_UNROLL
                    // groups of 64 doubles have their loads in flight
                    const auto T2rg = gl(p.T2r);
                    const auto T2eg = gl(p.T2e);
                    const u32 tot = (u32)(PB * QB);
                    for (u32 k = k0; k < k1; ++k) {
                        const u64 rbk = (u64)p.v_rb[k];
                        const u64 base = rbk * tot;
                        const double c = p.v_amp[k];
                        u32 x0 = 0, x1 = tot;
                        if (!whole_rows) {
                            const uint16_t* to2 = p.toff2 + rbk * (u64)(p.ntiles + 1) + tile;
                            x0 = to2[0];
                            x1 = to2[1];
                        }
                        for (u32 t0 = x0; t0 < x1; t0 += 64 * RT_UNROLL) {
                            u32 rt[RT_UNROLL];
                            double e[RT_UNROLL];
#pragma unroll
                            for (int u = 0; u < RT_UNROLL; ++u) {
                                const u32 t = t0 + (u32)u * 64 + lane;
                                rt[u] = 0xFFFFFFFFu;
                                e[u] = 0.0;
                                if (t < x1) {
                                    rt[u] = T2rg[base + t];
                                    e[u] = T2eg[base + t];
                                }
                            }
#pragma unroll
                            for (int u = 0; u < RT_UNROLL; ++u) {
                                const double t = e[u] * c;
                                if (rt[u] >= tlo && rt[u] < thi && e[u] != 0.0 && !xscreened(t, p.eps_x)) {
                                    atomicAdd(&acc[rt[u] - tlo], t);
                                    ++my_terms;
                                }
                            }
                        }
                    }
                    continue;
                }
                for (u32 k = k0; k < k1; ++k) {
                    const u32 beta = p.v_beta[k];
                    const double c = p.v_amp[k];
                    wave_sync();
                    if (lane < n) {
                        u32 below = (1u << lane) - 1u;
                        if ((beta >> lane) & 1u) W.occ[__popc(beta & below)] = (uint8_t)lane;
                        else W.vir[lane - __popc(beta & below)] = (uint8_t)lane;
                    }
                    wave_sync();
                    const int tot = PB * QB;
                    int po = lane / QB, pv = lane % QB;
                    const int dq = 64 / QB, dr = 64 % QB;
                    for (int t0 = 0; t0 < tot; t0 += 64) {
                        if (t0 + lane < tot) {
                            const unsigned pa = pairNB[po], pvv = pairVB[pv];
                            const int i2 = W.occ[pa & 255], j2 = W.occ[pa >> 8];
                            const int a2 = W.vir[pvv & 255], b2 = W.vir[pvv >> 8];
                            const u32 midb = beta ^ (1u << i2) ^ (1u << a2);
                            const u32 B2 = midb ^ (1u << j2) ^ (1u << b2);
                            const int top = 31 - __clz((int)B2);
                            if (top >= top_lo && top <= top_hi) {
                                const u64 rt = str_rank(B2, sB);
                                if (rt >= tlo && rt < thi) {
                                    const int par = between_parity(beta, i2, a2) ^ between_parity(midb, j2, b2);
                                    // (i2 a2|j2 b2) - (i2 b2|j2 a2), tabulated by orbital pairs
                                    double e = K4g[(u32)(j2 * (j2 - 1) / 2 + i2) * (u32)np2 + (u32)(b2 * (b2 - 1) / 2 + a2)];
                                    if (par) e = -e;
                                    const double t = e * c;
                                    if (e != 0.0 && !xscreened(t, p.eps_x)) {
                                        atomicAdd(&acc[rt - tlo], t);
                                        ++my_terms;
                                    }
                                }
                            }
                        }
                        pv += dr;
                        po += dq;
                        if (pv >= QB) { pv -= QB; po += 1; }
                    }
                }
                continue;
            }
            NbrRec r;
            if (!GRAD && li >= n1) {
                // beta singles of identity-row entries, b1_chunk per unit
                const u32 k0 = idb + (li - n1) * b1_chunk;
                r.As = At;
                r.rAs = (u32)rAt;
                r.rowb = k0;
                r.rowe = min(ide, k0 + b1_chunk);
                r.e0 = r.e1 = 0;
                r.cst = 0.0;
                r.type = 0;
                r.i = r.a = r.j = r.b = 0;
                r.par = 0;
            } else {
                r = list[li];
                if (r.type != 1) continue;  // (alpha singles come first: not reached)
            }
            const int T = r.type;
            const int I_ = r.i, A_ = r.a;
            double* slab = wslab;  // gradient: this row's (j, b) weights; sigma: the (ia|..) slab
            const bool gs = !GRAD && T == 1 && slab_n2 != 0 && r.rowe - r.rowb > p.gs_min;
            if (gs) {
                // stage this source row's alpha single's (ia|jb) as slab[j n + b]
                // (the index a table entry carries), with the alpha single's
                // phase folded in
                const u32 n2 = (u32)n * n;
                const double* Gia = p.I.g + ((u32)I_ * n + A_) * n2;
                const u64 sgn = r.par ? 0x8000000000000000ull : 0ull;
                wave_sync();
                for (u32 t = lane; t < n2; t += 64)
                    slab[t] = __longlong_as_double((long long)((u64)__double_as_longlong(Gia[t]) ^ sgn));
                wave_sync();
            }
            if (!GRAD && whole_rows && T == 1 && gs) {
                // Alpha-beta doubles, the bulk of the work.  Lanes over the
                // single-excitation index; 64 entries at a time are loaded one
                // per lane and taken in turn: an entry's table row and
                // amplitude are wavefront-uniform (readlane), so a term costs
                // one table load at a fixed per-lane offset, one slab read, a
                // multiply, a sign flip and one LDS add.  Terms are counted per
                // wavefront (ballot).
                auto run = [&](auto SCR) {
                    constexpr bool kScr = decltype(SCR)::value;
                    const auto rbg = gl(p.v_rb);
                    const auto ampg = gl(p.v_amp);
                    const double eps_x = p.eps_x;
                    for (int s0 = 0; s0 < sBn; s0 += 64) {
                        const int sidx = s0 + lane;
                        const bool act = sidx < sBn;
                        const u32 sl = act ? (u32)sidx : 0u;
                        for (u32 kb = r.rowb; kb < r.rowe; kb += 64) {
                            const u32 kk = kb + lane;
                            u32 rk = 0;
                            double ck = 0.0;
                            if (kk < r.rowe) {
                                rk = rbg[kk];
                                ck = ampg[kk];
                            }
                            const int cnt = (int)min(64u, r.rowe - kb);
                            auto trow = [&](int q) { return gl(p.T1 + (u64)rl32(rk, q) * (u32)sBn); };
                            int q = 0;
                            u32 te_next[RT_UNROLL];
                            if (RT_UNROLL <= cnt) {
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) te_next[u] = trow(u)[sl];
                            }
                            for (; q + RT_UNROLL <= cnt; q += RT_UNROLL) {
                                u32 te[RT_UNROLL];
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) te[u] = te_next[u];
                                if (q + 2 * RT_UNROLL <= cnt) {
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u) te_next[u] = trow(q + RT_UNROLL + u)[sl];
                                }
                                double x[RT_UNROLL];
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) x[u] = slab[t1_jb(te[u])];
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) {
                                    const double c = rlf64(ck, q + u);
                                    const double pr = x[u] * c;
                                    const double t = __hiloint2double(__double2hiint(pr) ^ (int)(te[u] & 0x80000000u),
                                                                      __double2loint(pr));
                                    const bool keep = act && (!kScr || !xscreened(t, eps_x));
                                    if (keep) atomicAdd(&acc[te[u] & 0x1FFFFFu], t);
                                    wterms += (u32)__popcll(__ballot(keep && x[u] != 0.0));
                                }
                            }
                            for (; q < cnt; ++q) {
                                const u32 te = trow(q)[sl];
                                const double x = slab[t1_jb(te)];
                                const double pr = x * rlf64(ck, q);
                                const double t = __hiloint2double(__double2hiint(pr) ^ (int)(te & 0x80000000u),
                                                                  __double2loint(pr));
                                const bool keep = act && (!kScr || !xscreened(t, eps_x));
                                if (keep) atomicAdd(&acc[te & 0x1FFFFFu], t);
                                wterms += (u32)__popcll(__ballot(keep && x != 0.0));
                            }
                        }
                    }
                };
                if (p.eps_x > 0.0) run(std::true_type{});
                else run(std::false_type{});
            } else if (whole_rows && T == 1) {
                // Alpha-beta doubles, the bulk of the work.  Lanes over the
                // single-excitation index; 64 entries at a time are loaded one
                // per lane and taken in turn (readlane), RT_UNROLL table reads
                // in flight.  Global-address-space loads keep the table reads
                // independent of the LDS traffic.
                const auto T1g = gl(p.T1);
                const auto rbg = gl(p.v_rb);
                const auto ampg = gl(p.v_amp);
                const int par_a = r.par;
                for (int s0 = 0; s0 < sBn; s0 += 64) {
                    const int sidx = s0 + lane;
                    const bool act = sidx < sBn;
                    for (u32 kb = r.rowb; kb < r.rowe; kb += 64) {
                        const u32 kk = kb + lane;
                        u32 rk = 0;
                        double ck = 0.0;
                        if (kk < r.rowe) {
                            rk = rbg[kk];
                            ck = ampg[kk];
                        }
                        const int cnt = (int)min(64u, r.rowe - kb);
                        // the element's integral comes from the staged LDS slab (GS) or from global memory
                        auto sweep = [&](auto GS) {
                            constexpr bool kGS = decltype(GS)::value;
                            auto element = [&](u32 te) -> double {
                                return kGS ? slab[t1_jb(te)] : p.I.g[((u32)I_ * n + A_) * (u32)(n * n) + t1_jb(te)];
                            };
                            // sign of both phases applied to x by flipping its sign bit
                            auto signed_ = [&](double x, u32 te) {
                                return __longlong_as_double(__double_as_longlong(x) ^
                                                            ((long long)(par_a ^ t1_par(te)) << 63));
                            };
                            int q = 0;
                            // the next group's table reads are issued before this group's accumulations
                            u32 te_next[RT_UNROLL];
                            if (act && RT_UNROLL <= cnt) {
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) te_next[u] = T1g[rl32(rk, u) * (u32)sBn + sidx];
                            }
                            for (; q + RT_UNROLL <= cnt; q += RT_UNROLL) {
                                if (!act) continue;
                                u32 te[RT_UNROLL];
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) te[u] = te_next[u];
                                if (q + 2 * RT_UNROLL <= cnt) {
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u)
                                        te_next[u] = T1g[rl32(rk, q + RT_UNROLL + u) * (u32)sBn + sidx];
                                }
                                if (GRAD) {
                                    // weight sbar(target) v(source) with both phases, into the (j, b) slab
                                    double sb[RT_UNROLL];
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u) sb[u] = acc[t1_rank(te[u]) - tlo];
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u) {
                                        const double c = rlf64(ck, q + u);
                                        if (sb[u] != 0.0) atomicAdd(&slab[t1_jb(te[u])], signed_(sb[u] * c, te[u]));
                                    }
                                } else {
                                    // all element reads first, then the accumulations (adding an exact
                                    // zero leaves a slot unchanged, so zero elements need no branch)
                                    double x[RT_UNROLL];
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u) x[u] = element(te[u]);
#pragma unroll
                                    for (int u = 0; u < RT_UNROLL; ++u) {
                                        const double c = rlf64(ck, q + u);
                                        const double t = signed_(x[u], te[u]) * c;
                                        if (!xscreened(t, p.eps_x)) {
                                            atomicAdd(&acc[t1_rank(te[u]) - tlo], t);
                                            my_terms += (x[u] != 0.0) ? 1u : 0u;
                                        }
                                    }
                                }
                            }
                            for (; q < cnt; ++q) {
                                if (!act) continue;
                                const u32 te = T1g[rl32(rk, q) * (u32)sBn + sidx];
                                const double c = rlf64(ck, q);
                                if (GRAD) {
                                    const double sb = acc[t1_rank(te) - tlo];
                                    if (sb != 0.0) atomicAdd(&slab[t1_jb(te)], signed_(sb * c, te));
                                } else {
                                    const double x = element(te);
                                    const double t = signed_(x, te) * c;
                                    if (!xscreened(t, p.eps_x)) {
                                        atomicAdd(&acc[t1_rank(te) - tlo], t);
                                        my_terms += (x != 0.0) ? 1u : 0u;
                                    }
                                }
                            }
                        };
                        if (gs || GRAD) sweep(std::true_type{});
                        else sweep(std::false_type{});
                    }
                }
            } else if (whole_rows) {
                // identity-row beta singles (sigma only): lanes over the
                // single-excitation index, entries in turn
                const auto T1g = gl(p.T1);
                const auto rbg = gl(p.v_rb);
                const auto ampg = gl(p.v_amp);
                const auto betag = gl(p.v_beta);
                (void)betag;
                for (int s0 = 0; s0 < sBn; s0 += 64) {
                    const int sidx = s0 + lane;
                    if (sidx >= sBn) continue;
                    const auto tsg = gl(p.TS);
                    // RT_UNROLL entries at a time, their loads in flight together;
                    // each element adds its tabulated beta part, then the alpha
                    // part in ascending orbital order
                    for (u32 k0 = r.rowb; k0 < r.rowe; k0 += RT_UNROLL) {
                        u32 te[RT_UNROLL];
                        double x[RT_UNROLL], c[RT_UNROLL];
#pragma unroll
                        for (int u = 0; u < RT_UNROLL; ++u) {
                            const u32 k = min(k0 + (u32)u, r.rowe - 1u);
                            const u32 ti = rbg[k] * (u32)sBn + sidx;
                            te[u] = T1g[ti];
                            x[u] = tsg[ti];
                            c[u] = (k0 + (u32)u < r.rowe) ? ampg[k] : 0.0;
                        }
                        if (ja_off) {
                            const u32 n2 = (u32)n * n;
                            for (int qi = 0; qi < na; ++qi) {
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u) x[u] += ja[(u32)qi * n2 + t1_jb(te[u])];
                            }
                        } else {
                            for (u32 m = At; m; m &= m - 1u) {
                                const int kq = __builtin_ctz(m);
#pragma unroll
                                for (int u = 0; u < RT_UNROLL; ++u)
                                    x[u] += p.I.g[(t1_jb(te[u]) * (u32)n + kq) * (u32)n + kq];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < RT_UNROLL; ++u) {
                            if (k0 + (u32)u >= r.rowe) continue;
                            if (t1_par(te[u])) x[u] = -x[u];
                            if (x[u] != 0.0) {
                                atomicAdd(&acc[t1_rank(te[u]) - tlo], x[u] * c[u]);
                                ++my_terms;
                            }
                        }
                    }
                }
            } else if (!GRAD && T == 1 && p.ab_it) {
                // Alpha-beta doubles of a row of several tiles: the source
                // row's items that land in this tile, listed per input chunk
                // (the chunks' item ranges read 64 at a time, a chunk per
                // lane); lanes over the items, AB_UNROLL groups of 64 loads in
                // flight.
                // The element is the staged slab's (alpha phase folded in) or
                // (ia|jb) from global memory with the alpha phase; the beta
                // phase flips the product's sign bit.
                const auto itg = gl(p.ab_it);
                const auto ampg = gl(p.v_amp);
                const auto grow = gl(p.I.g + ((u32)I_ * n + A_) * (u32)(n * n));
                const u64 nt = (u64)p.ntiles;
                const u64 c0 = p.ab_rowchunk[r.rAs];
                const u64 c1 = c0 + (r.rowe - r.rowb + AB_CHUNK - 1) / AB_CHUNK;
                const u32 pa_bit = (gs ? 0u : (u32)r.par) << 31;
                const double eps_x = p.eps_x;
                for (u64 cb = c0; cb < c1; cb += 64) {
                    // the item ranges in this tile of the row's next 64 chunks, one chunk per lane
                    u64 xl0 = 0, xl1 = 0;
                    if (cb + (u64)lane < c1) {
                        xl0 = p.ab_off[(cb + (u64)lane) * nt + (u64)tile];
                        xl1 = p.ab_off[(cb + (u64)lane) * nt + (u64)tile + 1];
                    }
                    const int ncb = (int)min((u64)64, c1 - cb);
                    for (int jc = 0; jc < ncb; ++jc) {
                        const u64 c = cb + (u64)jc;
                        const u64 x0 = rl64(xl0, jc), x1 = rl64(xl1, jc);
                        const u64 kc = (u64)r.rowb + (c - c0) * AB_CHUNK;  // the chunk's first entry
                        for (u64 xb = x0; xb < x1; xb += 64 * AB_UNROLL) {
                            u32 it[AB_UNROLL];
#pragma unroll
                            for (int u = 0; u < AB_UNROLL; ++u) {
                                const u64 x = xb + (u64)u * 64 + lane;
                                it[u] = (x < x1) ? itg[x] : 0u;
                            }
                            double e[AB_UNROLL], cc[AB_UNROLL];
#pragma unroll
                            for (int u = 0; u < AB_UNROLL; ++u) {
                                const u32 jb = (it[u] >> 14) & 1023u;
                                e[u] = gs ? slab[jb] : grow[jb];
                                cc[u] = ampg[kc + ((it[u] >> 24) & 63u)];
                            }
#pragma unroll
                            for (int u = 0; u < AB_UNROLL; ++u) {
                                const bool act = xb + (u64)u * 64 + lane < x1;
                                const double pr = e[u] * cc[u];
                                const double t = __hiloint2double(
                                    __double2hiint(pr) ^ (int)((it[u] ^ pa_bit) & 0x80000000u), __double2loint(pr));
                                const bool keep = act && !xscreened(t, eps_x);
                                if (keep) atomicAdd(&acc[it[u] & 0x3FFFu], t);
                                wterms += (u32)__popcll(__ballot(keep && e[u] != 0.0));
                            }
                        }
                    }
                }
            } else {
                for (u64 k0 = r.rowb; k0 < r.rowe; k0 += 64) {
                    const u64 k = k0 + lane;
                    unsigned len = 0, st = 0;
                    u32 beta = 0;
                    double c = 0.0;
                    if (k < r.rowe) {
                        const u64 rbeta = p.v_rb[k];
                        const uint16_t* to = p.toff + rbeta * (u64)(p.ntiles + 1);
                        const unsigned o0 = to[tile], o1 = to[tile + 1];
                        len = o1 - o0;
                        st = (unsigned)(rbeta * (u64)sBn) + o0;
                        beta = p.v_beta[k];
                        c = p.v_amp[k];
                    }
                    unsigned incl = len;
                    for (int off = 1; off < 64; off <<= 1) {
                        unsigned y = __shfl_up(incl, off);
                        if (lane >= off) incl += y;
                    }
                    const unsigned total = __shfl(incl, 63);
                    (void)beta;
                    const unsigned excl = incl - len;
                    // two groups of 64 items at a time: both table reads in flight together
                    for (unsigned q00 = 0; q00 < total; q00 += 128) {
                        unsigned qg[2], ig[2];
                        int xg[2];
                        u32 tg[2];
                        double cg[2];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            qg[u] = q00 + (unsigned)u * 64 + lane;
                            // entry of item q: the last lane whose first item is <= q
                            // (a lane with no items shares its first item with the next)
                            int x = 0;
                            for (int step = 32; step >= 1; step >>= 1) {
                                const unsigned v = (unsigned)__shfl((int)excl, x + step);
                                if (v <= qg[u]) x += step;
                            }
                            xg[u] = x;
                            // the item's table index and its entry's amplitude, from lane x
                            ig[u] = (unsigned)__shfl((int)st, x) + (qg[u] - (unsigned)__shfl((int)excl, x));
                            cg[u] = __shfl(c, x);
                        }
#pragma unroll
                        for (int u = 0; u < 2; ++u) tg[u] = (qg[u] < total) ? p.T1[ig[u]] : 0u;
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                        const unsigned q = qg[u];
                        const double cx = cg[u];
                        if (q < total) {
                            const u32 te = tg[u];
                            const u32 rt = t1_rank(te);
                            const u32 jb = t1_jb(te);
                            const int par_b = t1_par(te);
                            if (GRAD) {
                                const double sb = acc[rt - tlo];
                                if (sb != 0.0) {
                                    double w = sb * cx;
                                    if (r.par ^ par_b) w = -w;
                                    atomicAdd(&slab[jb], w);
                                }
                                continue;
                            }
                            double e;
                            if (T == 1) {
                                // the staged slab carries the alpha single's phase
                                e = gs ? slab[jb] : p.I.g[((u32)I_ * n + A_) * (u32)(n * n) + jb];
                                if ((gs ? 0 : r.par) ^ par_b) e = -e;
                            } else {
                                e = p.TS[ig[u]];
                                if (ja_off) {
                                    for (int qi = 0; qi < na; ++qi) e += ja[(u32)qi * (u32)(n * n) + jb];
                                } else {
                                    for (u32 m = At; m; m &= m - 1u) {
                                        const int kq = __builtin_ctz(m);
                                        e += p.I.g[(jb * (u32)n + kq) * (u32)n + kq];
                                    }
                                }
                                if (par_b) e = -e;
                            }
                            const double t = e * cx;
                            if (e != 0.0 && !(T == 1 && xscreened(t, p.eps_x))) {
                                atomicAdd(&acc[rt - tlo], t);
                                ++my_terms;
                            }
                        }
                        }
                    }
                }
            }
            if (GRAD) {
                // flush this row's (j, b) weights into dL/d(ia|jb)
                wave_sync();
                const u32 n2 = (u32)n * n;
                double* Rrow = p.Rg + ((u32)I_ * n + A_) * n2;
                const double pf = p.pair_half ? 2.0 : 1.0;  // the items are alpha-single rows
                for (u32 t = lane; t < n2; t += 64) {
                    const double v = slab[t];
                    if (v != 0.0) {
                        atomicAdd(Rrow + t, v * pf);
                        slab[t] = 0.0;
                    }
                }
                wave_sync();
            }
        }
        if (lane == 0) my_terms += wterms;  // the per-wavefront count, folded once per item
        wterms = 0;
        __syncthreads();
        if (!GRAD && p.fo) {
            // the list iteration's pass work on the finished tile (FusedOut)
            const FusedOut& f = *p.fo;
            const u64 rowbase = rAt * Nb;
            const double eps = p.eps;
            auto yval = [&](u32 x) -> double {
                const double v = acc[x];
                return (eps > 0.0 && fabs(v) < eps) ? 0.0 : v;
            };
            // the entries of w_l in this tile: lanes over w_l's entries of row A'
            auto scan_basis = [&](int l, auto&& fn) {
                const u64* rp = f.rowptr + (u64)l * (f.na_rows + 1);
                const u64 s0 = rp[rAt], s1 = rp[rAt + 1];
                const u64* wr = f.Wr + (u64)l * f.cap;
                for (u64 i = s0 + lane; i < s1; i += 64) {
                    const u64 rb = wr[i] - rowbase;
                    if (rb >= tlo && rb < thi) fn(i, (u32)(rb - tlo));
                }
            };
            for (int l = wave; l < f.nl; l += RT_WAVES)
                scan_basis(l, [&](u64 i, u32 x) { f.Y[(u64)l * f.cap + i] = yval(x); });
            if (f.distinct) {
                u32 nz = 0;
                for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) nz += (yval((u32)x) != 0.0) ? 1u : 0u;
                for (int off = 32; off >= 1; off >>= 1) nz += (u32)__shfl_xor((int)nz, off);
                if (lane == 0 && nz) atomicAdd((unsigned long long*)f.distinct, (unsigned long long)nz);
            }
            __syncthreads();
            for (int l = f.mark_from + wave; l < f.nl; l += RT_WAVES)
                scan_basis(l, [&](u64, u32 x) { acc[x] = 0.0; });
            __syncthreads();
            if (f.collect) {
                const u64 tb = *f.bound;
                for (int x0 = 0; x0 < tsz; x0 += RT_BLOCK) {
                    const int x = x0 + (int)threadIdx.x;
                    const double v = (x < tsz) ? yval((u32)x) : 0.0;
                    const bool pk = ((u64)__double_as_longlong(v) & 0x7fffffffffffffffull) > tb;
                    const u64 m = __ballot(pk);
                    if (m == 0) continue;
                    u64 at0 = 0;
                    if (lane == 0) at0 = atomicAdd((unsigned long long*)f.Rn, (unsigned long long)__popcll(m));
                    at0 = (u64)__shfl((long long)at0, 0);
                    if (pk) {
                        const u64 at = at0 + (u64)__popcll(m & ((1ull << lane) - 1ull));
                        if (at < f.Rcap) {
                            f.Rr[at] = rowbase + tlo + (u64)x;
                            f.Ra[at] = v;
                        } else {
                            *f.overflow = 1;
                        }
                    }
                }
            }
        } else if (!GRAD && s_touched) {
            double* dst = p.D + (rAt - p.row_base) * Nb + tlo;
            const double eps = p.eps;
            if (eps > 0.0)
                for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) dst[x] = (fabs(acc[x]) < eps) ? 0.0 : acc[x];
            else
                for (int x = threadIdx.x; x < tsz; x += RT_BLOCK) dst[x] = acc[x];
        }
        ph_add(timing, 5);
    }
    if (TIMED && !GRAD && s_cur >= 0 && p.phase_ns) {
        __syncthreads();
        if (threadIdx.x < RT_WAVES * RT_PH && s_ph[threadIdx.x / RT_PH][threadIdx.x % RT_PH])
            atomicAdd(p.phase_ns + (threadIdx.x % RT_PH), s_ph[threadIdx.x / RT_PH][threadIdx.x % RT_PH]);
    }
    if (lane == 0) my_terms += wterms;
    for (int off = 32; off >= 1; off >>= 1) my_terms += __shfl_xor(my_terms, off);
    if (lane == 0 && s_cur >= 0 && p.emitted && my_terms) atomicAdd(p.emitted, (unsigned long long)my_terms);
}

// slab_n2 > 0: every wavefront stages the (ia|jb) slab of its alpha-single
// source row in LDS at slab_off + wave * (slab_n2 + 32) doubles.
__global__ __launch_bounds__(RT_BLOCK) void k_sigma_rowtile(const RTParams* __restrict__ descs,
                                                            const u64* __restrict__ item_prefix, int n_inst,
                                                            unsigned* __restrict__ counter, void* nbr_scratch,
                                                            u64 nbr_cap, unsigned slab_off, unsigned slab_n2,
                                                            unsigned itab_off, unsigned b1_chunk, unsigned bb_chunk,
                                                            unsigned ja_off) {
    rowtile_body<RT_SIGMA>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, slab_n2, itab_off,
                           b1_chunk, bb_chunk, ja_off);
}

// The same with per-phase timing (a diagnostic build of the kernel, launched
// only when the description asks for it).
__global__ __launch_bounds__(RT_BLOCK) void k_sigma_rowtile_timed(const RTParams* __restrict__ descs,
                                                                  const u64* __restrict__ item_prefix, int n_inst,
                                                                  unsigned* __restrict__ counter, void* nbr_scratch,
                                                                  u64 nbr_cap, unsigned slab_off, unsigned slab_n2,
                                                                  unsigned itab_off, unsigned b1_chunk,
                                                                  unsigned bb_chunk, unsigned ja_off) {
    rowtile_body<RT_SIGMA, true>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, slab_n2,
                                 itab_off, b1_chunk, bb_chunk, ja_off);
}

// Integral gradients, first pass (alpha-side and alpha-beta terms).
// The same for launches whose rows are all one tile (the multi-tile code compiled out).
__global__ __launch_bounds__(RT_BLOCK) void k_sigma_rowtile_whole(const RTParams* __restrict__ descs,
                                                                  const u64* __restrict__ item_prefix, int n_inst,
                                                                  unsigned* __restrict__ counter, void* nbr_scratch,
                                                                  u64 nbr_cap, unsigned slab_off, unsigned slab_n2,
                                                                  unsigned itab_off, unsigned b1_chunk,
                                                                  unsigned bb_chunk, unsigned ja_off) {
    rowtile_body<RT_SIGMA, false, true>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, slab_n2,
                                        itab_off, b1_chunk, bb_chunk, ja_off);
}
__global__ __launch_bounds__(RT_BLOCK) void k_sigma_rowtile_whole_timed(const RTParams* __restrict__ descs,
                                                                        const u64* __restrict__ item_prefix,
                                                                        int n_inst, unsigned* __restrict__ counter,
                                                                        void* nbr_scratch, u64 nbr_cap,
                                                                        unsigned slab_off, unsigned slab_n2,
                                                                        unsigned itab_off, unsigned b1_chunk,
                                                                        unsigned bb_chunk, unsigned ja_off) {
    rowtile_body<RT_SIGMA, true, true>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, slab_n2,
                                       itab_off, b1_chunk, bb_chunk, ja_off);
}

__global__ __launch_bounds__(RT_BLOCK) void k_grad_rowtile_a(const RTParams* __restrict__ descs,
                                                             const u64* __restrict__ item_prefix, int n_inst,
                                                             unsigned* __restrict__ counter, void* nbr_scratch,
                                                             u64 nbr_cap, unsigned slab_off, unsigned slab_n2) {
    rowtile_body<RT_GRAD_A>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, slab_n2, 0u,
                            RT_B1_CHUNK, RT_BB_CHUNK, 0u);
}

// Integral gradients, second pass (beta-side terms on the spin-exchanged problem).
__global__ __launch_bounds__(RT_BLOCK) void k_grad_rowtile_b(const RTParams* __restrict__ descs,
                                                             const u64* __restrict__ item_prefix, int n_inst,
                                                             unsigned* __restrict__ counter, void* nbr_scratch,
                                                             u64 nbr_cap, unsigned slab_off) {
    rowtile_body<RT_GRAD_B>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, 0u, 0u, RT_B1_CHUNK,
                            RT_BB_CHUNK, 0u);
}

// The two passes for launches whose rows are all one tile.
__global__ __launch_bounds__(RT_BLOCK) void k_grad_rowtile_a_whole(const RTParams* __restrict__ descs,
                                                                   const u64* __restrict__ item_prefix, int n_inst,
                                                                   unsigned* __restrict__ counter, void* nbr_scratch,
                                                                   u64 nbr_cap, unsigned slab_off, unsigned slab_n2) {
    rowtile_body<RT_GRAD_A, false, true>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off,
                                         slab_n2, 0u, RT_B1_CHUNK, RT_BB_CHUNK, 0u);
}
__global__ __launch_bounds__(RT_BLOCK) void k_grad_rowtile_b_whole(const RTParams* __restrict__ descs,
                                                                   const u64* __restrict__ item_prefix, int n_inst,
                                                                   unsigned* __restrict__ counter, void* nbr_scratch,
                                                                   u64 nbr_cap, unsigned slab_off) {
    rowtile_body<RT_GRAD_B, false, true>(descs, item_prefix, n_inst, counter, nbr_scratch, nbr_cap, slab_off, 0u,
                                         0u, RT_B1_CHUNK, RT_BB_CHUNK, 0u);
}

// ---- per-problem tables ----
// T1: for every beta string, its singles sorted by target rank; toff: per-tile
// offsets into that sorted slice.  One wavefront per beta string; the sort is
// a rank-by-counting over at most 256 distinct keys.
__global__ __launch_bounds__(64) void k_build_T1(SpaceDev sp, const u64* __restrict__ binom, Ints I,
                                                 const u64* __restrict__ tile_lo, int ntiles, u32* __restrict__ T1,
                                                 double* __restrict__ TS, uint16_t* __restrict__ toff) {
    __shared__ BinomLds sB;
    __shared__ u64 key[SFCI_MAX_SINGLES];
    __shared__ uint8_t occ[32], vir[32];
    load_binom(sB, binom);
    __syncthreads();
    const int n = sp.n, nb = sp.nb, nvb = n - nb, sBn = nb * nvb;
    const int lane = threadIdx.x;
    for (u64 rb = blockIdx.x; rb < sp.Nb; rb += gridDim.x) {
        const u32 beta = str_unrank(rb, nb, n, sB);
        __syncthreads();
        if (lane < n) {
            u32 below = (1u << lane) - 1u;
            if ((beta >> lane) & 1u) occ[__popc(beta & below)] = (uint8_t)lane;
            else vir[lane - __popc(beta & below)] = (uint8_t)lane;
        }
        __syncthreads();
        for (int t = lane; t < sBn; t += 64) {
            int jj = occ[t / nvb], bb = vir[t % nvb];
            u32 B2 = beta ^ (1u << jj) ^ (1u << bb);
            u64 r = str_rank(B2, sB);
            key[t] = r | ((u64)jj << 32) | ((u64)bb << 40) | ((u64)between_parity(beta, jj, bb) << 48);
        }
        __syncthreads();
        for (int t = lane; t < sBn; t += 64) {
            const u64 me = key[t] & 0xFFFFFFFFull;
            int pos = 0;
            for (int u = 0; u < sBn; ++u) pos += ((key[u] & 0xFFFFFFFFull) < me) ? 1 : 0;
            const u64 kt = key[t];
            const int jj = (int)((kt >> 32) & 31), bb = (int)((kt >> 40) & 31);
            T1[rb * (u64)sBn + pos] = (u32)(kt & 0xFFFFFFFFull) | ((u32)(jj * sp.n + bb) << 21) |
                                      ((u32)((kt >> 48) & 1) << 31);
            // h_jb + sum_{k in beta, k != j} [(jb|kk) - (jk|kb)]: the leading part of the
            // single-excitation element, in the reference's order (the alpha part follows)
            double e = I.H(jj, bb);
            for (u32 m = beta & ~(1u << jj); m; m &= m - 1u) {
                const int k = __builtin_ctz(m);
                e += (I.G(jj, bb, k, k) - I.G(jj, k, k, bb));
            }
            TS[rb * (u64)sBn + pos] = e;
        }
        for (int t = lane; t <= ntiles; t += 64) {
            const u64 lo = tile_lo[t];
            int cnt = 0;
            for (int u = 0; u < sBn; ++u) cnt += ((key[u] & 0xFFFFFFFFull) < lo) ? 1 : 0;
            toff[rb * (u64)(ntiles + 1) + t] = (uint16_t)cnt;
        }
    }
}

// T2: for every beta string, its beta-beta doubles (i < j occupied -> a < b
// virtual, pairs in lexicographic order): the target rank, and the element
// (ia|jb) - (ib|ja) from the pair-indexed table with both phases applied,
// grouped by the target's tile (a stable grouping: pair order within a
// tile; with one tile per row, pair order) with per-tile offsets toff2.
// One wavefront per beta string; the doubles are generated twice, once to
// count per tile and once to place.
__device__ __forceinline__ void t2_double(int t, int QB, int nb, int nvb, u32 beta, const uint8_t* occ,
                                          const uint8_t* vir, u32 np2, const BinomLds& sB,
                                          const double* __restrict__ K4, u32& rt, double& e) {
    const uint16_t pa = decode_pair(t / QB, nb), pv = decode_pair(t % QB, nvb);
    const int i2 = occ[pa & 255], j2 = occ[pa >> 8];
    const int a2 = vir[pv & 255], b2 = vir[pv >> 8];
    const u32 midb = beta ^ (1u << i2) ^ (1u << a2);
    const u32 B2 = midb ^ (1u << j2) ^ (1u << b2);
    rt = (u32)str_rank(B2, sB);
    const int par = between_parity(beta, i2, a2) ^ between_parity(midb, j2, b2);
    const u32 k4 = (u32)(j2 * (j2 - 1) / 2 + i2) * np2 + (u32)(b2 * (b2 - 1) / 2 + a2);
    e = K4[k4];
    if (par) e = -e;
}

__global__ __launch_bounds__(64) void k_build_T2(SpaceDev sp, const u64* __restrict__ binom,
                                                 const double* __restrict__ K4, int nt, u32 step,
                                                 u32* __restrict__ T2r, double* __restrict__ T2e,
                                                 uint16_t* __restrict__ toff2) {
    __shared__ BinomLds sB;
    __shared__ uint8_t occ[32], vir[32];
    __shared__ u32 cnt[64];
    load_binom(sB, binom);
    __syncthreads();
    const int n = sp.n, nb = sp.nb, nvb = n - nb;
    const int QB = nvb * (nvb - 1) / 2, tot = (nb * (nb - 1) / 2) * QB;
    const u32 np2 = (u32)(n * (n - 1) / 2);
    const int lane = threadIdx.x;
    for (u64 rb = blockIdx.x; rb < sp.Nb; rb += gridDim.x) {
        const u32 beta = str_unrank(rb, nb, n, sB);
        __syncthreads();
        if (lane < n) {
            const u32 below = (1u << lane) - 1u;
            if ((beta >> lane) & 1u) occ[__popc(beta & below)] = (uint8_t)lane;
            else vir[lane - __popc(beta & below)] = (uint8_t)lane;
        }
        cnt[lane] = 0;
        __syncthreads();
        for (int t = lane; t < tot; t += 64) {
            u32 rt;
            double e;
            t2_double(t, QB, nb, nvb, beta, occ, vir, np2, sB, K4, rt, e);
            atomicAdd(&cnt[min(rt / step, (u32)(nt - 1))], 1u);
        }
        __syncthreads();
        // exclusive scan of the tile counts (lane = tile), offsets to toff2, cursors to cnt
        const u32 mine = (lane < nt) ? cnt[lane] : 0u;
        u32 incl = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const u32 y = (u32)__shfl_up((int)incl, off);
            if (lane >= off) incl += y;
        }
        const u32 excl = incl - mine;
        __syncthreads();
        if (lane <= nt) toff2[rb * (u64)(nt + 1) + lane] = (uint16_t)(lane < nt ? excl : (u32)tot);
        cnt[lane] = excl;
        __syncthreads();
        for (int t0 = 0; t0 < tot; t0 += 64) {
            const int t = t0 + lane;
            const bool act = t < tot;
            u32 rt = 0;
            double e = 0.0;
            u32 tl = 0;
            if (act) {
                t2_double(t, QB, nb, nvb, beta, occ, vir, np2, sB, K4, rt, e);
                tl = min(rt / step, (u32)(nt - 1));
            }
            // place the chunk tile by tile, lanes in order within a tile
            u64 left = __ballot(act);
            while (left) {
                const int first = __ffsll((long long)left) - 1;
                const u32 tf = (u32)__shfl((int)tl, first);
                const u64 m = __ballot(act && tl == tf);
                const u32 base = cnt[tf];
                if (act && tl == tf) {
                    const u64 at = rb * (u64)tot + base + (u32)__popcll(m & ((1ull << lane) - 1ull));
                    T2r[at] = rt;
                    T2e[at] = e;
                }
                wave_sync();
                if (lane == first) cnt[tf] = base + (u32)__popcll(m);
                wave_sync();
                left &= ~m;
            }
        }
    }
}

// K4[(i<j), (a<b)] = (ia|jb) - (ib|ja), rounded exactly as in the double's element.
__global__ void k_build_K4(int n, const double* __restrict__ g, double* __restrict__ K4) {
    const u64 np2 = (u64)n * (n - 1) / 2, t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np2 * np2) return;
    const u64 po = t / np2, pv = t % np2;
    int j = 1;
    while ((u64)(j * (j + 1) / 2) <= po) ++j;  // occupied pair (i, j): po = j(j-1)/2 + i
    const int i = (int)(po - (u64)(j * (j - 1) / 2));
    int b = 1;
    while ((u64)(b * (b + 1) / 2) <= pv) ++b;
    const int a = (int)(pv - (u64)(b * (b - 1) / 2));
    auto G = [&](int p, int q, int r, int s_) { return g[(((u64)p * n + q) * n + r) * n + s_]; };
    K4[t] = (G(i, a, j, b) - G(i, b, j, a));
}

// K2[p][q] = (pp|qq) - (pq|qp), rounded exactly as in the diagonal element.
__global__ void k_build_K(int n, const double* __restrict__ g, double* __restrict__ K) {
    const u64 n2 = (u64)n * n, t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    auto G = [&](int a, int b, int c, int d) { return g[(((u64)a * n + b) * n + c) * n + d]; };
    if (t < n2) {
        const int p = (int)(t / n), q = (int)(t % n);
        K[t] = (G(p, p, q, q) - G(p, q, q, p));
    }
}

// Row pointers of the sorted input (alpha-major ranks), the beta string of
// every entry, and per (alpha row, tile) the first entry whose beta rank is in
// that tile or above.  rowbeg/rowend/rtb must be zero-filled beforehand.
__global__ void k_rows(SpaceDev sp, const u64* __restrict__ binom, const u64* __restrict__ r, const u64* __restrict__ nnz_p,
                       const u64* __restrict__ tile_lo, int ntiles, u64* __restrict__ rowbeg, u64* __restrict__ rowend,
                       u32* __restrict__ rtb, u32* __restrict__ vbeta, u32* __restrict__ vrb) {
    __shared__ BinomLds sB;
    load_binom(sB, binom);
    __syncthreads();
    const u64 nnz = *nnz_p;
    const int nt1 = ntiles + 1;
    for (u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (u64)gridDim.x * blockDim.x) {
        const u64 R = r[k];
        const u64 ra = R / sp.Nb;
        const u64 rb = R - ra * sp.Nb;
        vbeta[k] = str_unrank(rb, sp.nb, sp.n, sB);
        vrb[k] = (u32)rb;
        int t = 0;
        while (t + 1 < ntiles && tile_lo[t + 1] <= rb) ++t;
        u32* tb = rtb + ra;  // boundary u at tb[u N_alpha]
        const bool first = (k == 0) || (r[k - 1] / sp.Nb != ra);
        const bool last = (k + 1 == nnz) || (r[k + 1] / sp.Nb != ra);
        int tprev = -1;
        if (!first) {
            const u64 rbp = r[k - 1] - ra * sp.Nb;
            tprev = 0;
            while (tprev + 1 < ntiles && tile_lo[tprev + 1] <= rbp) ++tprev;
        }
        for (int u = tprev + 1; u <= t; ++u) tb[(u64)u * sp.Na] = (u32)k;  // tiles that start at this entry
        if (last)
            for (int u = t + 1; u < nt1; ++u) tb[(u64)u * sp.Na] = (u32)(k + 1);
        if (first) rowbeg[ra] = k;
        if (last) rowend[ra] = k + 1;
    }
}

// ---- alpha-beta item lists of rows of several tiles (per sigma) ----
// An alpha-single source row feeds a target tile only through the beta
// singles of its entries that land in that tile.  Listing those items per
// (input chunk, tile) once per sigma lets every target tile stream exactly its
// items instead of revisiting each source entry once per tile of the row.

// Chunks of AB_CHUNK entries per alpha row.
__global__ void k_ab_nchunks(const u64* __restrict__ rowbeg, const u64* __restrict__ rowend, u64 Na,
                             u64* __restrict__ nch) {
    for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < Na; r += (u64)gridDim.x * blockDim.x)
        nch[r] = (rowend[r] - rowbeg[r] + AB_CHUNK - 1) / AB_CHUNK;
}

// chunkrow[c] = the alpha row of chunk c (rowchunk: Na + 1 exclusive offsets).
__global__ void k_ab_chunkmap(const u64* __restrict__ rowchunk, u64 Na, u32* __restrict__ chunkrow) {
    for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < Na; r += (u64)gridDim.x * blockDim.x)
        for (u64 c = rowchunk[r]; c < rowchunk[r + 1]; ++c) chunkrow[c] = (u32)r;
}

// cnt[c * nt + t]: items of chunk c landing in tile t.  One wavefront per
// chunk, lanes over its entries.
__global__ __launch_bounds__(256) void k_ab_count(const u64* __restrict__ rowbeg, const u64* __restrict__ rowend,
                                                  const u64* __restrict__ rowchunk, const u32* __restrict__ chunkrow,
                                                  u64 Na, const u32* __restrict__ vrb,
                                                  const uint16_t* __restrict__ toff, int nt, u64* __restrict__ cnt) {
    const u64 nch = rowchunk[Na];
    const int lane = threadIdx.x & 63;
    for (u64 c = ((u64)blockIdx.x * 256 + threadIdx.x) >> 6; c < nch; c += (u64)gridDim.x * 4) {
        const u32 r = chunkrow[c];
        const u64 k = rowbeg[r] + (c - rowchunk[r]) * AB_CHUNK + lane;
        const bool on = k < rowend[r];
        const uint16_t* to = toff + (on ? (u64)vrb[k] * (u64)(nt + 1) : 0);
        u32 prev = on ? to[0] : 0u;
        for (int t = 0; t < nt; ++t) {
            const u32 nx = on ? (u32)to[t + 1] : 0u;
            u32 len = nx - prev;
            prev = nx;
            for (int off = 32; off >= 1; off >>= 1) len += (u32)__shfl_xor((int)len, off);
            if (lane == 0) cnt[c * (u64)nt + t] = len;
        }
    }
}

// Fill the lists: one wavefront per chunk, its entries in order, lanes over
// each entry's beta singles (already sorted by target rank, so a tile's items
// of one entry are consecutive).  Within (chunk, tile) the items keep entry
// order, then the table's order.
__global__ __launch_bounds__(256) void k_ab_fill(const u64* __restrict__ rowbeg, const u64* __restrict__ rowend,
                                                 const u64* __restrict__ rowchunk, const u32* __restrict__ chunkrow,
                                                 u64 Na, const u32* __restrict__ vrb,
                                                 const uint16_t* __restrict__ toff, int nt, const u64* __restrict__ off,
                                                 const u32* __restrict__ T1, int sBn, u32 step, u64 items_cap,
                                                 u32* __restrict__ it_out) {
    __shared__ u64 s_cur[4][64];
    __shared__ u32 s_o[4][64];
    const u64 nch = rowchunk[Na];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (u64 c = ((u64)blockIdx.x * 256 + threadIdx.x) >> 6; c < nch; c += (u64)gridDim.x * 4) {
        const u32 r = chunkrow[c];
        const u64 k0 = rowbeg[r] + (c - rowchunk[r]) * AB_CHUNK;
        const u64 k1 = min(rowend[r], k0 + AB_CHUNK);
        wave_sync();
        if (lane < nt) s_cur[w][lane] = off[c * (u64)nt + lane];
        for (u64 k = k0; k < k1; ++k) {
            const u64 rb = vrb[k];
            wave_sync();
            if (lane <= nt) s_o[w][lane] = toff[rb * (u64)(nt + 1) + lane];
            wave_sync();
            for (int s0 = 0; s0 < sBn; s0 += 64) {
                const int sidx = s0 + lane;
                if (sidx < sBn) {
                    const u32 te = T1[rb * (u64)sBn + sidx];
                    const u32 t = min((te & 0x1FFFFFu) / step, (u32)(nt - 1));
                    const u64 dst = s_cur[w][t] + (u64)((u32)sidx - s_o[w][t]);
                    if (dst < items_cap) it_out[dst] = ab_item((te & 0x1FFFFFu) - t * step, te, (u32)(k - k0));
                }
            }
            wave_sync();
            if (lane < nt) s_cur[w][lane] += (u64)(s_o[w][lane + 1] - s_o[w][lane]);
        }
    }
}

u64 binom_u64(int a, int b) {
    if (b < 0 || a < b) return 0;
    u64 r = 1;
    for (int i = 1; i <= b; ++i) r = r * (u64)(a - b + i) / (u64)i;
    return r;
}

}  // namespace

static unsigned rt_itab_doubles(unsigned n2) { return (2 * n2 + 40 + 1) & ~1u; }

// The tile kernels' static LDS, as compiled (the largest of the three), so
// that static + dynamic LDS never exceeds what a workgroup may hold.
static size_t rt_static_lds() {
    static size_t cached = 0;
    if (cached == 0) {
        size_t mx = 0;
        for (const void* f : {(const void*)k_sigma_rowtile, (const void*)k_sigma_rowtile_timed,
                              (const void*)k_sigma_rowtile_whole, (const void*)k_sigma_rowtile_whole_timed,
                              (const void*)k_grad_rowtile_a, (const void*)k_grad_rowtile_b,
                              (const void*)k_grad_rowtile_a_whole, (const void*)k_grad_rowtile_b_whole}) {
            hipFuncAttributes attr{};
            SFCI_CHECK_HIP(hipFuncGetAttributes(&attr, f));
            mx = std::max(mx, (size_t)attr.sharedSizeBytes);
        }
        cached = mx + 64;  // a cache line of margin
    }
    return cached;
}

struct RowTileState {
    bool ready = false;
    int maxlds = 0;
    int ntiles = 0;
    int tile_max = 0;
    size_t lds_bytes = 0;
    std::vector<u64> tile_lo;
    u64* d_tile_lo = nullptr;
    u32* d_T1 = nullptr;
    double* d_TS = nullptr;
    double* d_K4 = nullptr;
    u32* d_T2r = nullptr;  // beta-beta doubles per beta string, grouped by target tile:
    double* d_T2e = nullptr;  // target rank, signed element
    uint16_t* d_toff2 = nullptr;  // per beta string, ntiles + 1 group offsets
    double* d_K = nullptr;  // (pp|qq) - (pq|qp), n^2
    uint16_t* d_toff = nullptr;
};

static RowTileState* rt_state(sfci_problem* P) { return (RowTileState*)P->rowtile; }

// Tiles: contiguous beta-rank ranges, equal pieces of the whole range, the
// fewest that fit in LDS.  Each tile revisits its row's source entries, so
// their number is what costs (measured at 26 orbitals: tiles of at most 2 400,
// 6 000, 13 571 ranks -> 30.9, 17.5, 10.4 s for ten sigma steps); the tables
// and ranges that select a tile's targets are exact for any boundary, and the
// top-orbital prefilter of the beta-beta doubles only widens.
static void plan_tiles(sfci_problem* P, RowTileState* S, int tile_max) {
    std::vector<std::pair<u64, u64>> tiles;  // [lo, hi), ascending
    const u64 pieces = (P->Nb + (u64)tile_max - 1) / (u64)tile_max;
    const u64 step = (P->Nb + pieces - 1) / pieces;
    for (u64 lo = 0; lo < P->Nb; lo += step) tiles.push_back({lo, std::min<u64>(P->Nb, lo + step)});
    S->tile_lo.clear();
    int mx = 0;
    for (auto& t : tiles) {
        S->tile_lo.push_back(t.first);
        mx = std::max<int>(mx, (int)(t.second - t.first));
    }
    S->tile_lo.push_back(P->Nb);
    S->ntiles = (int)tiles.size();
    S->tile_max = mx;
}

int rowtile_ntiles(sfci_problem* P) { return rowtile_available(P) ? rt_state(P)->ntiles : 0; }

const u32* rowtile_T1(sfci_problem* P) {
    const char* env = getenv("SFCI_RP_NO_T1");
    if (env && env[0] == '1') return nullptr;
    return rowtile_available(P) ? rt_state(P)->d_T1 : nullptr;
}

bool rowtile_available(sfci_problem* P) {
    // the packed single-excitation table holds a target beta rank in 21 bits
    if (P->n > 32 || P->nb * (P->n - P->nb) > SFCI_MAX_SINGLES || P->Nb >= (1ull << 21)) return false;
    RowTileState* S = rt_state(P);
    if (S && S->ready) return true;
    if (!S) {
        S = new RowTileState();
        P->rowtile = S;
    }
    int maxlds = 0;
    SFCI_CHECK_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device));
    const size_t static_lds = rt_static_lds();
    static_assert(sizeof(NbrRec) == 40, "neighbour record layout");
    // room for the element tables and the per-wavefront 32-double areas
    const size_t reserve = (rt_itab_doubles((unsigned)(P->n * P->n)) + RT_WAVES * 32) * sizeof(double);
    int tile_max = (int)(((size_t)maxlds - static_lds - reserve - 512) / sizeof(double));
    if (tile_max < 1024) return false;
    tile_max = std::min(tile_max, 16384);
    if (const char* env = getenv("SFCI_TILE_MAX")) tile_max = std::max(1024, std::min(tile_max, atoi(env)));
    plan_tiles(P, S, tile_max);
    S->lds_bytes = (size_t)S->tile_max * sizeof(double);
    const u64 sBn = (u64)P->nb * (P->n - P->nb);
    SFCI_CHECK_HIP(hipMalloc(&S->d_tile_lo, S->tile_lo.size() * sizeof(u64)));
    SFCI_CHECK_HIP(hipMemcpy(S->d_tile_lo, S->tile_lo.data(), S->tile_lo.size() * sizeof(u64), hipMemcpyHostToDevice));
    SFCI_CHECK_HIP(hipMalloc(&S->d_T1, std::max<u64>(1, P->Nb * sBn) * sizeof(u32)));
    SFCI_CHECK_HIP(hipMalloc(&S->d_toff, P->Nb * (u64)(S->ntiles + 1) * sizeof(uint16_t)));
    unsigned g = (unsigned)std::min<u64>(P->Nb, (u64)P->num_cu * 16);
    SFCI_CHECK_HIP(hipMalloc(&S->d_TS, std::max<u64>(1, P->Nb * sBn) * sizeof(double)));
    hipLaunchKernelGGL(k_build_T1, dim3(g), dim3(64), 0, P->stream, SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb},
                       P->d_binom, Ints{P->d_h, P->d_g, P->n}, S->d_tile_lo, S->ntiles, S->d_T1, S->d_TS, S->d_toff);
    SFCI_CHECK_HIP(hipGetLastError());
    {
        // same-spin double elements by orbital pairs
        const u64 np2 = (u64)P->n * (P->n - 1) / 2;
        SFCI_CHECK_HIP(hipMalloc(&S->d_K4, std::max<u64>(1, np2 * np2) * sizeof(double)));
        hipLaunchKernelGGL(k_build_K4, dim3((unsigned)std::max<u64>(1, (np2 * np2 + 255) / 256)), dim3(256), 0,
                           P->stream, P->n, P->d_g, S->d_K4);
        SFCI_CHECK_HIP(hipGetLastError());
    }
    {
        // beta-beta doubles per beta string, when a target row is one tile
        // (each double lands in it) and the table is small
        const u64 tot = (u64)(P->nb * (P->nb - 1) / 2) * (u64)((P->n - P->nb) * (P->n - P->nb - 1) / 2);
        const u64 bytes = P->Nb * tot * (sizeof(u32) + sizeof(double));
        const char* env = getenv("SFCI_NO_T2");
        // rows of one tile: up to 1 GiB (measured a win at 20 orbitals, 42 MB
        // per instance); rows of several tiles, where the on-the-fly walk
        // enumerates every double of an entry once per tile: up to a quarter
        // of the free memory
        size_t freeb = 0, totb = 0;
        SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
        const bool fits = (S->ntiles == 1) ? bytes <= (1ull << 30) : (bytes <= freeb / 4 && S->ntiles < 64);
        if (tot > 0 && tot < 65536 && fits && !(env && env[0] == '1')) {
            SFCI_CHECK_HIP(hipMalloc(&S->d_T2r, P->Nb * tot * sizeof(u32)));
            SFCI_CHECK_HIP(hipMalloc(&S->d_T2e, P->Nb * tot * sizeof(double)));
            SFCI_CHECK_HIP(hipMalloc(&S->d_toff2, P->Nb * (u64)(S->ntiles + 1) * sizeof(uint16_t)));
            const u32 step = (u32)(S->tile_lo.size() > 1 ? S->tile_lo[1] - S->tile_lo[0] : P->Nb);
            hipLaunchKernelGGL(k_build_T2, dim3(g), dim3(64), 0, P->stream, SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb},
                               P->d_binom, (const double*)S->d_K4, S->ntiles, std::max<u32>(1, step), S->d_T2r,
                               S->d_T2e, S->d_toff2);
            SFCI_CHECK_HIP(hipGetLastError());
        }
    }
    const u64 nK = (u64)P->n * P->n;
    SFCI_CHECK_HIP(hipMalloc(&S->d_K, nK * sizeof(double)));
    hipLaunchKernelGGL(k_build_K, dim3((unsigned)((nK + 255) / 256)), dim3(256), 0, P->stream, P->n, P->d_g, S->d_K);
    SFCI_CHECK_HIP(hipGetLastError());
    S->maxlds = maxlds;
    const int dyn_max = maxlds - (int)rt_static_lds();
    for (const void* f : {(const void*)k_sigma_rowtile, (const void*)k_sigma_rowtile_timed,
                          (const void*)k_sigma_rowtile_whole, (const void*)k_sigma_rowtile_whole_timed,
                          (const void*)k_grad_rowtile_a, (const void*)k_grad_rowtile_b})
        SFCI_CHECK_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_max));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    S->ready = true;
    return true;
}

void rowtile_release(sfci_problem* P) {
    RowTileState* S = rt_state(P);
    if (!S) return;
    if (S->d_tile_lo) (void)hipFree(S->d_tile_lo);
    if (S->d_T1) (void)hipFree(S->d_T1);
    if (S->d_TS) (void)hipFree(S->d_TS);
    if (S->d_K4) (void)hipFree(S->d_K4);
    if (S->d_T2r) (void)hipFree(S->d_T2r);
    if (S->d_T2e) (void)hipFree(S->d_T2e);
    if (S->d_toff2) (void)hipFree(S->d_toff2);
    if (S->d_K) (void)hipFree(S->d_K);
    if (S->d_toff) (void)hipFree(S->d_toff);
    delete S;
    P->rowtile = nullptr;
}

// The alpha-beta item lists of a sigma over rows of several tiles (see
// k_ab_fill), when the tiles are fewer than 64 and the lists take at most a
// third of the free device memory; otherwise the kernel walks each source
// entry's table slice per tile.  SFCI_AB_LISTS=0 switches them off.
static void build_ab_lists(sfci_problem* P, RowTileState* S, const SigmaLaunch& v, const u64* rowbeg,
                           const u64* rowend, const u32* vrb, RTParams& rp) {
    const u64 nt = (u64)S->ntiles;
    if (nt < 2 || nt >= 64) return;
    if (const char* env = getenv("SFCI_AB_LISTS"))
        if (env[0] == '0') return;
    const u64 cap = std::max<u64>(1, v.cap);
    const u64 sBn = (u64)rp.sB;
    const u64 chunks_max = cap / AB_CHUNK + std::min<u64>(P->Na, cap) + 1;
    const u64 items = cap * sBn;
    const u64 n_off = chunks_max * nt + 1;
    const size_t need = items * sizeof(u32) + n_off * sizeof(u64) + (P->Na + 1) * sizeof(u64) +
                        chunks_max * sizeof(u32);
    size_t freeb = 0, totb = 0;
    SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
    const size_t held = P->ws_ab_rc.bytes + P->ws_ab_cr.bytes + P->ws_ab_off.bytes + P->ws_ab_it.bytes;
    if (need > (freeb + held) / 3 || S->tile_max > 16384) return;
    u64* rowchunk = (u64*)P->ws_ab_rc.get((P->Na + 1) * sizeof(u64));
    u32* chunkrow = (u32*)P->ws_ab_cr.get(chunks_max * sizeof(u32));
    u64* off = (u64*)P->ws_ab_off.get(n_off * sizeof(u64));
    u32* it = (u32*)P->ws_ab_it.get(items * sizeof(u32));
    hipStream_t st = P->stream;
    const unsigned gr = (unsigned)std::min<u64>((P->Na + 255) / 256, 16384);
    hipLaunchKernelGGL(k_ab_nchunks, dim3(gr), dim3(256), 0, st, rowbeg, rowend, P->Na, rowchunk);
    exclusive_scan_u64(P, rowchunk, rowchunk, P->Na, rowchunk + P->Na);
    hipLaunchKernelGGL(k_ab_chunkmap, dim3(gr), dim3(256), 0, st, (const u64*)rowchunk, P->Na, chunkrow);
    launch_fill_u64(off, n_off, 0, st);
    // four wavefronts per block, one chunk each at a time
    const unsigned gc = (unsigned)std::min<u64>((chunks_max + 3) / 4, (u64)P->num_cu * 32);
    hipLaunchKernelGGL(k_ab_count, dim3(gc), dim3(256), 0, st, rowbeg, rowend, (const u64*)rowchunk,
                       (const u32*)chunkrow, P->Na, vrb, (const uint16_t*)S->d_toff, (int)nt, off);
    exclusive_scan_u64(P, off, off, n_off, nullptr);
    const u32 step = (u32)(S->tile_lo.size() > 1 ? S->tile_lo[1] - S->tile_lo[0] : P->Nb);
    hipLaunchKernelGGL(k_ab_fill, dim3(gc), dim3(256), 0, st, rowbeg, rowend, (const u64*)rowchunk,
                       (const u32*)chunkrow, P->Na, vrb, (const uint16_t*)S->d_toff, (int)nt, (const u64*)off,
                       (const u32*)S->d_T1, (int)sBn, step, items, it);
    SFCI_CHECK_HIP(hipGetLastError());
    rp.ab_it = it;
    rp.ab_off = off;
    rp.ab_rowchunk = rowchunk;
}

// Per-instance preparation on the instance's stream: row pointers, per-tile
// entry offsets and beta strings of the input vector; returns the kernel's
// description of this instance.  rowtile_available(P) must hold.
RowTileDesc rowtile_prepare(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted, double eps,
                            bool ab_lists, bool full_rows) {
    RowTileState* S = rt_state(P);
    const u64 cap = std::max<u64>(1, v.cap);
    const u64 nt1 = (u64)S->ntiles + 1;
    // rowbeg | rowend | 8 spare words | rtb (u32 per row and tile boundary)
    const u64 words = 2 * P->Na + 8 + (P->Na * nt1 + 1) / 2;
    u64* rowbeg = (u64*)P->ws_rt_rows.get(words * sizeof(u64));
    u64* rowend = rowbeg + P->Na;
    u32* rtb = (u32*)(rowend + P->Na + 8);
    u32* vbeta = (u32*)P->ws_rt_beta.get(2 * cap * sizeof(u32));
    u32* vrb = vbeta + cap;
    launch_fill_u64(rowbeg, words, 0, P->stream);
    unsigned g = (unsigned)std::min<u64>((cap + 255) / 256, 16384);
    hipLaunchKernelGGL(k_rows, dim3(g), dim3(256), 0, P->stream, SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb}, P->d_binom,
                       v.v_rank, v.v_nnz, S->d_tile_lo, S->ntiles, rowbeg, rowend, rtb, vbeta, vrb);
    SFCI_CHECK_HIP(hipGetLastError());
    RowTileDesc out;
    static_assert(sizeof(RTParams) <= sizeof(out.raw), "descriptor storage");
    RTParams& rp = *(RTParams*)out.raw;
    rp.sp = SpaceDev{P->n, P->na, P->nb, P->Na, P->Nb};
    rp.I = Ints{P->d_h, P->d_g, P->n};
    rp.binom = P->d_binom;
    rp.v_rank = v.v_rank;
    rp.v_amp = v.v_amp;
    rp.v_beta = vbeta;
    rp.v_rb = vrb;
    rp.rowbeg = rowbeg;
    rp.rowend = rowend;
    rp.rtb = rtb;
    rp.T1 = S->d_T1;
    rp.toff = S->d_toff;
    rp.tile_lo = S->d_tile_lo;
    rp.ntiles = S->ntiles;
    rp.sB = P->nb * (P->n - P->nb);
    rp.D = D;
    rp.emitted = emitted;
    rp.Rh = nullptr;
    rp.Rg = nullptr;
    rp.K2 = S->d_K;
    rp.TS = S->d_TS;
    rp.K4 = S->d_K4;
    rp.T2r = S->d_T2r;
    rp.T2e = S->d_T2e;
    rp.toff2 = S->d_toff2;
    rp.eps = eps;
    rp.eps_x = P->excite_eps;
    rp.item_base = 0;
    rp.row_base = 0;
    rp.ab_it = nullptr;
    rp.ab_off = nullptr;
    rp.ab_rowchunk = nullptr;
    if (ab_lists) build_ab_lists(P, S, v, rowbeg, rowend, vrb, rp);
    rp.fo = nullptr;
    rp.phase_ns = nullptr;
    if (const char* env = getenv("SFCI_RT_PHASES"))
        if (env[0] == '1') {
            if (!P->ws_rt_phase.p) {
                launch_fill_u64((u64*)P->ws_rt_phase.get(RT_PH * sizeof(u64)), RT_PH, 0, P->stream);
            }
            rp.phase_ns = (unsigned long long*)P->ws_rt_phase.p;
        }
    const int na = P->na, nva = P->n - P->na;
    // work units: chunks of up to tile_chunk consecutive tiles of one target
    // row (a workgroup walks a chunk's tiles in turn, reusing the row's
    // neighbour records); SFCI_TILE_CHUNK overrides the default
    // (M = 1e7, sigma per step: 28 orbitals, 24 tiles a row: 2, 3, 4, 6 tiles -> 2.297, 2.242,
    // 2.226, 2.232 s; 26 orbitals, 5 tiles: 1, 2, 3, 5 -> 0.351, 0.354, 0.356, 0.362 s)
    unsigned chunk = (S->ntiles >= 16) ? 4u : 2u;
    if (const char* env = getenv("SFCI_TILE_CHUNK")) chunk = (unsigned)std::max(1, atoi(env));
    rp.tile_chunk = std::min<unsigned>(chunk, (unsigned)S->ntiles);
    // alpha doubles added while the records are built: one thread walks the
    // entries (RT_UNROLL loads at a time), so only short ranges; ranges above
    // 8 entries go to the direct phase's wavefront stream (rows of several
    // tiles, M = 1e7: thresholds 4, 8, 16, 32, 64 give 2.297, 2.297, 2.315,
    // 2.347, 2.393 s per sigma at 28 orbitals and 0.354, 0.354, 0.357, 0.366,
    // 0.381 s at 26 orbitals).  SFCI_SHORT_DOUBLE overrides.
    rp.short_dbl = 8u;
    rp.pair_half = 0;
    rp.full_rows = full_rows ? 1u : 0u;
    // one-tile rows: a source row of at most 32 entries reads its elements from
    // global memory (staging n^2 of them would cost more than its terms);
    // measured on the 32-instance benchmark: thresholds 0, 4, 16, 32, 64, 256
    // and never staged give 1086, 1074, 1071, 1070, 1072, 1100 and 1180 ms of
    // sigma per run.  SFCI_GS_MIN overrides.
    rp.gs_min = (S->ntiles == 1) ? 32u : 0u;
    if (const char* env = getenv("SFCI_GS_MIN")) rp.gs_min = (u32)std::max(0, atoi(env));
    rp.pad_gs = 0;
    if (const char* env = getenv("SFCI_SHORT_DOUBLE")) rp.short_dbl = (u32)std::max(0, atoi(env));
    out.n_items = P->Na * (u64)((S->ntiles + rp.tile_chunk - 1) / rp.tile_chunk);
    out.nbr_cap = 1 + (u64)na * nva + (u64)(na * (na - 1) / 2) * (u64)(nva * (nva - 1) / 2);
    out.lds_bytes = S->lds_bytes;
    out.n2 = (unsigned)(P->n * P->n);
    out.ja_doubles = (unsigned)(P->na * P->n * P->n);
    out.max_lds = S->maxlds;
    return out;
}

size_t rowtile_desc_bytes() { return sizeof(RTParams); }

// One launch over n_inst instances whose descriptions (and the exclusive
// prefix of their item counts, n_inst + 1 values) are already on the device.
RowTileGeom rowtile_geom(const RowTileDesc* d, int n_inst) {
    size_t tile = 0;
    unsigned n2 = 0;
    int maxlds = 1 << 30;
    for (int k = 0; k < n_inst; ++k) {
        tile = std::max(tile, d[k].lds_bytes);
        n2 = std::max(n2, d[k].n2);
        maxlds = std::min(maxlds, d[k].max_lds);
    }
    // [tile | element tables: 2 n^2 + 40 | per wavefront: (ia|jb) slab (optional) + 32]
    tile = (tile + 15) & ~(size_t)15;
    const unsigned itab_off = (unsigned)(tile / sizeof(double));
    const unsigned slab_off = itab_off + rt_itab_doubles(n2);
    const size_t base = (size_t)slab_off * sizeof(double);
    RowTileGeom g{base + (size_t)RT_WAVES * 32 * sizeof(double), slab_off, 0u, itab_off, 0u, true};
    for (int k = 0; k < n_inst; ++k) g.whole = g.whole && ((const RTParams*)d[k].raw)->ntiles == 1;
    const size_t with = base + (size_t)RT_WAVES * (n2 + 32) * sizeof(double);
    if (with + rt_static_lds() <= (size_t)maxlds) g.lds = with, g.slab_n2 = n2;
    // then the identity row's alpha-part table, if it still fits
    unsigned ja = 0;
    for (int k = 0; k < n_inst; ++k) ja = std::max(ja, d[k].ja_doubles);
    const size_t ja_at = (g.lds + 15) & ~(size_t)15;
    if (ja && ja_at + (size_t)ja * sizeof(double) + rt_static_lds() <= (size_t)maxlds) {
        g.ja_off = (unsigned)(ja_at / sizeof(double));
        g.lds = ja_at + (size_t)ja * sizeof(double);
    }
    return g;
}

void rowtile_run(hipStream_t stream, int num_cu, const void* d_descs, const u64* d_prefix, int n_inst,
                 unsigned* d_counter, void* scratch, u64 nbr_cap, const RowTileGeom& geom, u64 total_items,
                 bool fill_counter, const RowTileTune& tune, bool timed) {
    if (fill_counter) launch_fill_u64((u64*)d_counter, 1, 0, stream);
    const unsigned grid = rowtile_grid(num_cu, geom.lds, total_items, tune.per_cu);
    auto* kern = geom.whole ? (timed ? k_sigma_rowtile_whole_timed : k_sigma_rowtile_whole)
                            : (timed ? k_sigma_rowtile_timed : k_sigma_rowtile);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(RT_BLOCK), geom.lds, stream,
                       (const RTParams*)d_descs,
                       d_prefix, n_inst, d_counter, scratch, nbr_cap, geom.slab_off, geom.slab_n2, geom.itab_off,
                       tune.b1_chunk ? tune.b1_chunk : RT_B1_CHUNK, tune.bb_chunk ? tune.bb_chunk : RT_BB_CHUNK,
                       geom.ja_off);
    SFCI_CHECK_HIP(hipGetLastError());
}

unsigned rowtile_grid(int num_cu, size_t lds_bytes, u64 total_items, unsigned per_cu_override) {
    const int per_cu = per_cu_override ? (int)per_cu_override
                                       : std::max(1, (int)((160 * 1024) / (lds_bytes + 40 * 1024)));
    return (unsigned)std::min<u64>(std::max<u64>(1, total_items), (u64)num_cu * per_cu);
}

size_t rowtile_scratch_bytes(unsigned grid, u64 nbr_cap) { return (size_t)grid * 2 * nbr_cap * sizeof(NbrRec); }

// SFCI_RT_PHASES=1: the tile kernel's wavefront time per phase since the last
// report, printed to stderr as shares (a diagnostic; it synchronises the stream).
static void report_phases(sfci_problem* P, const char* what) {
    if (!P->ws_rt_phase.p) return;
    u64 h[RT_PH] = {};
    SFCI_CHECK_HIP(hipMemcpyAsync(h, P->ws_rt_phase.p, sizeof(h), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    launch_fill_u64((u64*)P->ws_rt_phase.p, RT_PH, 0, P->stream);
    double tot = 0;
    for (u64 x : h) tot += (double)x;
    if (tot <= 0) return;
    static const char* names[RT_PH] = {"records", "direct", "alpha-beta", "id-beta-singles", "beta-beta",
                                       "wait+write", "other-units", "fetch", "clear", "records-wait"};
    std::fprintf(stderr, "# tile kernel phases (%s, %.3g wave-ticks):", what, tot);
    for (int k = 0; k < RT_PH; ++k) std::fprintf(stderr, " %s %.1f%%", names[k], 100.0 * (double)h[k] / tot);
    std::fprintf(stderr, "\n");
}

void launch_sigma_rowtile(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted, double eps) {
    RowTileDesc d = rowtile_prepare(P, v, D, emitted, eps, true);
    // descriptor | prefix (2 words) | counter
    char* buf = (char*)P->ws_rt_desc.get(sizeof(RTParams) + 64);
    u64 prefix[2] = {0, d.n_items};
    SFCI_CHECK_HIP(hipMemcpyAsync(buf, d.raw, sizeof(RTParams), hipMemcpyHostToDevice, P->stream));
    SFCI_CHECK_HIP(hipMemcpyAsync(buf + sizeof(RTParams), prefix, sizeof(prefix), hipMemcpyHostToDevice, P->stream));
    const RowTileGeom geom = rowtile_geom(&d, 1);
    const unsigned grid = rowtile_grid(P->num_cu, geom.lds, d.n_items);
    void* scratch = P->ws_rt_nbr.get(rowtile_scratch_bytes(grid, d.nbr_cap));
    const bool timed = ((RTParams*)d.raw)->phase_ns != nullptr;
    rowtile_run(P->stream, P->num_cu, buf, (const u64*)(buf + sizeof(RTParams)), 1,
                (unsigned*)(buf + sizeof(RTParams) + 16), scratch, d.nbr_cap, geom, d.n_items, true, RowTileTune{},
                timed);
    if (timed) report_phases(P, "sigma");
}

void launch_sigma_rowtile_rows(sfci_problem* P, const RowTileDesc& all, u64 lo, u64 hi, double* Dp) {
    RowTileDesc d = all;
    RTParams& rp = *(RTParams*)d.raw;
    rp.item_base = lo * (u64)rp.ntiles;
    rp.row_base = lo;
    rp.D = Dp;
    d.n_items = (hi - lo) * (u64)((rp.ntiles + rp.tile_chunk - 1) / rp.tile_chunk);
    char* buf = (char*)P->ws_rt_desc.get(sizeof(RTParams) + 64);
    u64 prefix[2] = {0, d.n_items};
    SFCI_CHECK_HIP(hipMemcpyAsync(buf, d.raw, sizeof(RTParams), hipMemcpyHostToDevice, P->stream));
    SFCI_CHECK_HIP(hipMemcpyAsync(buf + sizeof(RTParams), prefix, sizeof(prefix), hipMemcpyHostToDevice, P->stream));
    const RowTileGeom geom = rowtile_geom(&d, 1);
    const unsigned grid = rowtile_grid(P->num_cu, geom.lds, d.n_items);
    void* scratch = P->ws_rt_nbr.get(rowtile_scratch_bytes(grid, d.nbr_cap));
    rowtile_run(P->stream, P->num_cu, buf, (const u64*)(buf + sizeof(RTParams)), 1,
                (unsigned*)(buf + sizeof(RTParams) + 16), scratch, d.nbr_cap, geom, d.n_items, true, RowTileTune{},
                rp.phase_ns != nullptr);
    // the host buffers above are copied before this returns
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    if (rp.phase_ns && hi == P->Na) report_phases(P, "sigma, all row slices");
}

void launch_sigma_rowtile_rows_fused(sfci_problem* P, const RowTileDesc& all, u64 lo, u64 hi, const FusedOut* d_fo) {
    RowTileDesc d = all;
    RTParams& rp = *(RTParams*)d.raw;
    rp.fo = d_fo;
    rp.D = nullptr;
    launch_sigma_rowtile_rows(P, d, lo, hi, nullptr);
}

// ---- integral gradients through the tiles ----
namespace {

// D[rank with alpha and beta exchanged] = a (or 0): rank = r_a * N_b + r_b
// becomes r_b * N_a + r_a.
__global__ void k_scatter_tr(double* __restrict__ D, const u64* __restrict__ r, const double* __restrict__ a,
                             const u64* __restrict__ nnz, u64 Na, u64 Nb) {
    const u64 n = *nnz;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        const u64 R = r[i];
        const u64 ra = R / Nb, rb = R - ra * Nb;
        D[rb * Na + ra] = a ? a[i] : 0.0;
    }
}


unsigned g256(u64 n) { return (unsigned)std::max<u64>(1, std::min<u64>((n + 255) / 256, 16384)); }

}  // namespace

// The alpha/beta-exchanged shadow of P (created on first use).
static sfci_problem* rowtile_swapped(sfci_problem* P) {
    if (!P->swapped) {
        auto* Q = new sfci_problem();
        Q->n = P->n;
        Q->na = P->nb;
        Q->nb = P->na;
        Q->Na = P->Nb;
        Q->Nb = P->Na;
        Q->Ndet = P->Ndet;
        Q->kg = P->kg;
        Q->device = P->device;
        Q->num_cu = P->num_cu;
        Q->borrowed = true;
        P->swapped = Q;
    }
    sfci_problem* Q = P->swapped;
    Q->stream = P->stream;
    Q->d_h = P->d_h;
    Q->d_g = P->d_g;
    Q->d_binom = P->d_binom;
    Q->d_D = P->d_D;
    Q->dense_state = P->dense_state;
    return Q;
}

bool rowtile_grad_available(sfci_problem* P) {
    if (!P->d_D || !rowtile_available(P)) return false;
    sfci_problem* Q = rowtile_swapped(P);
    if (!rowtile_available(Q)) return false;
    int maxlds = 0;
    SFCI_CHECK_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device));
    const size_t n2 = (size_t)P->n * P->n;
    const size_t need_a = rt_state(P)->lds_bytes + RT_WAVES * (n2 + 32) * sizeof(double);
    const size_t need_b = rt_state(Q)->lds_bytes + RT_WAVES * 32 * sizeof(double);
    return std::max(need_a, need_b) + rt_static_lds() <= (size_t)maxlds;
}

namespace {

// One launch of a gradient pass over all jobs' descriptions.
void grad_pass(hipStream_t st, int pass, std::vector<RowTileDesc>& d, unsigned slab_n2, int num_cu,
               RowTileGradWs& ws) {
    const int n = (int)d.size();
    std::vector<u64> pre(n + 1, 0);
    u64 nbr_cap = 0;
    size_t tile_bytes = 0;
    for (int k = 0; k < n; ++k) {
        pre[k + 1] = pre[k] + d[k].n_items;
        nbr_cap = std::max(nbr_cap, d[k].nbr_cap);
        tile_bytes = std::max(tile_bytes, d[k].lds_bytes);
    }
    tile_bytes = (tile_bytes + 15) & ~(size_t)15;
    const unsigned slab_off = (unsigned)(tile_bytes / sizeof(double));
    const size_t lds = tile_bytes + (size_t)RT_WAVES * (slab_n2 + 32) * sizeof(double);
    const size_t db = sizeof(RTParams);
    char* dd = (char*)ws.desc.get((size_t)n * db);
    u64* dpre = (u64*)ws.prefix.get((size_t)(n + 1) * sizeof(u64));
    unsigned* cnt = (unsigned*)ws.counter.get(64);
    std::vector<unsigned char> host((size_t)n * db);
    for (int k = 0; k < n; ++k) std::memcpy(host.data() + (size_t)k * db, d[k].raw, db);
    SFCI_CHECK_HIP(hipMemcpyAsync(dd, host.data(), host.size(), hipMemcpyHostToDevice, st));
    SFCI_CHECK_HIP(hipMemcpyAsync(dpre, pre.data(), pre.size() * sizeof(u64), hipMemcpyHostToDevice, st));
    launch_fill_u64((u64*)cnt, 1, 0, st);
    const unsigned grid = rowtile_grid(num_cu, lds, pre[n]);
    void* scr = ws.scratch.get(rowtile_scratch_bytes(grid, nbr_cap));
    bool whole = true;  // every row one tile: the kernels with the multi-tile code compiled out
    for (int k = 0; k < n; ++k) whole = whole && ((const RTParams*)d[k].raw)->ntiles == 1;
    if (pass == 0) {
        auto* kern = whole ? k_grad_rowtile_a_whole : k_grad_rowtile_a;
        SFCI_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(RT_BLOCK), lds, st, (const RTParams*)dd, dpre, n, cnt, scr, nbr_cap,
                           slab_off, slab_n2);
    } else {
        auto* kern = whole ? k_grad_rowtile_b_whole : k_grad_rowtile_b;
        SFCI_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(RT_BLOCK), lds, st, (const RTParams*)dd, dpre, n, cnt, scr, nbr_cap,
                           slab_off);
    }
    SFCI_CHECK_HIP(hipGetLastError());
    SFCI_CHECK_HIP(hipStreamSynchronize(st));  // the host staging buffer goes out of scope
}

}  // namespace

void rowtile_gradients(hipStream_t st, int n_jobs, const GradJob* jobs, RowTileGradWs& ws) {
    std::vector<RowTileDesc> d(n_jobs);
    unsigned slab_n2 = 0;
    int num_cu = 256;
    // first pass: sbar dense in D, the sources are v
    for (int k = 0; k < n_jobs; ++k) {
        const GradJob& J = jobs[k];
        sfci_problem* P = J.P;
        if (P->stream != st) throw sfci_error(-1, "gradient jobs must run on the given stream");
        const u64 n2 = (u64)P->n * P->n;
        launch_fill_f64(J.Rh, n2, 0.0, st);
        launch_fill_f64(J.Rg, n2 * n2, 0.0, st);
        launch_scatter_set(P, P->d_D, J.s_rank, J.s_amp, J.s_nnz, J.s_cap);
        d[k] = rowtile_prepare(P, J.v, P->d_D, nullptr);
        RTParams& rp = *(RTParams*)d[k].raw;
        rp.Rh = J.Rh;
        rp.Rg = J.Rg;
        rp.pair_half = J.pair_sym ? 1u : 0u;
        slab_n2 = std::max(slab_n2, (unsigned)n2);
        num_cu = P->num_cu;
    }
    grad_pass(st, 0, d, slab_n2, num_cu, ws);
    // second pass: the spin-exchanged problem, transposed sbar and v
    for (int k = 0; k < n_jobs; ++k) {
        const GradJob& J = jobs[k];
        sfci_problem* P = J.P;
        launch_scatter_zero(P, P->d_D, J.s_rank, J.s_nnz, J.s_cap);
        hipLaunchKernelGGL(k_scatter_tr, dim3(g256(J.v.cap)), dim3(256), 0, st, P->d_D, J.v.v_rank, J.v.v_amp,
                           J.v.v_nnz, P->Na, P->Nb);
        SFCI_CHECK_HIP(hipGetLastError());
        CandSrc src{};
        src.dense = P->d_D;
        select_topm(P, src, UINT64_MAX, J.vt_rank, J.vt_amp, J.vt_nnz, true);  // sorted, and D back to zero
        hipLaunchKernelGGL(k_scatter_tr, dim3(g256(J.s_cap)), dim3(256), 0, st, P->d_D, J.s_rank, J.s_amp, J.s_nnz,
                           P->Na, P->Nb);
        SFCI_CHECK_HIP(hipGetLastError());
        sfci_problem* Q = rowtile_swapped(P);
        d[k] = rowtile_prepare(Q, SigmaLaunch{J.vt_rank, J.vt_amp, J.vt_nnz, J.v.cap}, P->d_D, nullptr);
        RTParams& rp = *(RTParams*)d[k].raw;
        rp.Rh = J.Rh;
        rp.Rg = J.Rg;
        rp.pair_half = J.pair_sym ? 1u : 0u;
    }
    grad_pass(st, 1, d, 0u, num_cu, ws);
    for (int k = 0; k < n_jobs; ++k) {
        const GradJob& J = jobs[k];
        sfci_problem* P = J.P;
        hipLaunchKernelGGL(k_scatter_tr, dim3(g256(J.s_cap)), dim3(256), 0, st, P->d_D, J.s_rank,
                           (const double*)nullptr, J.s_nnz, P->Na, P->Nb);
        SFCI_CHECK_HIP(hipGetLastError());
        launch_symmetrise(P, J.Rh, J.Rg, J.dh, J.dg);
    }
}
