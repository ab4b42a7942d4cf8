// Target-row-driven emission for the sort path (Sec. 2.2's sort-and-merge
// with buckets that are ranges of the spin-up rank, Sec. 3).
//
// A source determinant (A, B) reaches target alpha rows A' that are A itself,
// an alpha single of A, or an alpha double of A; the relation is symmetric,
// so the source rows that feed a target row are found by exciting the target
// string.  Per sigma application:
//   1. row pointers of the input (entries are rank-sorted, so each source
//      alpha row is one contiguous range);
//   2. per target row, the exact number of tuples it receives: each nonempty
//      neighbouring source row contributes (entries) x (beta options of its
//      relation: all beta singles and doubles plus the diagonal for the row
//      itself, the unchanged beta string and all beta singles for an alpha
//      single, the unchanged beta string for an alpha double);
//   3. the host cuts the rows into passes of at most the tuple buffer;
//   4. per pass: the (target row, source row) pairs, sorted by source row
//      inside each target row, with their tuple offsets; an alpha-double pair
//      (most pairs, one tuple per entry) writes its tuples right there, every
//      entry of the other pairs emits its tuples at fixed positions after.
// Inside a target, contributions therefore sit in ascending source row and,
// within a row, ascending entry order, i.e. ascending source rank; the stable
// radix sort by target keeps that order and the in-order segmented sum adds
// in it.  Every option is emitted, exact-zero elements included (adding an
// exact zero leaves a sum's bits unchanged), so the counts are closed-form and
// no pass ever re-enumerates a source it does not feed.  Elements use the
// same expressions, in the same order, as the source-driven enumeration.
#include <algorithm>
#include <vector>

#include "sfci_internal.h"

namespace {

constexpr int RP_WPB = 4;
constexpr int RP_BLOCK = 64 * RP_WPB;
constexpr u32 RP_IDENT = 0, RP_SINGLE = 1, RP_DOUBLE = 2;

struct RPPair {
    u64 tup_off;    // pass-local index of the pair's first tuple
    u32 src_row;    // source alpha rank
    u32 tgt_local;  // target alpha rank minus the pass's first row
    u32 beg, ne;    // the source row's entries
    u32 info;       // type | i << 2 | a << 7 | j << 12 | b << 17 | phase << 22 (source frame)
    u32 pad;
    double e2;      // alpha-alpha double: element with its phase
};

struct RPConst {
    SpaceDev sp;
    Ints I;
    const u64* binom;
    const u64* v_rank;
    const double* v_amp;
    const u64* v_nnz;
    const u32* row_beg;
    const u32* row_end;
    int sA, sB, PA, QA, PB, QB;
    u64 c_id, c_s;  // tuples per entry of an identity pair / a single pair
    // beta singles of every beta string (target rank | (j n + b) << 21 |
    // phase << 31), or nullptr: then they are enumerated and ranked per entry
    const u32* T1;
    // excitation screen: a double's term below this magnitude is emitted as
    // 0.0 (an exact zero leaves every in-order sum's bits unchanged)
    double eps_x;
};

__device__ __forceinline__ double xterm(double t, double eps_x) { return xscreened(t, eps_x) ? 0.0 : t; }

__device__ __forceinline__ u64 wave_sum(u64 x) {
    for (int off = 32; off >= 1; off >>= 1) x += (u64)__shfl_xor((long long)x, off);
    return x;
}

// exclusive prefix over the wave; *total receives the sum
__device__ __forceinline__ u64 wave_excl_scan(u64 v, u64* total) {
    const int lane = lane_id();
    u64 x = v;
    for (int off = 1; off < 64; off <<= 1) {
        u64 y = (u64)__shfl_up((long long)x, off);
        if (lane >= off) x += y;
    }
    *total = (u64)__shfl((long long)x, 63);
    return x - v;
}

// Occupied / virtual orbital lists of a string (lanes < n write).
__device__ __forceinline__ void fill_lists(u32 S, int n, uint8_t* occ, uint8_t* vir) {
    const int lane = lane_id();
    if (lane < n) {
        const u32 below = (1u << lane) - 1u;
        if ((S >> lane) & 1u) occ[__popc(S & below)] = (uint8_t)lane;
        else vir[lane - __popc(S & below)] = (uint8_t)lane;
    }
}

// Neighbour t of target string At: t = 0 itself, then its single
// excitations, then its double excitations (pair tables pO, pV).
__device__ __forceinline__ u32 neighbour(int t, u32 At, const uint8_t* occ, const uint8_t* vir,
                                         const uint16_t* pO, const uint16_t* pV, int nv, int sA, int QA,
                                         u32* type) {
    if (t == 0) {
        *type = RP_IDENT;
        return At;
    }
    if (t <= sA) {
        const int idx = t - 1;
        *type = RP_SINGLE;
        return At ^ (1u << occ[idx / nv]) ^ (1u << vir[idx % nv]);
    }
    const int idx = t - 1 - sA;
    const u32 po = pO[idx / QA], pv = pV[idx % QA];
    *type = RP_DOUBLE;
    return At ^ (1u << occ[po & 255]) ^ (1u << occ[po >> 8]) ^ (1u << vir[pv & 255]) ^ (1u << vir[pv >> 8]);
}

__device__ __forceinline__ u64 tuples_per_entry(const RPConst& c, u32 type) {
    return type == RP_IDENT ? c.c_id : (type == RP_SINGLE ? c.c_s : 1ull);
}

__global__ void k_fill_u32(u32* p, u64 n) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_rp_rowptr(const u64* __restrict__ v_rank, const u64* __restrict__ v_nnz, u64 Nb,
                            u32* __restrict__ beg, u32* __restrict__ end) {
    const u64 n = *v_nnz;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        const u64 ra = v_rank[i] / Nb;
        if (i == 0 || v_rank[i - 1] / Nb != ra) beg[ra] = (u32)i;
        if (i + 1 == n || v_rank[i + 1] / Nb != ra) end[ra] = (u32)(i + 1);
    }
}

// Per target row: tuples received and the nonempty neighbouring source rows
// that are the row itself or an alpha single of it (the pair records the
// emission kernel walks).
__global__ __launch_bounds__(RP_BLOCK) void k_rp_count(RPConst c, u64* __restrict__ cnt, u32* __restrict__ npair) {
    __shared__ BinomLds B;
    __shared__ uint16_t pO[SFCI_MAX_PAIRS], pV[SFCI_MAX_PAIRS];
    __shared__ uint8_t occ[RP_WPB][32], vir[RP_WPB][32];
    load_binom(B, c.binom);
    const int n = c.sp.n, na = c.sp.na, nva = n - na;
    for (int t = threadIdx.x; t < c.PA; t += blockDim.x) pO[t] = decode_pair(t, na);
    for (int t = threadIdx.x; t < c.QA; t += blockDim.x) pV[t] = decode_pair(t, nva);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int K = 1 + c.sA + c.PA * c.QA;
    for (u64 r = (u64)blockIdx.x * RP_WPB + wave; r < c.sp.Na; r += (u64)gridDim.x * RP_WPB) {
        const u32 At = str_unrank(r, na, n, B);
        wave_sync();
        fill_lists(At, n, occ[wave], vir[wave]);
        wave_sync();
        u64 s = 0, k = 0;
        for (int t = lane; t < K; t += 64) {
            u32 type;
            const u32 As = neighbour(t, At, occ[wave], vir[wave], pO, pV, nva, c.sA, c.QA, &type);
            const u64 rs = str_rank(As, B);
            const u32 ne = c.row_end[rs] - c.row_beg[rs];
            if (ne) {
                s += (u64)ne * tuples_per_entry(c, type);
                if (type != RP_DOUBLE) ++k;  // alpha doubles are emitted with the pairs
            }
        }
        s = wave_sum(s);
        k = wave_sum(k);
        if (lane == 0) {
            cnt[r] = s;
            npair[r] = (u32)k;
        }
    }
}

// Pairs of the target rows [lo, hi): a block of RPP_WAVES wavefronts per row
// collects the nonempty neighbours (in any order: they are sorted next),
// sorts them by source rank (bitonic, in LDS) and assigns their tuple offsets
// in that order.  An alpha-double pair has one tuple per entry with one
// element: its wavefront writes those tuples at once, lanes over the flattened
// (pair, entry) list.  The other pairs are written as records for the
// emission kernel.
constexpr int RPP_WAVES = 4;
constexpr int RPP_BLOCK = 64 * RPP_WAVES;

__global__ __launch_bounds__(RPP_BLOCK) void k_rp_pairs(RPConst c, u64 lo, u64 hi, const u64* __restrict__ tup_pre,
                                                        const u64* __restrict__ pair_pre, RPPair* __restrict__ pairs,
                                                        u32* __restrict__ tkeys, double* __restrict__ tvals,
                                                        unsigned long long* __restrict__ nonzero) {
    extern __shared__ u64 keys[];
    __shared__ BinomLds B;
    __shared__ uint16_t pO[SFCI_MAX_PAIRS], pV[SFCI_MAX_PAIRS];
    __shared__ uint8_t occ[32], vir[32];
    __shared__ unsigned kcount;
    __shared__ u64 wtot[RPP_WAVES], wrec[RPP_WAVES];
    load_binom(B, c.binom);
    const int n = c.sp.n, na = c.sp.na, nva = n - na;
    for (int t = threadIdx.x; t < c.PA; t += blockDim.x) pO[t] = decode_pair(t, na);
    for (int t = threadIdx.x; t < c.QA; t += blockDim.x) pV[t] = decode_pair(t, nva);
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const u64 lt = (1ull << lane) - 1ull;
    const int K = 1 + c.sA + c.PA * c.QA;
    const u64 Nb = c.sp.Nb;
    u64 nz = 0;
    for (u64 r = lo + blockIdx.x; r < hi; r += gridDim.x) {
        const u32 At = str_unrank(r, na, n, B);
        if (wave == 0) fill_lists(At, n, occ, vir);
        if (threadIdx.x == 0) kcount = 0;
        __syncthreads();
        for (int t0 = 0; t0 < K; t0 += RPP_BLOCK) {
            const int t = t0 + (int)threadIdx.x;
            bool ok = false;
            u64 key = 0;
            if (t < K) {
                u32 type;
                const u32 As = neighbour(t, At, occ, vir, pO, pV, nva, c.sA, c.QA, &type);
                const u64 rs = str_rank(As, B);
                ok = c.row_end[rs] != c.row_beg[rs];
                key = (rs << 16) | (u64)t;
            }
            const u64 m = __ballot(ok);
            unsigned at = 0;
            if (lane == 0 && m) at = atomicAdd(&kcount, (unsigned)__popcll(m));
            at = (unsigned)__shfl((int)at, 0);
            if (ok) keys[at + (unsigned)__popcll(m & lt)] = key;
        }
        __syncthreads();
        const u32 k = kcount;
        u32 N = 1;
        while (N < k) N <<= 1;
        for (u32 t = k + threadIdx.x; t < N; t += RPP_BLOCK) keys[t] = ~0ull;
        __syncthreads();
        for (u32 size = 2; size <= N; size <<= 1) {
            for (u32 stride = size >> 1; stride > 0; stride >>= 1) {
                for (u32 t = threadIdx.x; t < N / 2; t += RPP_BLOCK) {
                    const u32 i = 2 * t - (t & (stride - 1));
                    const u32 j = i + stride;
                    const bool up = (i & size) == 0;
                    const u64 x = keys[i], y = keys[j];
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[j] = x;
                    }
                }
                __syncthreads();
            }
        }
        const u64 tbase = tup_pre[r] - tup_pre[lo];
        const u64 pbase = pair_pre[r] - pair_pre[lo];
        u64 run = 0, prun = 0;
        for (u32 q0 = 0; q0 < k; q0 += RPP_BLOCK) {
            const u32 q = q0 + threadIdx.x;
            u64 cntq = 0;
            RPPair pr{};
            if (q < k) {
                const u64 key = keys[q];
                const u64 rs = key >> 16;
                const int t = (int)(key & 0xffff);
                u32 type;
                const u32 As = neighbour(t, At, occ, vir, pO, pV, nva, c.sA, c.QA, &type);
                pr.src_row = (u32)rs;
                pr.tgt_local = (u32)(r - lo);
                pr.beg = c.row_beg[rs];
                pr.ne = c.row_end[rs] - pr.beg;
                u32 info = type;
                if (type == RP_SINGLE) {
                    // source A = As moves i -> a to reach At
                    const int i = __builtin_ctz(As & ~At), a = __builtin_ctz(At & ~As);
                    info |= (u32)i << 2 | (u32)a << 7 | (u32)between_parity(As, i, a) << 22;
                } else if (type == RP_DOUBLE) {
                    const u32 d1 = As & ~At, d2 = At & ~As;
                    const int i = __builtin_ctz(d1), j = __builtin_ctz(d1 & (d1 - 1u));
                    const int a = __builtin_ctz(d2), b = __builtin_ctz(d2 & (d2 - 1u));
                    const u32 mid = As ^ (1u << i) ^ (1u << a);
                    const int par = between_parity(As, i, a) ^ between_parity(mid, j, b);
                    double e = (c.I.G(i, a, j, b) - c.I.G(i, b, j, a));
                    if (par) e = -e;
                    pr.e2 = e;
                    info |= (u32)i << 2 | (u32)a << 7 | (u32)j << 12 | (u32)b << 17 | (u32)par << 22;
                }
                pr.info = info;
                cntq = (u64)pr.ne * tuples_per_entry(c, type);
            }
            // tuple offsets and record slots in ascending q over the block
            u64 wt;
            const u64 pre = wave_excl_scan(cntq, &wt);
            const bool dbl = q < k && (pr.info & 3u) == RP_DOUBLE;
            const bool rec = q < k && !dbl;
            const u64 mrec = __ballot(rec);
            if (lane == 0) {
                wtot[wave] = wt;
                wrec[wave] = (u64)__popcll(mrec);
            }
            __syncthreads();
            u64 before = 0, rbefore = 0, tot = 0, rtot = 0;
            for (int w = 0; w < RPP_WAVES; ++w) {
                if (w < wave) {
                    before += wtot[w];
                    rbefore += wrec[w];
                }
                tot += wtot[w];
                rtot += wrec[w];
            }
            __syncthreads();
            const u64 at = tbase + run + before + pre;
            if (rec) {
                pr.tup_off = at;
                pairs[pbase + prun + rbefore + (u64)__popcll(mrec & lt)] = pr;
            }
            // this wavefront's alpha-double tuples: lanes over the flattened
            // (pair, entry) list, each lane's pair found by a binary search
            // over the lanes' prefix counts
            const u64 dne = dbl ? pr.ne : 0;
            if (dbl && pr.e2 != 0.0 && !(c.eps_x > 0.0)) nz += dne;
            u64 dtot;
            const u64 dpre = wave_excl_scan(dne, &dtot);
            const u64 src_base = (u64)pr.src_row * Nb - (u64)pr.tgt_local * Nb;  // rank shift, mod 2^64
            // four groups of 64 at a time: the lane searches first, then all
            // the groups' loads together
            constexpr int DU = 4;
            for (u64 f0 = 0; f0 < dtot; f0 += 64 * DU) {
                u64 s[DU], o[DU], sb[DU];
                double e2[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const u64 f = f0 + (u64)u * 64 + lane;
                    int L = 0;
                    for (int step = 32; step >= 1; step >>= 1) {
                        const u64 v = (u64)__shfl((long long)dpre, L + step);
                        if (v <= f) L += step;
                    }
                    const u64 e = f - (u64)__shfl((long long)dpre, L);
                    s[u] = (u64)__shfl((long long)pr.beg, L) + e;
                    o[u] = (u64)__shfl((long long)at, L) + e;
                    sb[u] = (u64)__shfl((long long)src_base, L);
                    e2[u] = __shfl(pr.e2, L);
                }
                u64 rk[DU];
                double am[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const bool ok = f0 + (u64)u * 64 + lane < dtot;
                    rk[u] = ok ? c.v_rank[s[u]] : 0;
                    am[u] = ok ? c.v_amp[s[u]] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    if (f0 + (u64)u * 64 + lane < dtot) {
                        tkeys[o[u]] = (u32)(rk[u] - sb[u]);
                        const double tv = xterm(e2[u] * am[u], c.eps_x);
                        tvals[o[u]] = tv;
                        if (c.eps_x > 0.0) nz += (e2[u] != 0.0 && tv != 0.0) ? 1 : 0;
                    }
                }
            }
            run += tot;
            prun += rtot;
        }
        __syncthreads();
    }
    nz = wave_sum(nz);
    if (lane == 0 && nz) atomicAdd(nonzero, (unsigned long long)nz);
}

// Emission of the identity and alpha-single pairs (alpha-double tuples are
// written with the pairs): every wavefront owns the entries whose first tuple
// falls in its share of the pass's tuples and walks an entry's beta options
// across its lanes (alpha singles with the beta-single table: lanes over
// (entry, option) of the pair).
__global__ __launch_bounds__(RP_BLOCK) void k_rp_emit(RPConst c, const RPPair* __restrict__ pairs, u64 npairs,
                                                      u64 total, u32* __restrict__ keys, double* __restrict__ vals,
                                                      unsigned long long* __restrict__ nonzero) {
    __shared__ BinomLds B;
    __shared__ uint16_t pO[SFCI_MAX_PAIRS], pV[SFCI_MAX_PAIRS];
    __shared__ uint8_t occ[RP_WPB][32], vir[RP_WPB][32];
    load_binom(B, c.binom);
    const int n = c.sp.n, na = c.sp.na, nb = c.sp.nb, nvb = n - nb;
    for (int t = threadIdx.x; t < c.PB; t += blockDim.x) pO[t] = decode_pair(t, nb);
    for (int t = threadIdx.x; t < c.QB; t += blockDim.x) pV[t] = decode_pair(t, nvb);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const u64 gw = (u64)blockIdx.x * RP_WPB + wave, NW = (u64)gridDim.x * RP_WPB;
    const u64 T0 = (u64)(((unsigned __int128)total * gw) / NW);
    const u64 T1 = (u64)(((unsigned __int128)total * (gw + 1)) / NW);
    u64 nz = 0;
    if (T0 < T1 && npairs > 0) {
        // last pair whose first tuple is <= T0
        u64 lo = 0, hi = npairs;
        while (hi - lo > 1) {
            const u64 mid = lo + ((hi - lo) >> 1);
            if (pairs[mid].tup_off <= T0) lo = mid;
            else hi = mid;
        }
        const u64 Nb = c.sp.Nb;
        for (u64 p = lo; p < npairs; ++p) {
            const RPPair pr = pairs[p];
            if (pr.tup_off >= T1) break;
            const u32 type = pr.info & 3u;
            const u64 cp = tuples_per_entry(c, type);
            // entries whose first tuple lies in [T0, T1)
            u64 e0 = (pr.tup_off >= T0) ? 0 : (T0 - pr.tup_off + cp - 1) / cp;
            u64 e1 = (T1 - pr.tup_off + cp - 1) / cp;
            if (e1 > pr.ne) e1 = pr.ne;
            if (e0 >= e1) continue;
            const u64 tgt_base = (u64)pr.tgt_local * Nb;
            const u32 A = str_unrank(pr.src_row, na, n, B);
            const int i = (pr.info >> 2) & 31, a = (pr.info >> 7) & 31, pa = (pr.info >> 22) & 1;
            if (type == RP_SINGLE && c.T1) {
                // beta unchanged: a lane per entry
                for (u64 e = e0 + lane; e < e1; e += 64) {
                    const u64 s = pr.beg + e;
                    const u64 rB = c.v_rank[s] - (u64)pr.src_row * Nb;
                    const u32 Bs = str_unrank(rB, nb, n, B);
                    double el = single_element_nophase(c.I, A, Bs, i, a);
                    if (pa) el = -el;
                    const u64 at = pr.tup_off + e * cp;
                    keys[at] = (u32)(tgt_base + rB);
                    vals[at] = el * c.v_amp[s];
                    nz += (el != 0.0) ? 1 : 0;
                }
                // alpha-beta doubles: lanes over (entry, beta single), the
                // single's target, orbitals and phase from the table.  An
                // entry's targets are distinct, so the order of its options
                // does not matter to any sum.
                const u32 sBn = (u32)c.sB;
                const u32 nf = (u32)(e1 - e0) * sBn;
                const __attribute__((address_space(1))) double* gia =
                    (const __attribute__((address_space(1))) double*)c.I.g + (u64)(i * n + a) * n * n;
                // four groups of 64 options at a time: each level of the
                // dependent loads (entry rank, table entry, integral) is in
                // flight for all four groups together
                constexpr int EU = 4;
                for (u32 f0 = 0; f0 < nf; f0 += 64 * EU) {
                    u64 s[EU], at[EU];
                    u32 o[EU], t[EU];
                    double am[EU], el[EU];
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        const u32 f = min(f0 + (u32)u * 64 + lane, nf - 1u);
                        const u32 de = f / sBn;
                        o[u] = f - de * sBn;
                        s[u] = pr.beg + e0 + de;
                        at[u] = pr.tup_off + (e0 + de) * cp + 1 + o[u];
                    }
                    u64 rB[EU];
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        rB[u] = c.v_rank[s[u]] - (u64)pr.src_row * Nb;
                        am[u] = c.v_amp[s[u]];
                    }
#pragma unroll
                    for (int u = 0; u < EU; ++u) t[u] = c.T1[rB[u] * sBn + o[u]];
#pragma unroll
                    for (int u = 0; u < EU; ++u) el[u] = gia[(t[u] >> 21) & 1023u];  // (i a | j b), j n + b from the table
#pragma unroll
                    for (int u = 0; u < EU; ++u) {
                        if (f0 + (u32)u * 64 + lane >= nf) continue;
                        double e = el[u];
                        if (pa ^ (int)(t[u] >> 31)) e = -e;
                        keys[at[u]] = (u32)(tgt_base + (t[u] & 0x1FFFFFu));
                        const double tv = xterm(e * am[u], c.eps_x);
                        vals[at[u]] = tv;
                        nz += (e != 0.0 && !(tv == 0.0 && c.eps_x > 0.0)) ? 1 : 0;
                    }
                }
                continue;
            }
            for (u64 e = e0; e < e1; ++e) {
                const u64 s = pr.beg + e;
                const u64 rB = c.v_rank[s] - (u64)pr.src_row * Nb;
                const double amp = c.v_amp[s];
                const u32 Bs = str_unrank(rB, nb, n, B);
                wave_sync();
                fill_lists(Bs, n, occ[wave], vir[wave]);
                wave_sync();
                const u64 base = pr.tup_off + e * cp;
                for (u64 o = lane; o < cp; o += 64) {
                    double el;
                    u64 tb;
                    if (type == RP_SINGLE) {
                        if (o == 0) {
                            el = single_element_nophase(c.I, A, Bs, i, a);
                            if (pa) el = -el;
                            tb = rB;
                        } else {
                            const int idx = (int)o - 1;
                            const int jj = occ[wave][idx / nvb], bb = vir[wave][idx % nvb];
                            const u32 B2 = Bs ^ (1u << jj) ^ (1u << bb);
                            el = c.I.G(i, a, jj, bb);
                            if (pa ^ between_parity(Bs, jj, bb)) el = -el;
                            tb = str_rank(B2, B);
                        }
                    } else if (o == 0) {
                        el = diag_element(c.I, A, Bs);
                        tb = rB;
                    } else if ((int)o <= c.sB) {
                        const int idx = (int)o - 1;
                        const int jj = occ[wave][idx / nvb], bb = vir[wave][idx % nvb];
                        const u32 B2 = Bs ^ (1u << jj) ^ (1u << bb);
                        el = single_element_nophase(c.I, Bs, A, jj, bb);
                        if (between_parity(Bs, jj, bb)) el = -el;
                        tb = str_rank(B2, B);
                    } else {
                        const int idx = (int)o - 1 - c.sB;
                        const u32 po = pO[idx / c.QB], pv = pV[idx % c.QB];
                        const int ii = occ[wave][po & 255], jj = occ[wave][po >> 8];
                        const int aa = vir[wave][pv & 255], bb = vir[wave][pv >> 8];
                        const u32 mid = Bs ^ (1u << ii) ^ (1u << aa);
                        const u32 B2 = mid ^ (1u << jj) ^ (1u << bb);
                        const int par = between_parity(Bs, ii, aa) ^ between_parity(mid, jj, bb);
                        el = (c.I.G(ii, aa, jj, bb) - c.I.G(ii, bb, jj, aa));
                        if (par) el = -el;
                        tb = str_rank(B2, B);
                    }
                    // the alpha-beta doubles of a single pair (o >= 1) and the
                    // beta-beta doubles of the identity pair (o > sB) are screened
                    const bool dbl = (type == RP_SINGLE) ? (o >= 1) : ((int)o > c.sB);
                    const double tv = dbl ? xterm(el * amp, c.eps_x) : el * amp;
                    keys[base + o] = (u32)(tgt_base + tb);
                    vals[base + o] = tv;
                    nz += (el != 0.0 && !(dbl && tv == 0.0 && c.eps_x > 0.0)) ? 1 : 0;
                }
            }
        }
    }
    nz = wave_sum(nz);
    if (lane == 0 && nz) atomicAdd(nonzero, (unsigned long long)nz);
}

unsigned g1(u64 n) {
    u64 g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace

u64 sigma_rowpass(sfci_problem* P, const SigmaLaunch& v, SortPassSink& sink, u64* emitted_dev, u64 tup_cap,
                  double eps) {
    if (v.cap >= (1ull << 32)) throw sfci_error(-8, "sort path: more than 2^32 input entries");
    const int n = P->n, na = P->na, nb = P->nb;
    const u64 Na = P->Na, Nb = P->Nb;
    RPConst c;
    c.sp = SpaceDev{n, na, nb, Na, Nb};
    c.I = Ints{P->d_h, P->d_g, n};
    c.binom = P->d_binom;
    c.v_rank = v.v_rank;
    c.v_amp = v.v_amp;
    c.v_nnz = v.v_nnz;
    c.sA = na * (n - na);
    c.sB = nb * (n - nb);
    c.PA = na * (na - 1) / 2;
    c.QA = (n - na) * (n - na - 1) / 2;
    c.PB = nb * (nb - 1) / 2;
    c.QB = (n - nb) * (n - nb - 1) / 2;
    c.c_id = 1 + (u64)c.sB + (u64)c.PB * c.QB;
    c.c_s = 1 + (u64)c.sB;
    c.T1 = rowtile_T1(P);
    c.eps_x = P->excite_eps;
    const int K = 1 + c.sA + c.PA * c.QA;
    if (K > 65536) throw sfci_error(-8, "sort path: more than 65536 alpha neighbours per string");
    u32 Kp2 = 1;
    while (Kp2 < (u32)K) Kp2 <<= 1;
    if ((size_t)Kp2 * sizeof(u64) > 128 * 1024) throw sfci_error(-8, "sort path: neighbour list exceeds LDS");
    if ((size_t)Kp2 * sizeof(u64) > 48 * 1024)
        SFCI_CHECK_HIP(hipFuncSetAttribute((const void*)k_rp_pairs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(Kp2 * sizeof(u64))));
    if (tup_cap == 0) tup_cap = sort_tuple_cap(P);

    RowPassWs& ws = P->rowpass_ws;
    u32* beg = (u32*)ws.beg.get(Na * sizeof(u32));
    u32* end = (u32*)ws.end.get(Na * sizeof(u32));
    u64* cnt = (u64*)ws.cnt.get(Na * sizeof(u64));
    u32* np = (u32*)ws.npair.get(Na * sizeof(u32));
    u64* tpre = (u64*)ws.tup_pre.get((Na + 1) * sizeof(u64));
    u64* ppre = (u64*)ws.pair_pre.get((Na + 1) * sizeof(u64));
    unsigned long long* nz = (unsigned long long*)ws.scal.get(8 * sizeof(u64));
    c.row_beg = beg;
    c.row_end = end;
    hipLaunchKernelGGL(k_fill_u32, dim3(g1(Na)), dim3(256), 0, P->stream, beg, Na);
    hipLaunchKernelGGL(k_fill_u32, dim3(g1(Na)), dim3(256), 0, P->stream, end, Na);
    launch_fill_u64((u64*)nz, 1, 0, P->stream);
    hipLaunchKernelGGL(k_rp_rowptr, dim3(g1(v.cap)), dim3(256), 0, P->stream, v.v_rank, v.v_nnz, Nb, beg, end);
    const unsigned cgrid = (unsigned)std::max<u64>(1, std::min<u64>((Na + RP_WPB - 1) / RP_WPB, (u64)P->num_cu * 16));
    hipLaunchKernelGGL(k_rp_count, dim3(cgrid), dim3(RP_BLOCK), 0, P->stream, c, cnt, np);
    SFCI_CHECK_HIP(hipGetLastError());
    std::vector<u64> hc(Na), htp(Na + 1), hpp(Na + 1), htt(Na + 1);
    std::vector<u32> hn(Na);
    SFCI_CHECK_HIP(hipMemcpyAsync(hc.data(), cnt, Na * sizeof(u64), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipMemcpyAsync(hn.data(), np, Na * sizeof(u32), hipMemcpyDeviceToHost, P->stream));
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    htp[0] = hpp[0] = htt[0] = 0;
    for (u64 r = 0; r < Na; ++r) {
        htp[r + 1] = htp[r] + hc[r];
        hpp[r + 1] = hpp[r] + hn[r];
        htt[r + 1] = htt[r] + (hc[r] + SFCI_SORT_TILE - 1) / SFCI_SORT_TILE;
    }
    u64* ttile = (u64*)ws.tile_pre.get((Na + 1) * sizeof(u64));
    SFCI_CHECK_HIP(hipMemcpyAsync(tpre, htp.data(), (Na + 1) * sizeof(u64), hipMemcpyHostToDevice, P->stream));
    SFCI_CHECK_HIP(hipMemcpyAsync(ppre, hpp.data(), (Na + 1) * sizeof(u64), hipMemcpyHostToDevice, P->stream));
    SFCI_CHECK_HIP(hipMemcpyAsync(ttile, htt.data(), (Na + 1) * sizeof(u64), hipMemcpyHostToDevice, P->stream));

    const u64 pair_cap = 1ull << 26;
    // pass-local keys (target row within the pass) * N_beta + beta rank fit 32 bits
    const u64 rows_cap = (1ull << 32) / Nb;
    const unsigned egrid = (unsigned)P->num_cu * 8;
    u64 passes = 0;
    u64 lo = 0;
    while (lo < Na) {
        if (hc[lo] > tup_cap) throw sfci_error(-5, "sort path: one alpha row exceeds the tuple buffer");
        u64 hi = lo + 1;
        while (hi < Na && htp[hi + 1] - htp[lo] <= tup_cap && hpp[hi + 1] - hpp[lo] <= pair_cap &&
               hi + 1 - lo <= rows_cap)
            ++hi;
        const u64 tuples = htp[hi] - htp[lo], npairs = hpp[hi] - hpp[lo];
        if (tuples > 0) {
            ++passes;
            RPPair* pairs = (RPPair*)ws.pairs.get(std::max<u64>(1, npairs) * sizeof(RPPair));
            u32* k1 = (u32*)P->ws_tup_k.get(tuples * sizeof(u32));
            double* v1 = (double*)P->ws_tup_v.get(tuples * sizeof(double));
            u32* k2 = (u32*)P->ws_tup_k2.get(tuples * sizeof(u32));
            double* v2 = (double*)P->ws_tup_v2.get(tuples * sizeof(double));
            const unsigned pgrid = (unsigned)std::min<u64>(hi - lo, (u64)P->num_cu * 16);
            hipLaunchKernelGGL(k_rp_pairs, dim3(pgrid), dim3(RPP_BLOCK), Kp2 * sizeof(u64), P->stream, c, lo, hi, tpre,
                               ppre, pairs, k1, v1, nz);
            if (npairs > 0)
                hipLaunchKernelGGL(k_rp_emit, dim3(egrid), dim3(RP_BLOCK), 0, P->stream, c, (const RPPair*)pairs,
                                   npairs, tuples, k1, v1, nz);
            SFCI_CHECK_HIP(hipGetLastError());
            u32* ks;
            double* vs;
            // tuples sit grouped by target row: only the beta rank is sorted
            const u64 ntiles = htt[hi] - htt[lo];
            u32* tile_row = (u32*)ws.tile_row.get(ntiles * sizeof(u32));
            radix_sort_rows(P, k1, v1, k2, v2, tuples, tpre, ttile, lo, hi, ntiles, tile_row, &ks, &vs);
            SortPassOut out = sink.begin(lo, hi, tuples);
            segmented_sum_append(P, ks, vs, tuples, lo * Nb, eps, out.base_dev, out.cap, out.r, out.a);
            sink.end(lo, hi);
        }
        lo = hi;
    }
    if (emitted_dev) launch_add_u64(P, emitted_dev, (const u64*)nz);
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    return passes;
}
