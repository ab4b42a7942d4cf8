// Sort-and-merge deduplication of the intermediate elements (Sec. 2.2: the
// paper sorts each bucket by determinant and merges equal determinants with a
// linear scan; buckets are ranges of the hash, restricted to the spin-up part
// of the string in Sec. 3).  On the GPU:
//   * a pass covers a range of target alpha ranks (a contiguous rank range);
//   * tuples are emitted at fixed offsets so that the contributions to every
//     target sit in ascending source order (target-row-driven emission, or the
//     source-driven one kept as a cross-check);
//   * a stable LSD radix sort by target keeps that order inside equal keys
//     (with row-grouped tuples only the beta rank is sorted, inside each row);
//   * each run of equal keys is added in index order by one lane.
// Every target therefore receives its contributions in ascending source
// order: the result is bit-reproducible and independent of scheduling.
#include <algorithm>
#include <vector>

#include "sfci_internal.h"

namespace {

constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 16;
constexpr u64 RS_TILE = (u64)RS_BLOCK * RS_ITEMS;
constexpr int RS_SBLOCK = 512;  // threads of the scatter kernel
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;

static_assert(RS_TILE == SFCI_SORT_TILE, "sort tile");

// Where block b's tile lies (a pass's digits take nbins <= RS_BINS values).
// Plain sort: tiles of RS_TILE entries, the (digit, block) counts
// digit-major over all blocks.  Row-segmented sort
// (the input is already grouped by target row, rows in ascending order):
// tiles never cross a row, every row's counts are laid out digit-major over
// the row's own tiles, rows one after another, so one exclusive scan gives
// every (row, digit, tile) its output position; the digits are those of the
// key minus the row's first key, i.e. of the beta rank alone.
struct SortTiles {
    const u32* tile_row;  // nullptr: plain sort; else each tile's target row
    const u64* tpre;      // entries before each row (rows of the whole space)
    const u64* ttile;     // tiles before each row
    u64 lo;               // the pass's first row
    u64 Nb;               // keys per row
};

struct TileInfo {
    u64 base, len;  // the tile's entries
    u64 hb, hs;     // count of digit d at hist[hb + d * hs]
    u64 kbase;      // subtracted from the keys before the digits are taken
};

__device__ __forceinline__ TileInfo tile_info(const SortTiles& st, u64 n, u64 nblk, u64 b, u64 nbins) {
    TileInfo t;
    if (!st.tile_row) {
        t.base = b * RS_TILE;
        t.len = (n - t.base < RS_TILE) ? (n - t.base) : RS_TILE;
        t.hb = b;
        t.hs = nblk;
        t.kbase = 0;
        return t;
    }
    const u64 R = st.tile_row[b];
    const u64 t0 = st.ttile[R] - st.ttile[st.lo];
    const u64 it = b - t0;
    const u64 rlen = st.tpre[R + 1] - st.tpre[R];
    t.base = st.tpre[R] - st.tpre[st.lo] + it * RS_TILE;
    t.len = (rlen - it * RS_TILE < RS_TILE) ? (rlen - it * RS_TILE) : RS_TILE;
    t.hb = t0 * nbins + it;
    t.hs = st.ttile[R + 1] - st.ttile[R];
    t.kbase = (R - st.lo) * st.Nb;
    return t;
}

template <class K>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const K* __restrict__ keys, u64 n, int shift, int bits,
                                                      u64* __restrict__ hist, u64 nblk, SortTiles st) {
    __shared__ unsigned h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const u64 nbins = 1ull << bits;
    const TileInfo ti = tile_info(st, n, nblk, blockIdx.x, nbins);
    const K kb = (K)ti.kbase;
    const K mask = (K)(nbins - 1);
    for (int k = 0; k < RS_ITEMS; ++k) {
        const u64 i = (u64)k * RS_BLOCK + threadIdx.x;
        if (i < ti.len) atomicAdd(&h[((keys[ti.base + i] - kb) >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x < nbins) hist[ti.hb + (u64)threadIdx.x * ti.hs] = h[threadIdx.x];
}

// Rows [lo, hi) of the pass: every tile records its row.
__global__ void k_rs_tile_rows(const u64* __restrict__ ttile, u64 lo, u64 hi, u32* __restrict__ tile_row) {
    const u64 r = lo + (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= hi) return;
    for (u64 t = ttile[r]; t < ttile[r + 1]; ++t) tile_row[t - ttile[lo]] = (u32)r;
}

// One stable LSD pass (RS_SBLOCK threads).  Wavefront w of a block ranks the
// contiguous share [w * PER_WAVE, (w+1) * PER_WAVE) of the block's tile on
// its own (64 entries at a time, digit peers from ballots, running per-digit
// counts in its own LDS row: no block barrier), the block then orders the tile
// by digit in LDS (wavefront order = tile order, so the pass is stable) and
// writes every digit's run to its global slot as one contiguous stretch.  offs
// holds the exclusive prefix of the counts in the layout tile_info describes.
// Eight wavefronts per block keep more loads in flight than the LDS share of
// a four-wavefront block would allow.
template <class K>
__global__ __launch_bounds__(RS_SBLOCK) void k_rs_scatter(const K* __restrict__ keys,
                                                          const double* __restrict__ vals, u64 n, int shift,
                                                          int bits, const u64* __restrict__ offs, u64 nblk,
                                                          SortTiles st, K* __restrict__ ko,
                                                          double* __restrict__ vo) {
    constexpr int NW = RS_SBLOCK / 64;
    constexpr int DW = RS_BINS / 64;        // wavefronts holding one digit per lane
    constexpr int PER_WAVE = RS_TILE / NW;  // entries per wavefront
    static_assert(RS_SBLOCK >= RS_BINS && RS_TILE % RS_SBLOCK == 0, "scatter block");
    __shared__ K sk[RS_TILE];
    __shared__ double sv[RS_TILE];
    __shared__ u64 gstart[RS_BINS];
    __shared__ unsigned lstart[RS_BINS];
    __shared__ uint16_t wcnt[NW][RS_BINS];  // counts, then tile positions (< RS_TILE)
    __shared__ unsigned wsum[DW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 nbins = 1ull << bits;
    const TileInfo ti = tile_info(st, n, nblk, blockIdx.x, nbins);
    const K kb = (K)ti.kbase;
    const K mask = (K)(nbins - 1);
    for (int q = threadIdx.x; q < NW * RS_BINS; q += RS_SBLOCK) (&wcnt[0][0])[q] = 0;
    if (threadIdx.x < RS_BINS)
        gstart[threadIdx.x] = (threadIdx.x < nbins) ? offs[ti.hb + (u64)threadIdx.x * ti.hs] : 0;
    __syncthreads();
    // ranks inside this wavefront's share
    K key[PER_WAVE / 64];
    double val[PER_WAVE / 64];
    unsigned dig[PER_WAVE / 64], loc[PER_WAVE / 64];
    const u64 wbase = (u64)wave * PER_WAVE;
#pragma unroll
    for (int k = 0; k < PER_WAVE / 64; ++k) {
        const u64 i = wbase + (u64)k * 64 + lane;
        const bool valid = i < ti.len;
        key[k] = valid ? keys[ti.base + i] : (K)0;
        val[k] = valid ? vals[ti.base + i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < PER_WAVE / 64; ++k) {
        const u64 i = wbase + (u64)k * 64 + lane;
        const bool valid = i < ti.len;
        const unsigned d = (unsigned)(((key[k] - kb) >> shift) & mask);
        dig[k] = valid ? d : 0xffffffffu;
        u64 peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const u64 m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(peers & ((1ull << lane) - 1ull));
        loc[k] = valid ? (unsigned)wcnt[wave][d] + rank : 0u;
        wave_sync();
        if (valid && rank == 0) wcnt[wave][d] = (uint16_t)(wcnt[wave][d] + __popcll(peers));
        wave_sync();
    }
    __syncthreads();
    // block-local start of every digit (the first DW wavefronts, a digit per
    // lane), then wcnt[w][d] becomes the tile position of wavefront w's first
    // digit-d entry: lower wavefronts first, then this one's order
    const unsigned d = threadIdx.x;
    unsigned cnt = 0, x = 0;
    if (wave < DW) {
        for (int w = 0; w < NW; ++w) cnt += wcnt[w][d];
        x = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
    }
    __syncthreads();
    if (wave < DW) {
        unsigned run = x - cnt;
        for (int w = 0; w < wave; ++w) run += wsum[w];
        lstart[d] = run;
        for (int w = 0; w < NW; ++w) {
            const unsigned c = wcnt[w][d];
            wcnt[w][d] = (uint16_t)run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER_WAVE / 64; ++k) {
        const unsigned d = dig[k];
        if (d == 0xffffffffu) continue;
        const unsigned pos = wcnt[wave][d] + loc[k];
        sk[pos] = key[k];
        sv[pos] = val[k];
    }
    __syncthreads();
    for (u64 t = threadIdx.x; t < ti.len; t += RS_SBLOCK) {
        const K kk = sk[t];
        const unsigned d = (unsigned)(((kk - kb) >> shift) & mask);
        const u64 gpos = gstart[d] + (t - lstart[d]);
        ko[gpos] = kk;
        vo[gpos] = sv[t];
    }
}

// In-order sums of the runs of equal keys.  Each wavefront owns the runs
// whose first element lies in its span of SEG_SPAN positions.  It stages the
// span's values in LDS and lists the run heads, then its lanes take the runs
// in turn (run j to lane j mod 64) and each adds its run's values one by one
// in index order from a zero start, so every sum rounds exactly as a
// sequential loop does; the last run, which may cross the span's end, is
// finished by the whole wavefront staging 64 values at a time.  Sums that
// are nonzero (and, with eps > 0, have |sum| >= eps: the screening of Sec. 3)
// are written in head order, with key + key_base, to the span's own stretch
// of the staging arrays; span_cnt receives their number.  Short spans keep
// many wavefronts resident (measured at 28 orbitals: 1024, 512, 256 entries
// -> 4.8, 3.4, 3.8 ms per 5.5e8 tuples).
constexpr int SEG_SPAN = 512;
constexpr int SEG_WAVES = 4;

__device__ __forceinline__ bool keep_sum(double s, double eps) { return s != 0.0 && !(fabs(s) < eps); }

template <class K>
__global__ __launch_bounds__(64 * SEG_WAVES) void k_seg_runs(const K* __restrict__ keys,
                                                             const double* __restrict__ vals, u64 n, u64 key_base,
                                                             double eps, u64* __restrict__ stage_r,
                                                             double* __restrict__ stage_a,
                                                             u64* __restrict__ span_cnt) {
    __shared__ double sv[SEG_WAVES][SEG_SPAN];
    __shared__ uint16_t hpos[SEG_WAVES][SEG_SPAN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 lt = (1ull << lane) - 1ull;
    const u64 nspans = (n + SEG_SPAN - 1) / SEG_SPAN;
    const u64 nw = (u64)gridDim.x * SEG_WAVES;
    for (u64 w = (u64)blockIdx.x * SEG_WAVES + wave; w < nspans; w += nw) {
        const u64 a = w * SEG_SPAN;
        const int len = (int)min((u64)SEG_SPAN, n - a);
        int H = 0;
        for (int c = 0; c < SEG_SPAN; c += 64) {
            const int q = c + lane;
            const u64 i = a + q;
            const bool valid = q < len;
            const bool is_head = valid && (i == 0 || keys[i - 1] != keys[i]);
            sv[wave][q] = valid ? vals[i] : 0.0;
            const u64 m = __ballot(is_head);
            if (is_head) hpos[wave][H + __popcll(m & lt)] = (uint16_t)q;
            H += __popcll(m);
        }
        wave_sync();
        if (H == 0) {
            if (lane == 0) span_cnt[w] = 0;
            continue;
        }
        // every run but the last ends inside the span
        const int e_last = len;
        u64 kept = 0;
        double part = 0.0;  // the last run's sum over its in-span part
        for (int r0 = 0; r0 < H; r0 += 64) {
            const int j = r0 + lane;
            double acc = 0.0;
            bool keep = false;
            K key = 0;
            if (j < H) {
                const int s0 = hpos[wave][j];
                const int e = (j + 1 < H) ? (int)hpos[wave][j + 1] : e_last;
                // four values read ahead, added one by one in index order
                int q = s0;
                for (; q + 4 <= e; q += 4) {
                    const double x0 = sv[wave][q], x1 = sv[wave][q + 1], x2 = sv[wave][q + 2], x3 = sv[wave][q + 3];
                    acc += x0;
                    acc += x1;
                    acc += x2;
                    acc += x3;
                }
                for (; q < e; ++q) acc += sv[wave][q];
                key = keys[a + s0];
                if (j + 1 < H) keep = keep_sum(acc, eps);
                else part = acc;
            }
            const u64 m = __ballot(keep);
            if (keep) {
                const u64 at = a + kept + (u64)__popcll(m & lt);
                stage_r[at] = (u64)key + key_base;
                stage_a[at] = acc;
            }
            kept += (u64)__popcll(m);
        }
        // the last run continues past the span while the keys stay equal: the
        // wavefront stages 64 values at a time, lane 0 goes on adding in order
        double acc = __shfl(part, (H - 1) & 63);
        const K hk = keys[a + hpos[wave][H - 1]];
        wave_sync();
        for (u64 base = a + len; base < n; base += 64) {
            const u64 i = base + lane;
            const bool same = i < n && keys[i] == hk;
            const u64 diff = __ballot(!same);
            const int cnt = diff ? (int)__builtin_ctzll(diff) : 64;
            sv[wave][lane] = (lane < cnt) ? vals[i] : 0.0;
            wave_sync();
            if (lane == 0) {
                int q = 0;
                for (; q + 4 <= cnt; q += 4) {
                    const double x0 = sv[wave][q], x1 = sv[wave][q + 1], x2 = sv[wave][q + 2], x3 = sv[wave][q + 3];
                    acc += x0;
                    acc += x1;
                    acc += x2;
                    acc += x3;
                }
                for (; q < cnt; ++q) acc += sv[wave][q];
            }
            wave_sync();
            if (diff) break;
        }
        if (lane == 0 && keep_sum(acc, eps)) {
            stage_r[a + kept] = (u64)hk + key_base;
            stage_a[a + kept] = acc;
            ++kept;
        }
        if (lane == 0) span_cnt[w] = kept;
        wave_sync();
    }
}

// Move every span's kept sums to out[*out_base + span offset + ...] (entries
// past out_cap are dropped; the caller sees the total).
__global__ __launch_bounds__(256) void k_seg_copy(const u64* __restrict__ stage_r, const double* __restrict__ stage_a,
                                                  const u64* __restrict__ span_cnt, const u64* __restrict__ span_off,
                                                  u64 nspans, const u64* __restrict__ out_base, u64 out_cap,
                                                  u64* __restrict__ out_r, double* __restrict__ out_a) {
    const int lane = threadIdx.x & 63;
    const u64 ob = *out_base;
    const u64 nw = ((u64)gridDim.x * blockDim.x) >> 6;
    for (u64 w = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nspans; w += nw) {
        const u64 c = span_cnt[w], o = ob + span_off[w], a = w * SEG_SPAN;
        for (u64 t = lane; t < c; t += 64) {
            if (o + t < out_cap) {
                out_r[o + t] = stage_r[a + t];
                out_a[o + t] = stage_a[a + t];
            }
        }
    }
}

__global__ void k_add_scalar(u64* __restrict__ acc, const u64* __restrict__ add) {
    if (threadIdx.x == 0) *acc += *add;
}

__global__ void k_set_scalar(u64* __restrict__ dst, const u64* __restrict__ src) {
    if (threadIdx.x == 0) *dst = *src;
}

unsigned g1(u64 n, u64 per = 256) {
    u64 g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

int bits_for(u64 maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

}  // namespace

// Stable LSD radix sort of (keys, vals) on the low kbits of the key; the
// result ends in (*k_out, *v_out), which is one of the two buffer pairs.
template <class K>
void radix_passes(sfci_problem* P, K* k1, double* v1, K* k2, double* v2, u64 n, u64 nblk, int kbits,
                  const SortTiles& st, K** k_out, double** v_out) {
    // the key bits split evenly over the fewest passes of at most RS_BITS:
    // longer digit runs per tile and fewer counts to scan than full digits
    const int npass = (kbits + RS_BITS - 1) / RS_BITS;
    u64* hist = (u64*)P->ws_hist.get((u64)RS_BINS * nblk * sizeof(u64));
    for (int p = 0, shift = 0; p < npass; ++p) {
        const int bits = (kbits - shift + (npass - p) - 1) / (npass - p);
        const u64 nbins = 1ull << bits;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)nblk), dim3(RS_BLOCK), 0, P->stream, k1, n, shift, bits,
                           hist, nblk, st);
        exclusive_scan_u64(P, hist, hist, nbins * nblk, nullptr);
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)nblk), dim3(RS_SBLOCK), 0, P->stream, k1, v1, n, shift,
                           bits, hist, nblk, st, k2, v2);
        shift += bits;
        std::swap(k1, k2);
        std::swap(v1, v2);
    }
    SFCI_CHECK_HIP(hipGetLastError());
    *k_out = k1;
    *v_out = v1;
}

template <class K>
void radix_sort_pairs(sfci_problem* P, K* k1, double* v1, K* k2, double* v2, u64 n, int kbits, K** k_out,
                      double** v_out) {
    *k_out = k1;
    *v_out = v1;
    if (n == 0) return;
    radix_passes(P, k1, v1, k2, v2, n, (n + RS_TILE - 1) / RS_TILE, kbits, SortTiles{}, k_out, v_out);
}
template void radix_sort_pairs<u64>(sfci_problem*, u64*, double*, u64*, double*, u64, int, u64**, double**);
template void radix_sort_pairs<u32>(sfci_problem*, u32*, double*, u32*, double*, u64, int, u32**, double**);

int key_bits(u64 maxval) { return bits_for(maxval); }

void radix_sort_rows(sfci_problem* P, u32* k1, double* v1, u32* k2, double* v2, u64 n, const u64* tpre,
                     const u64* ttile, u64 lo, u64 hi, u64 ntiles, u32* tile_row, u32** k_out, double** v_out) {
    *k_out = k1;
    *v_out = v1;
    if (n == 0) return;
    hipLaunchKernelGGL(k_rs_tile_rows, dim3((unsigned)((hi - lo + 255) / 256)), dim3(256), 0, P->stream, ttile, lo,
                       hi, tile_row);
    const SortTiles st{tile_row, tpre, ttile, lo, P->Nb};
    radix_passes(P, k1, v1, k2, v2, n, ntiles, bits_for(P->Nb - 1), st, k_out, v_out);
}


// Sum runs of equal keys of a key-sorted list in order and append the nonzero
// sums (key + key_base, sum) at out[*out_base + ...]; *out_base += their
// number.  eps > 0 drops sums with |sum| < eps.
template <class K>
void segmented_sum_append(sfci_problem* P, const K* keys, const double* vals, u64 n, u64 key_base, double eps,
                          u64* out_base_dev, u64 out_cap, u64* out_r, double* out_a) {
    if (n == 0) return;
    u64* scal = (u64*)P->ws_scalar.get(8 * sizeof(u64));
    double* stage_a = (double*)P->ws_seg_v.get(n * sizeof(double));
    u64* stage_r = (u64*)P->ws_seg_f.get(n * sizeof(u64));
    const u64 nspans = (n + SEG_SPAN - 1) / SEG_SPAN;
    u64* cnt = (u64*)P->ws_scan2.get(2 * nspans * sizeof(u64));
    u64* off = cnt + nspans;
    const unsigned sgrid =
        (unsigned)std::max<u64>(1, std::min<u64>((nspans + SEG_WAVES - 1) / SEG_WAVES, (u64)P->num_cu * 16));
    hipLaunchKernelGGL(k_seg_runs<K>, dim3(sgrid), dim3(64 * SEG_WAVES), 0, P->stream, keys, vals, n, key_base, eps,
                       stage_r, stage_a, cnt);
    exclusive_scan_u64(P, cnt, off, nspans, &scal[2]);
    const unsigned cgrid = (unsigned)std::max<u64>(1, std::min<u64>((nspans + 3) / 4, (u64)P->num_cu * 16));
    hipLaunchKernelGGL(k_seg_copy, dim3(cgrid), dim3(256), 0, P->stream, stage_r, stage_a, cnt, off, nspans,
                       out_base_dev, out_cap, out_r, out_a);
    hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, P->stream, out_base_dev, &scal[2]);
    SFCI_CHECK_HIP(hipGetLastError());
}
template void segmented_sum_append<u64>(sfci_problem*, const u64*, const double*, u64, u64, double, u64*, u64, u64*,
                                        double*);
template void segmented_sum_append<u32>(sfci_problem*, const u32*, const double*, u64, u64, double, u64*, u64, u64*,
                                        double*);

u64 sort_tuple_cap(sfci_problem* P) {
    // Tuple buffer: a quarter of free memory (6 words per tuple over the
    // emission, sort and reduction buffers), or the share a batch assigned.
    // SFCI_SORT_TUPLE_CAP lowers it.
    size_t freeb = 0, totb = 0;
    SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
    u64 cap = P->tup_cap_hint ? P->tup_cap_hint : (u64)(freeb / 4) / SFCI_SORT_TUPLE_BYTES;
    if (const char* env = getenv("SFCI_SORT_TUPLE_CAP")) {
        long long e = atoll(env);
        if (e > 0) cap = std::min<u64>(cap, (u64)e);
    }
    if (cap < 4096) cap = 4096;
    return cap;
}

u64 sigma_sorted_passes(sfci_problem* P, const SigmaLaunch& v, SortPassSink& sink, u64* emitted_dev, u64 tup_cap,
                        double eps) {
    const char* how = getenv("SFCI_SORT_EMIT");
    if (!how || std::string(how) != "source") return sigma_rowpass(P, v, sink, emitted_dev, tup_cap, eps);
    const u64 cap_src = v.cap > 0 ? v.cap : 1;
    u64* counts = (u64*)P->ws_src_cnt.get(cap_src * sizeof(u64));
    u64* offs = (u64*)P->ws_src_off.get(cap_src * sizeof(u64));
    u64* scal = (u64*)P->ws_scalar.get(8 * sizeof(u64));  // [0] pass total, [2] segment count, [3] emitted
    launch_fill_u64(scal, 8, 0, P->stream);
    launch_fill_u64(counts, cap_src, 0, P->stream);
    if (tup_cap == 0) tup_cap = sort_tuple_cap(P);

    std::vector<std::pair<u64, u64>> todo;
    todo.push_back({0, P->Na});
    u64 emitted_total = 0, passes = 0;
    while (!todo.empty()) {
        auto [lo, hi] = todo.front();
        todo.erase(todo.begin());
        launch_sigma_count(P, v, lo, hi, counts);
        exclusive_scan_u64(P, counts, offs, cap_src, &scal[0]);
        u64 total = 0;
        SFCI_CHECK_HIP(hipMemcpyAsync(&total, &scal[0], sizeof(u64), hipMemcpyDeviceToHost, P->stream));
        SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
        if (total > tup_cap) {
            if (hi - lo <= 1) throw sfci_error(-5, "sort path: one alpha row exceeds the tuple buffer");
            u64 mid = lo + (hi - lo) / 2;
            todo.insert(todo.begin(), {mid, hi});
            todo.insert(todo.begin(), {lo, mid});
            continue;
        }
        emitted_total += total;
        if (total == 0) continue;
        ++passes;
        u64* k1 = (u64*)P->ws_tup_k.get(total * sizeof(u64));
        double* v1 = (double*)P->ws_tup_v.get(total * sizeof(double));
        u64* k2 = (u64*)P->ws_tup_k2.get(total * sizeof(u64));
        double* v2 = (double*)P->ws_tup_v2.get(total * sizeof(double));
        const u64 key_base = lo * P->Nb;
        launch_sigma_emit(P, v, lo, hi, offs, key_base, k1, v1);
        u64* ks;
        double* vs;
        radix_sort_pairs(P, k1, v1, k2, v2, total, bits_for((hi - lo) * P->Nb - 1), &ks, &vs);
        SortPassOut out = sink.begin(lo, hi, total);
        segmented_sum_append(P, ks, vs, total, key_base, eps, out.base_dev, out.cap, out.r, out.a);
        sink.end(lo, hi);
    }
    if (emitted_dev) {
        SFCI_CHECK_HIP(hipMemcpyAsync(&scal[3], &emitted_total, sizeof(u64), hipMemcpyHostToDevice, P->stream));
        hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, P->stream, emitted_dev, &scal[3]);
    }
    SFCI_CHECK_HIP(hipStreamSynchronize(P->stream));
    return passes;
}

namespace {
// Every pass appends to one rank-ordered list.
struct AppendSink : SortPassSink {
    u64 *r, *count_dev;
    double* a;
    u64 cap;
    SortPassOut begin(u64, u64, u64) override { return SortPassOut{r, a, cap, count_dev}; }
    void end(u64, u64) override {}
};
}  // namespace

void sigma_sorted(sfci_problem* P, const SigmaLaunch& v, u64 out_cap, u64* out_rank, double* out_amp,
                  u64* out_count_dev, u64* emitted_dev, double eps) {
    launch_fill_u64(out_count_dev, 1, 0, P->stream);
    AppendSink sink;
    sink.r = out_rank;
    sink.a = out_amp;
    sink.cap = out_cap;
    sink.count_dev = out_count_dev;
    sigma_sorted_passes(P, v, sink, emitted_dev, 0, eps);
}
