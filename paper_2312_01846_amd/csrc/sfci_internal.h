// Internal host-side declarations of libsfci (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/sfci.h"
#include "sfci_device.h"

#define SFCI_CHECK_HIP(expr)                                                       \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) throw sfci_error(-6, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

struct sfci_error {
    int code;
    std::string msg;
    sfci_error(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void* get(size_t need);
    void release();
};

// Counter of frees of library-owned device memory (workspaces, tables,
// problem arrays), process-wide.  A captured graph stays launchable only
// while the counter is unchanged since its capture: every buffer it points
// to is then still allocated.
u64 device_free_epoch();
void note_device_free();

// Launch buffers of the gradient passes through the target-owned tiles.
struct RowTileGradWs {
    DevBuf desc, prefix, counter, scratch;
    void release() { desc.release(); prefix.release(); counter.release(); scratch.release(); }
};

// Top-M selection state (device resident): a radix select over the 128-bit
// key K = (bits(|c|) << rank_bits) | (N_det - 1 - rank), 11-bit digits from
// the top, so that larger K = larger |c|, then lower rank.
struct SelState {
    u64 need;       // entries still to take inside the current prefix
    u64 pre_hi, pre_lo;
    int level;      // digits fixed so far
    int done;       // selection decided
    int take_all;   // keep every nonzero entry
    int pad;
    u64 total;      // nonzero candidates (filled at level 0)
    u64 count_out;  // entries written by the compaction
    u64 cmin;       // bits of the smallest |c| among the M selected
    u64 thr_bits;   // bits of cmin * (1 - 2^-36)
    u64 count_thr;  // nonzero candidates with |c| >= that
    int use_thr;    // keep every |c| >= thr (count_thr <= M + SFCI_TIE_SLACK)
    int cand;       // compaction predicate: |c| >= cand_bits instead of the selection
    u64 cand_bits;  // dense sources: bits of the candidate bound (binade of the M-th |c|, less 2^-36)
    u64 count_cand; // candidates compacted into the list
    u64 hist[2048];
};

struct KeyGeom {
    int rank_bits;  // bits of N_det - 1 (>= 1)
    int ndig;       // number of 11-bit digits covering 63 + rank_bits bits
    int pad_bits;   // left shift that aligns the key to ndig digits
    u64 ndet_m1;
};

// Buffers of the target-row-driven sort-path emission (rowpass.hip).
struct RowPassWs {
    DevBuf beg, end, cnt, npair, tup_pre, pair_pre, pairs, scal, tile_pre, tile_row;
    void release() {
        for (DevBuf* b : {&beg, &end, &cnt, &npair, &tup_pre, &pair_pre, &pairs, &scal, &tile_pre, &tile_row})
            b->release();
    }
};

// Buffers of the list-based iteration and sigma (listlz.hip).
struct ListWs {
    DevBuf scal, pr, pa, mark, Rr, Ra, R2r, R2a, yg, taken, psi_r, psi_a, dpass, dcnt, scal2, rowptr, fo;
    void release() {
        for (DevBuf* b : {&scal, &pr, &pa, &mark, &Rr, &Ra, &R2r, &R2a, &yg, &taken, &psi_r, &psi_a, &dpass, &dcnt,
                          &scal2, &rowptr, &fo})
            b->release();
    }
};

struct sfci_problem {
    int n, na, nb;
    u64 Na, Nb, Ndet;
    KeyGeom kg;
    hipStream_t stream;
    int device;
    double* d_h = nullptr;
    double* d_g = nullptr;
    u64* d_binom = nullptr;
    double* d_D = nullptr;  // dense accumulator (N_det doubles), all zero between calls
    int dense_state = 0;    // 0 untried, 1 allocated, -1 does not fit
    int num_cu = 256;
    DevBuf ws_sel, ws_cnt, ws_scan, ws_scan2, ws_scalar, ws_red;
    DevBuf ws_tup_k, ws_tup_v, ws_tup_k2, ws_tup_v2, ws_seg_v, ws_seg_f, ws_src_cnt, ws_src_off, ws_hist;
    DevBuf ws_list_r, ws_list_a, ws_prod;
    DevBuf ws_sel2, ws_cand_r, ws_cand_a;  // top-M of a dense source: candidate list and its selection state
    DevBuf ws_lz[8];
    DevBuf ws_rt_rows, ws_rt_beta, ws_rt_nbr, ws_rt_desc;
    DevBuf ws_ab_rc, ws_ab_cr, ws_ab_off, ws_ab_it;  // alpha-beta item lists (rows of several tiles)
    DevBuf ws_rt_phase;  // optional per-phase timing of the tile kernel (SFCI_RT_PHASES=1)
    void* rowtile = nullptr;  // tables of the target-owned dense kernel (rowtile.hip)
    // The same space with alpha and beta exchanged (gradient second pass):
    // shares this problem's integrals, binomial table and dense array.
    sfci_problem* swapped = nullptr;
    RowTileGradWs grad_ws;
    ListWs list_ws;
    RowPassWs rowpass_ws;
    // projected roots of the excited-state iteration: H Psi_i lists and scalars
    DevBuf ws_hroot_r[SFCI_MAX_ROOTS], ws_hroot_a[SFCI_MAX_ROOTS], ws_roots_sc, ws_roots_cnt;
    bool borrowed = false;  // true for such a shadow: d_h, d_g, d_binom, d_D belong to another problem
    // Truncation extension (off = the paper's rule, exactly min(M, nonzero)
    // entries kept): also keep entries within a relative 2^-36 of the M-th
    // |c|, at most SFCI_TIE_SLACK of them.  Set from the options of each call.
    int tie_band = 0;
    // Sort-path tuples per pass assigned by a batch (0: a quarter of free memory).
    u64 tup_cap_hint = 0;
    // Excitation screen of the sigma kernels (0 = off): a double excitation's
    // term H_ki v_i with |H_ki v_i| < excite_eps is not added.  Set from the
    // options of each call.
    double excite_eps = 0.0;
};

// Entries a truncated vector can hold beyond M (the tie band's reach).
inline u64 tie_extra(const sfci_problem* P) { return P->tie_band ? (u64)SFCI_TIE_SLACK : 0; }

// ---- launchers (sigma.hip) ----
struct SigmaLaunch {
    const u64* v_rank;
    const double* v_amp;
    const u64* v_nnz;  // device scalar
    u64 cap;           // upper bound on nnz (grid sizing)
};
void launch_sigma_dense(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted);
void launch_sigma_count(sfci_problem* P, const SigmaLaunch& v, u64 alo, u64 ahi, u64* counts);
void launch_sigma_emit(sfci_problem* P, const SigmaLaunch& v, u64 alo, u64 ahi, const u64* offs, u64 key_base,
                       u64* keys, double* vals);
void launch_rank(sfci_problem* P, const u64* a, const u64* b, u64 cnt, u64* rank, int* bad);
void launch_unrank(sfci_problem* P, const u64* rank, u64 cnt, u64* a, u64* b, int* bad);
// Backward of sigma = H v (backward.hip).  The cotangent must already be
// scattered into the zero dense array D.  Rh (n^2) and Rg (n^4) are scratch.
void launch_backward_dense(sfci_problem* P, const SigmaLaunch& v, const double* D, double* vbar, double* dh, double* dg,
                           double* Rh, double* Rg);
void launch_scatter_zero(sfci_problem* P, double* D, const u64* r, const u64* nnz, u64 cap);

// ---- target-owned dense sigma (rowtile.hip) ----
bool rowtile_available(sfci_problem* P);  // builds the per-problem tables on first use
// The packed beta singles of every beta string (sorted by target rank), or
// nullptr where the tables cannot be built (or SFCI_RP_NO_T1=1).
const u32* rowtile_T1(sfci_problem* P);
// Beta-rank tiles per target row of the tile kernel (0 where it is unavailable).
int rowtile_ntiles(sfci_problem* P);
void rowtile_release(sfci_problem* P);
// eps > 0: accumulated entries with |c| < eps are written as zero (screening, Sec. 3).
void launch_sigma_rowtile(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted,
                          double eps = 0.0);
// Batched form: prepare each instance, put the descriptions on the device,
// then one launch drains the items of all instances.
struct RowTileDesc {
    alignas(8) unsigned char raw[384];  // kernel-side description of one instance
    u64 n_items, nbr_cap;
    size_t lds_bytes;  // the tile
    unsigned n2;       // n^2 of the instance
    unsigned ja_doubles;  // n_alpha n^2: the identity row's alpha-part table
    int max_lds;       // LDS per workgroup on the device
};
// Launch geometry for a set of descriptions: dynamic LDS, and where the
// per-wavefront integral slabs start (slab_n2 = 0: no slabs, the kernel
// reads the integrals from global memory).
struct RowTileGeom {
    size_t lds;
    unsigned slab_off, slab_n2;
    unsigned itab_off;  // per-item element tables
    unsigned ja_off;    // the identity row's alpha-part table (0: not staged)
    bool whole = false; // every instance's rows are one tile (the one-tile kernel runs)
};
RowTileGeom rowtile_geom(const RowTileDesc* d, int n_inst);
// Launch-time work sizes of the sigma tile kernel (0 = the built-in default):
// identity-row beta singles and beta-beta doubles per work unit (entries),
// and workgroups per compute unit in the grid.
struct RowTileTune {
    unsigned b1_chunk = 0, bb_chunk = 0, per_cu = 0;
};
// ab_lists: for rows of several tiles, also list the alpha-beta doubles' items
// per (input chunk, target tile) for the sigma kernel (when they fit in memory).
// full_rows: every target row of D is written (zeros where no term lands), so
// D need not be zero before the launch.
RowTileDesc rowtile_prepare(sfci_problem* P, const SigmaLaunch& v, double* D, unsigned long long* emitted,
                            double eps = 0.0, bool ab_lists = false, bool full_rows = false);
size_t rowtile_desc_bytes();
// Target alpha rows [lo, hi) of a prepared description only, written into
// Dp[rank - lo * N_beta] (touched tiles are overwritten, the rest is left
// as it is: Dp must be zero there).  Synchronises the stream.
void launch_sigma_rowtile_rows(sfci_problem* P, const RowTileDesc& all, u64 lo, u64 hi, double* Dp);
// What the tile kernel does with each finished tile instead of writing it to
// a dense slice (the list iteration's passes, fused): (1) y is gathered at the
// entries of w_l, l < nl, that fall in the tile (T_lj; Y[l cap + i]); (2) the
// entries of w_l, l >= mark_from, are left out of the candidates (Eq. 10 forms
// them afterwards); (3) with collect, every other entry with |y| above the
// running bound joins the candidate list (Rr, Ra at atomically taken
// positions; overflow set when Rcap is reached, Rn still counts); (4) the
// nonzero entries are counted into *distinct when it is set.  y is the
// screened value (|y| < eps written as 0).  Lives in device memory.
struct FusedOut {
    const u64* Wr;      // basis ranks, w_l at Wr + l cap (rank-sorted)
    const u64* rowptr;  // per l < nl: na_rows + 1 offsets, the first entry of w_l in each alpha row
    double* Y;          // gathered y, Y[l cap + i]
    u64 cap;
    u64 na_rows;
    int nl, mark_from;
    int collect, pad;
    const u64* bound;   // bits of |c| a candidate must exceed
    u64* Rr;
    double* Ra;
    u64* Rn;
    u64 Rcap;
    int* overflow;
    u64* distinct;      // may be NULL
};
// Target alpha rows [lo, hi) of a prepared description, each finished tile
// handed to the FusedOut at d_fo (device) instead of being written.
// Synchronises the stream.
void launch_sigma_rowtile_rows_fused(sfci_problem* P, const RowTileDesc& all, u64 lo, u64 hi, const FusedOut* d_fo);
unsigned rowtile_grid(int num_cu, size_t lds_bytes, u64 total_items, unsigned per_cu_override = 0);
size_t rowtile_scratch_bytes(unsigned grid, u64 nbr_cap);
// fill_counter = false: the caller has already zeroed *d_counter on the stream.
// timed: the diagnostic build with per-phase timing (descriptions carrying phase_ns).
void rowtile_run(hipStream_t stream, int num_cu, const void* d_descs, const u64* d_prefix, int n_inst,
                 unsigned* d_counter, void* scratch, u64 nbr_cap, const RowTileGeom& geom, u64 total_items,
                 bool fill_counter = true, const RowTileTune& tune = RowTileTune{}, bool timed = false);

// Integral gradients through the target-owned tiles: for each job,
// L = s^T H(h, g) v with s and v sparse (ascending unique ranks).  Raw
// gradients accumulate into Rh (n^2) and Rg (n^4), which the call zeroes
// first, and are then symmetrised into dh / dg (either may be NULL).  The
// dense array of every problem must be zero on entry; it is zero on exit.
// vt_* is scratch for the transposed v (capacity v.cap).
struct GradJob {
    sfci_problem* P;
    SigmaLaunch v;
    const u64* s_rank;
    const double* s_amp;
    const u64* s_nnz;
    u64 s_cap;
    double *Rh, *Rg, *dh, *dg;
    u64* vt_rank;
    double* vt_amp;
    u64* vt_nnz;
    // sbar is v scaled by a constant (the energy's gradient): each pair of
    // distinct connected rows is then visited once and counted twice
    bool pair_sym;
};
bool rowtile_grad_available(sfci_problem* P);
void rowtile_gradients(hipStream_t st, int n_jobs, const GradJob* jobs, RowTileGradWs& ws);
void launch_symmetrise(sfci_problem* P, const double* Rh, const double* Rg, double* dh, double* dg);

// ---- utilities (util.hip) ----
void launch_fill_f64(double* p, u64 n, double val, hipStream_t s);
void launch_fill_u64(u64* p, u64 n, u64 val, hipStream_t s);
// exclusive scan of n u64 counts into out (may alias); total -> *total_dev (device scalar).
// bsum_ws (may be NULL: the problem's buffer) holds scan_block_sums(n) u64.
void exclusive_scan_u64(sfci_problem* P, const u64* in, u64* out, u64 n, u64* total_dev, u64* bsum_ws = nullptr);
u64 scan_block_sums(u64 n);

// ---- selection (select.hip) ----
// Source of candidates: either a dense array (index = rank) or a list.
struct CandSrc {
    const double* dense;  // if non-null: D[0..Ndet)
    const u64* lrank;     // else list
    const double* lval;
    const u64* lcount;    // device scalar
    u64 lcap;
};
// ---- batched iteration steps: one launch serves every instance ----
// One instance of a batch, in a device array indexed by blockIdx.y: its basis
// vectors, dense accumulator, block matrices, and selection workspaces.
struct BInst {
    u64* Wr;                  // basis vector l: ranks Wr + l cap, amplitudes Wa + l cap, count sc[l]
    double* Wa;
    u64* sc;
    u64 cap;
    double* D;                // dense accumulator, N_det doubles (all zero between steps)
    u64 Ndet;
    double* T;                // n_L x n_L, T[l n_L + j]
    double* S;
    double* x;                // block end: the lowest eigenvector, its eigenvalue, energies[*blk]
    double* lam;
    double* energies;
    int* blk;
    int* status;
    double* red;              // reduction partials, bstep_red_doubles(n_L)
    SelState* st;             // selection on the dense accumulator, then on the candidate list
    SelState* st2;
    u64* cr;                  // candidate list (N_det capacity)
    double* ca;
    u64* cnt;                 // per-chunk counts (select chunks of N_det) and their scan's block sums
    u64* bsum;
    u64* psi_r;               // the final Psi of the last block
    double* psi_a;
    u64* psi_n;
    u64 M;                    // truncation (UINT64_MAX: every nonzero entry)
    u64 ndet_m1;              // key geometry of the selection
    int rank_bits;
    int nL;
};
// Where a batched selection writes: w_{j+1}, w_0 (a block end) or Psi.
enum { BOUT_NEXT = 0, BOUT_W0 = 1, BOUT_PSI = 2 };
u64 bstep_red_doubles(int nL);
// T[l][j] = T[j][l] = <w_l|D> and S[l][j] = S[j][l] = <w_l|w_j> for l <= j
void bstep_dots(hipStream_t st, const BInst* d, int n, int j, int nL);
// kind 0: D -= T[l][j] w_l;  kind 1: D += x[l] w_l
void bstep_axpy(hipStream_t st, const BInst* d, int n, int l, int j, int kind, u64 max_cap);
// Eq. 11 on the selection's output vector
void bstep_normalise(hipStream_t st, const BInst* d, int n, int out_kind, int j, u64 max_cap);
void bstep_fill_zero(hipStream_t st, const BInst* d, int n, u64 max_ndet);
void bstep_geneig(hipStream_t st, const BInst* d, int n, int nL);
void bstep_inc_blk(hipStream_t st, const BInst* d, int n);
// Exclusive scans of u64 counts, one per job: out[i] = sum in[0..i), *total = sum (may be null).
struct BScanJob {
    const u64* in;
    u64* out;
    u64 n;
    u64* bsum;  // scan_block_sums(n) words
    u64* total;
};
void bscan_u64(hipStream_t st, const BScanJob* d_jobs, int n_jobs, u64 max_n);
// select_topm of every instance's dense accumulator (zeroed on the way unless
// !zero) into the out_kind vector, keeping M entries (all != 0: every nonzero entry);
// scan jobs: the accumulator's chunk counts (total to st->count_cand) and the
// candidate list's (total to st2->count_out).
void bstep_select(hipStream_t st, const BInst* d, int n, int out_kind, int j, u64 max_ndet, int num_cu, int band,
                  int max_ndig, const BScanJob* d_scan_dense, const BScanJob* d_scan_list, int all, bool zero = true);

// Select the M largest (|c|, then lower rank) nonzero candidates and write them
// by ascending rank to (out_rank, out_amp); *out_count_dev receives the count.
// If zero_dense, the dense source is cleared to 0.0 in the same pass.
// M == UINT64_MAX keeps all nonzero candidates.
void select_topm(sfci_problem* P, const CandSrc& src, u64 M, u64* out_rank, double* out_amp, u64* out_count_dev,
                 bool zero_dense);
// Two-phase form: prepare (selection levels + counts; the count goes to
// *count_dev), then write.  The state lives in the problem's workspace, so no
// other selection may run in between.
void select_prepare(sfci_problem* P, const CandSrc& src, u64 M, u64* count_dev);
void select_write(sfci_problem* P, const CandSrc& src, u64* out_rank, double* out_amp, bool zero_dense);
// The same two phases on a candidate list with caller-given working memory
// (no allocation): the state, select_chunks(lcap) per-chunk counts and
// scan_block_sums(select_chunks(lcap)) scan sums.
struct SelWs {
    SelState* st;
    u64* cnt;
    u64* bsum;
};
u64 select_chunks(u64 n_upper);
void select_prepare_ws(sfci_problem* P, const CandSrc& src, u64 M, u64* count_dev, const SelWs& ws);
void select_write_ws(sfci_problem* P, const CandSrc& src, u64* out_rank, double* out_amp, const SelWs& ws);

// ---- sort path (sortpath.hip) ----
// sigma = H v by stable sort + in-order segmented sum; result sorted by rank,
// zeros dropped, in (out_rank, out_amp) with *out_count_dev; returns false if
// the result would exceed out_cap (then *out_count_dev = needed).
// eps > 0 drops sums with |sum| < eps (screening, Sec. 3).
void sigma_sorted(sfci_problem* P, const SigmaLaunch& v, u64 out_cap, u64* out_rank, double* out_amp,
                  u64* out_count_dev, u64* emitted_dev, double eps = 0.0);
// Pass-by-pass form: a pass covers a range [alo, ahi) of target alpha ranks
// (ascending, disjoint).  Before a pass's reduction the sink says where its
// entries go (appended at out[*base_dev ...], *base_dev advanced by their
// number); after it, the sink may consume them.  tup_cap = 0: sized from free
// memory.  Returns the number of passes run.
struct SortPassOut {
    u64* r;
    double* a;
    u64 cap;
    u64* base_dev;
};
struct SortPassSink {
    virtual SortPassOut begin(u64 alo, u64 ahi, u64 tuples) = 0;
    virtual void end(u64 alo, u64 ahi) = 0;
    virtual ~SortPassSink() = default;
};
// Device bytes per sort-path tuple over the emission, sort and reduction buffers.
constexpr u64 SFCI_SORT_TUPLE_BYTES = 2 * (sizeof(u64) + sizeof(double)) + sizeof(double) + sizeof(u64);
u64 sort_tuple_cap(sfci_problem* P);
u64 sigma_sorted_passes(sfci_problem* P, const SigmaLaunch& v, SortPassSink& sink, u64* emitted_dev, u64 tup_cap,
                        double eps);
// The same passes with target-row-driven emission (rowpass.hip): per-row
// tuple counts once per call, then per pass only the (target row, source
// row) pairs that land in it.
u64 sigma_rowpass(sfci_problem* P, const SigmaLaunch& v, SortPassSink& sink, u64* emitted_dev, u64 tup_cap,
                  double eps);
// K = u64 or u32.
template <class K>
void radix_sort_pairs(sfci_problem* P, K* k1, double* v1, K* k2, double* v2, u64 n, int kbits, K** k_out,
                      double** v_out);
int key_bits(u64 maxval);
// Entries per radix-sort tile.
constexpr u64 SFCI_SORT_TILE = 4096;
// Stable sort of pass-local keys (target row - lo) * N_beta + beta rank whose
// entries are already grouped by target row in ascending row order: only the
// beta rank is sorted, inside each row.  tpre / ttile hold the entries and the
// tiles (ceil(entries / SFCI_SORT_TILE)) before every row of the space,
// ntiles = ttile[hi] - ttile[lo]; tile_row has room for ntiles entries.
void radix_sort_rows(sfci_problem* P, u32* k1, double* v1, u32* k2, double* v2, u64 n, const u64* tpre,
                     const u64* ttile, u64 lo, u64 hi, u64 ntiles, u32* tile_row, u32** k_out, double** v_out);
template <class K>
void segmented_sum_append(sfci_problem* P, const K* keys, const double* vals, u64 n, u64 key_base, double eps,
                          u64* out_base_dev, u64 out_cap, u64* out_r, double* out_a);

// ---- Lanczos vector ops (lanczos.hip) ----
void launch_dot_dense(sfci_problem* P, const u64* r, const double* a, const u64* nnz, u64 cap, const double* D,
                      double* out1, double* out2, bool ordered);
// The same sum with Y[i] (the y value already gathered for entry i) in place of D[r[i]].
void launch_dot_gathered(sfci_problem* P, const double* a, const u64* nnz, u64 cap, const double* Y, double* out1,
                         double* out2, bool ordered);
// sum of x[0..*nnz) (ordered: strictly in index order) and sum of squares
void launch_sum(sfci_problem* P, const double* x, const u64* nnz, u64 cap, double* out, bool ordered);
void launch_sumsq(sfci_problem* P, const double* a, const u64* nnz, u64 cap, double* out, bool ordered);
void launch_dot_sparse(sfci_problem* P, const u64* xr, const double* xa, const u64* xn, u64 xcap, const u64* yr,
                       const double* ya, const u64* yn, double* out1, double* out2, bool ordered);
void launch_axpy_scatter(sfci_problem* P, double* D, const u64* r, const double* a, const u64* nnz, u64 cap,
                         const double* coef, double sign);
void launch_normalise(sfci_problem* P, double* a, const u64* nnz, u64 cap, bool ordered, double* part_ws = nullptr);
// doubles of working memory launch_normalise needs (part_ws)
u64 normalise_ws_doubles();
void launch_scatter_set(sfci_problem* P, double* D, const u64* r, const double* a, const u64* nnz, u64 cap);
// energy_slot[blk ? *blk : 0] receives lambda (blk: device block index, may be null)
void launch_geneig_full(sfci_problem* P, int m, const double* T, const double* S, double* lambda, double* x,
                        double* energy_slot, int* status, const int* blk = nullptr);
void launch_inc_int(sfci_problem* P, int* p);
void launch_add_u64(sfci_problem* P, u64* dst, const u64* src);  // *dst += *src
void launch_div_by_sumsq(sfci_problem* P, const double* a, const u64* nnz, u64 cap, double* out);
void launch_copy_vec(sfci_problem* P, const u64* r, const double* a, const u64* nnz, u64 cap, u64* r2, double* a2,
                     u64* nnz2);

int sfci_set_error(int code, const std::string& msg);

// ---- host helpers shared by the ABI files (abi.hip) ----
void sfci_sync(sfci_problem* P);
void launch_set_u64(sfci_problem* P, u64* p, u64 v);
void validate_vec(sfci_problem* P, const u64* r, u64 n);  // throws on out-of-range or unsorted ranks
bool ensure_dense(sfci_problem* P);                       // allocates the zeroed N_det accumulator if it fits
void dense_sigma(sfci_problem* P, const SigmaLaunch& sl, int dedup, unsigned long long* emitted, double eps = 0.0);
// Screening (Sec. 3): D[i] = 0 where 0 < |D[i]| < eps.
void launch_screen(sfci_problem* P, double* D, u64 n, double eps);

// Device time of a sequence of bracketed regions on a stream (HIP events).
struct EventTimer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    bool on = false;
    void begin(hipStream_t s) {
        if (!on) return;
        hipEvent_t a, b;
        SFCI_CHECK_HIP(hipEventCreate(&a));
        SFCI_CHECK_HIP(hipEventCreate(&b));
        SFCI_CHECK_HIP(hipEventRecord(a, s));
        ev.push_back({a, b});
    }
    void end(hipStream_t s) {
        if (!on) return;
        SFCI_CHECK_HIP(hipEventRecord(ev.back().second, s));
    }
    double total_ms() {
        double t = 0.0;
        for (auto& p : ev) {
            float ms = 0.f;
            SFCI_CHECK_HIP(hipEventElapsedTime(&ms, p.first, p.second));
            t += ms;
        }
        return t;
    }
    ~EventTimer() {
        for (auto& p : ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
};

// ---- list-based iteration and truncated sigma without an N_det array (listlz.hip) ----
// sigma = H v in passes of target alpha rows (the sort path's, or with
// tiles_ok the tile kernel's slices when the per-sigma cost rule picks them);
// the top-M (tie rule) sorted by rank into out when it fits out_cap.  Returns
// the selected count; *distinct_host (may be NULL) receives the number of
// distinct nonzero entries.
u64 sigma_list_topm(sfci_problem* P, const SigmaLaunch& v, u64 M, u64* out_rank, double* out_amp, u64 out_cap,
                    u64* emitted_dev, u64* distinct_host, bool tiles_ok, double eps = 0.0);
// Fast mode's per-sigma choice between the tile kernel's slices (true) and
// the sort path, from the input's size (SFCI_LIST_SIGMA=tile|sort forces one).
bool list_sigma_tiles(sfci_problem* P, u64 nnz);
// sigma = H v in full through the sort path's passes, no N_det array: the
// nonzero entries sorted by rank in list_ws.Rr / Ra; returns their number.
u64 sigma_list_full(sfci_problem* P, const SigmaLaunch& v, u64* emitted_dev, u64** r, double** a);
// H v in full as a rank-sorted list (zeros dropped): the sort path when
// deterministic or when the N_det array does not fit, else the dense tile
// kernel compacted in rank order (the accumulator is zero again afterwards).
// The list lives in the problem's workspace until the next such call;
// *cnt_dev receives its length, which is also returned.
u64 sigma_full_list(sfci_problem* P, const SigmaLaunch& sl, bool det, u64* emitted, u64** yr, double** ya,
                    u64* cnt_dev);
// The basis and the per-block outputs the iteration writes (device).
struct ListBasis {
    u64 cap;        // entries per basis vector
    u64* Wr;        // n_L x cap ranks
    double* Wa;     // n_L x cap amplitudes
    u64* sc;        // [0, n_L) nnz per vector, [32] emitted-term counter
    double *Td, *Sd, *xd, *lam, *energies_d;
    int* status_d;
    u64* nnz_hist;  // nnz of each sigma input, block after block
};
// w_0 must already hold the normalised start vector.  *psi_n_out receives the
// last Psi's length; it is copied to psi_out when it fits.
void lanczos_list(sfci_problem* P, const sfci_lanczos_opts* o, const ListBasis& B, sfci_svec* psi_out, u64* psi_n_out,
                  u64* sigma_calls, EventTimer& tsig, int* blocks_run);
// Halting test of Sec. 2.1 after block b (energies on the device): true when
// o->conv_eps > 0, b >= 1 and E(b-1) - E(b) < conv_eps.  Synchronises when it
// has to look.
bool halt_after_block(sfci_problem* P, const sfci_lanczos_opts* o, const double* energies_d, int b);

// Device-resident sparse vector with a device nnz (Lanczos basis storage).
struct DVec {
    u64* r = nullptr;
    double* a = nullptr;
    u64* nnz = nullptr;
    u64 cap = 0;
};
