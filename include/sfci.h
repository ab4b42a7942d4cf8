/* sfci.h -- C ABI of the MI355X sparse-FCI hot path (libsfci.so).
 *
 * What it computes (Wang, "Sparse Full Configuration Interaction",
 * arXiv 2312.01846):
 *   sigma = H v for the second-quantized Hamiltonian
 *     H = sum_pq h_pq sum_s a+_ps a_qs
 *       + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs
 *   applied to a sparse vector of Slater determinants (Sec. 2.2: a sparse
 *   vector is a set of (index, amplitude) pairs; matrix elements are
 *   generated on the fly for single and double excitations, Sec. 3), the
 *   determinant index being the combinatorial hash of Sec. 2.2, Eq. 12,
 *   truncated to the M largest amplitudes (Sec. 2.1, Eqs. 10-11), and the
 *   truncated-Lanczos iteration built on it (Sec. 2.1).
 *
 * Conventions shared by every call:
 *   - A spin string is an n-bit mask (bit p set = spatial orbital p occupied),
 *     1 <= n <= 32.  String rank r = sum_{t=1..k} C(c_t, t) over the ascending
 *     0-based occupied orbitals c_t (Eq. 12).  Determinant rank
 *     R = r_alpha * C(n, n_beta) + r_beta (alpha-major), 0 <= R < N_det.
 *   - Integrals are FP64, real, row-major: h[p*n+q]; eri[((p*n+q)*n+r)*n+s]
 *     = (pq|rs) in chemist notation.  h must be exactly symmetric and eri
 *     exactly 8-fold symmetric (bitwise), else SFCI_E_NOTSYM.
 *   - Phase convention: spin orbitals ordered all-alpha then all-beta,
 *     orbital ascending (Jordan-Wigner).
 *   - Sparse vectors (sfci_svec) are caller-owned DEVICE arrays: rank[] u64
 *     strictly ascending (unique), amp[] f64; nnz entries used, capacity
 *     allocated.  The library never frees caller memory.
 *   - Every call returns sfci_status; SFCI_OK = 0, errors are negative and
 *     leave the problem handle usable.  sfci_last_error() returns a
 *     thread-local message for the last failing call on this thread.
 *   - All device work is issued on the stream given at sfci_problem_create.
 *     Calls that return a host count (nnz) synchronise that stream.
 *   - The library allocates its own device workspace (dense FP64 accumulator
 *     of N_det slots when it fits, selection and sort buffers) on first use
 *     and keeps it until sfci_problem_destroy.
 */
#ifndef SFCI_H
#define SFCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFCI_OK = 0,
    SFCI_E_ARG = -1,         /* NULL pointer, bad size or bad option */
    SFCI_E_RANGE = -2,       /* rank >= N_det, or N_det does not fit in 64 bits */
    SFCI_E_DUP = -3,         /* input ranks not strictly ascending */
    SFCI_E_CAPACITY = -4,    /* output capacity too small; out->nnz holds the size needed */
    SFCI_E_NOMEM = -5,       /* device allocation failed */
    SFCI_E_DEVICE = -6,      /* HIP runtime error */
    SFCI_E_NOTSYM = -7,      /* h or eri not exactly symmetric */
    SFCI_E_UNSUPPORTED = -8  /* n > 32, or a mode not available for this space */
} sfci_status;

typedef struct sfci_problem sfci_problem; /* opaque; owns device copies of integrals and tables */

typedef struct {
    int32_t n_orb;   /* spatial orbitals, 1..32 */
    int32_t n_alpha; /* alpha electrons, 0..n_orb */
    int32_t n_beta;  /* beta electrons, 0..n_orb */
} sfci_space;

typedef struct {
    uint64_t* rank;    /* device, strictly ascending */
    double* amp;       /* device */
    uint64_t nnz;      /* entries in use (host value) */
    uint64_t capacity; /* entries allocated */
} sfci_svec;

/* Truncation to M (Sec. 2.1, Eqs. 10-11: each basis vector keeps N_d = M
 * entries, the largest in magnitude).  Nonzero entries are ordered by |c|
 * descending and exact ties by rank ascending (the paper leaves ties open);
 * the first min(M, nonzero) are kept.  This is the default everywhere.
 *
 * tie_band = 1 in the options switches on an extension that is not the
 * paper's rule: every further entry whose |c| is >= (1 - 2^-36) times the M-th
 * |c| is kept too, so partners of equal magnitude in exact arithmetic (e.g.
 * alpha/beta-exchanged determinants when n_alpha = n_beta) are not split by
 * rounding -- unless that adds more than SFCI_TIE_SLACK entries, in which
 * case exactly M are kept.  With the band a truncated vector holds at most
 * M + SFCI_TIE_SLACK entries; size outputs accordingly. */
#define SFCI_TIE_SLACK 256

/* Deduplication of the intermediate elements (Sec. 2.2 merge step). */
enum {
    SFCI_DEDUP_AUTO = 0,         /* dense if 8*N_det bytes fit the device, else sort */
    SFCI_DEDUP_DENSE = 1,        /* dense N_det array, target-owned tiles accumulated in LDS (order not fixed) */
    SFCI_DEDUP_SORT = 2,         /* stable radix sort + in-order segmented sum (deterministic) */
    SFCI_DEDUP_DENSE_ATOMIC = 3  /* dense N_det array, one FP64 global atomic per term (the first GPU path) */
};

typedef struct {
    uint64_t M;        /* keep the M largest |sigma_k| (ties: see SFCI_TIE_SLACK); UINT64_MAX = all */
    int32_t dedup;     /* SFCI_DEDUP_* */
    int32_t deterministic; /* 1: sort dedup and ordered reductions, bit-reproducible */
    double screen_eps; /* Sec. 3: merged entries with |sigma_k| < screen_eps are dropped before the
                          truncation (the paper uses 5e-5); 0 = off */
    int32_t tie_band;  /* 1: the truncation extension described at SFCI_TIE_SLACK; 0 = the paper's rule */
    int32_t reserved;  /* must be 0 */
    double excite_eps; /* excitation screen (the heat-bath idea Sec. 4 names for future work): a double
                          excitation's term H_ki v_i with |H_ki v_i| < excite_eps is not generated; singles
                          and the diagonal always are.  0 = off */
} sfci_sigma_opts;

typedef struct {
    uint64_t terms_enumerated; /* (source, excitation) pairs visited */
    uint64_t terms_emitted;    /* of those, with a nonzero element */
    uint64_t candidates;       /* distinct nonzero entries of sigma before truncation */
    double ms;                 /* device time of the call (HIP events) */
} sfci_sigma_stats;

/* N_det = C(n, n_alpha) * C(n, n_beta).  SFCI_E_RANGE if it exceeds 2^64-1. */
sfci_status sfci_space_size(const sfci_space* space, uint64_t* n_det);

/* Validate and upload the integrals (host pointers h[n*n], eri[n^4]).
 * stream: a hipStream_t (NULL = default stream).  *out receives the handle. */
sfci_status sfci_problem_create(const sfci_space* space, const double* h, const double* eri, void* stream,
                                sfci_problem** out);
sfci_status sfci_problem_destroy(sfci_problem* prob);

/* Eq. 12 on device arrays: rank[i] = r(a_bits[i]) * C(n, n_beta) + r(b_bits[i]).
 * Strings must have n_alpha / n_beta bits set within the low n bits, else SFCI_E_ARG
 * (checked on device; the call synchronises to report it). */
sfci_status sfci_rank(sfci_problem* prob, const uint64_t* a_bits, const uint64_t* b_bits, uint64_t count,
                      uint64_t* rank);
/* Inverse of sfci_rank.  SFCI_E_RANGE if some rank >= N_det. */
sfci_status sfci_unrank(sfci_problem* prob, const uint64_t* rank, uint64_t count, uint64_t* a_bits,
                        uint64_t* b_bits);

/* sigma = H v, then the M largest entries (Eqs. 10-11 order, not normalised),
 * written to out sorted by rank.  v must be strictly ascending with ranks < N_det.
 * When the N_det accumulator does not fit the device, sigma is formed in
 * passes of target alpha rows into a running top-M candidate list (the sort
 * path; in fast mode the tile kernel's row slices once the input is large).
 * On SFCI_E_CAPACITY, out->nnz is set to the size needed and nothing is written.
 * stats may be NULL.  Synchronises the stream (returns out->nnz). */
sfci_status sfci_sigma(sfci_problem* prob, const sfci_svec* v, const sfci_sigma_opts* opts, sfci_svec* out,
                       sfci_sigma_stats* stats);

/* Truncation alone (Eqs. 10-11 without the division): the M largest |amp| of v
 * (ties: see SFCI_TIE_SLACK), by ascending rank, into out.  Zero amplitudes are dropped.
 * normalise != 0 divides the kept amplitudes by their 2-norm (Eq. 11).
 * tie_band: as in sfci_sigma_opts. */
sfci_status sfci_topm(sfci_problem* prob, const sfci_svec* v, uint64_t M, int32_t normalise, int32_t tie_band,
                      sfci_svec* out);

typedef struct {
    uint64_t M;            /* N_d of Sec. 2.1: entries kept per basis vector (at most M + SFCI_TIE_SLACK); UINT64_MAX = all */
    int32_t n_L;           /* basis vectors per block (N_L), 1..32 */
    int32_t n_iter;        /* sigma applications; n_iter / n_L blocks are run */
    int32_t deterministic; /* 1: sort dedup and ordered reductions */
    int32_t dedup;         /* SFCI_DEDUP_* (ignored when deterministic) */
    double screen_eps;     /* Sec. 3: entries of H w_j with |c| < eps are dropped before T, Eq. 10
                              and the truncation (the paper uses 5e-5); 0 = off */
    int32_t no_dense;      /* 1: keep every vector as a rank list and never allocate the N_det array
                              (sort path, alpha-range passes); implied when 8 N_det bytes do not fit */
    int32_t autotune;      /* batched fast mode: 1 = choose the tile kernel's work sizes (beta singles and
                              beta-beta doubles per work unit, workgroups per CU) by timing candidates on the
                              last eager sigma step, once per batch; later calls reuse the choice */
    double conv_eps;       /* Sec. 2.1 halting: > 0 stops after block n >= 1 once E(n-1) - E(n) < conv_eps
                              (the signed change, as the paper writes it); 0 = run n_iter / n_L blocks.
                              Not available in the batched call (SFCI_E_UNSUPPORTED there). */
    int32_t tie_band;      /* 1: the truncation extension described at SFCI_TIE_SLACK; 0 = the paper's rule */
    int32_t reserved;      /* must be 0 */
    double excite_eps;     /* excitation screen of every H w_j, as in sfci_sigma_opts; 0 = off.  The
                              gradients of the batched call are those of the unscreened energy at Psi. */
} sfci_lanczos_opts;

typedef struct {
    uint64_t sigma_calls;      /* sigma applications run */
    uint64_t terms_enumerated; /* (source, excitation) pairs visited over all sigma calls */
    uint64_t terms_emitted;    /* of those, with a nonzero element */
    double sigma_ms;           /* summed device time of the sigma expansion kernels (HIP events) */
    double total_ms;           /* device time of the whole call */
    int32_t blocks_run;        /* blocks run (fewer than n_iter / n_L when conv_eps halted the run) */
    int32_t reserved;
} sfci_lanczos_stats;

/* The SFCI iteration of Sec. 2.1 from start vector v0 (normalised internally).
 * energies[b] (host, n_iter/n_L entries) receives each block's lowest
 * generalized eigenvalue of (T, S); blocks not run (conv_eps halting) get
 * NaN.  psi_out (device, may be NULL) receives the
 * last block's Psi = sum_j x_j w_j before truncation; SFCI_E_CAPACITY (with
 * psi_out->nnz = needed) if it does not fit, energies still valid.
 * T_out/S_out (host, may be NULL) receive each block's n_L x n_L matrices,
 * block after block.  stats may be NULL. */
sfci_status sfci_lanczos(sfci_problem* prob, const sfci_svec* v0, const sfci_lanczos_opts* opts, double* energies,
                         sfci_svec* psi_out, double* T_out, double* S_out, sfci_lanczos_stats* stats);

/* Excited states (Sec. 4: project the previously found eigenvectors out of
 * the effective Hamiltonian): the iteration of sfci_lanczos on P H P with
 * P y = y - sum_i Psi_i <Psi_i|y> / <Psi_i|Psi_i>, roots[0..n_roots) the found
 * eigenvectors (device vectors, ascending ranks, any norm, applied in order).
 * Each sigma becomes H w - sum_i c_i H Psi_i (c_i = <Psi_i|w>/<Psi_i|Psi_i>,
 * H Psi_i computed once) followed by P; the start vector is projected and
 * truncated to M; the block-end Psi is projected before its truncation, and
 * psi_out receives the projected Psi.  energies: the lowest eigenvalue of each
 * block's (T, S), i.e. the next state.  n_roots = 0 is sfci_lanczos.  Needs
 * the dense accumulator (SFCI_E_UNSUPPORTED with no_dense or when it does not
 * fit); at most SFCI_MAX_ROOTS roots. */
#define SFCI_MAX_ROOTS 8
sfci_status sfci_lanczos_roots(sfci_problem* prob, const sfci_svec* v0, const sfci_lanczos_opts* opts,
                               const sfci_svec* roots, int32_t n_roots, double* energies, sfci_svec* psi_out,
                               double* T_out, double* S_out, sfci_lanczos_stats* stats);

/* Backward of sigma = H(h, eri) v for a cotangent sbar (device vectors):
 *   v_bar[i] = sum_k H_ki sbar_k for the entries i of v (device, nnz(v) doubles, may be NULL),
 *   dh  = sym(gamma),  gamma_pq = sum_ki sbar_k v_i <k|E_pq|i>      (device n*n, may be NULL),
 *   deri = the 8-fold symmetrisation of Gamma/2, with
 *          Gamma_pqrs = sum_ki sbar_k v_i <k| sum_st a+_ps a+_rt a_st a_qs |i>  (device n^4, may be NULL),
 * i.e. the gradients of sbar^T H v along symmetric perturbations of h and eri.
 * Outputs are overwritten.  Asynchronous. */
sfci_status sfci_sigma_backward(sfci_problem* prob, const sfci_svec* v, const sfci_svec* sbar, double* v_bar,
                                double* dh, double* deri);

/* Second-order Epstein-Nesbet correction of a variational vector Psi (device
 * vector, strictly ascending ranks, not necessarily normalised): the
 * perturbative correction the paper names for future work (the F2 discussion
 * in its results).  Diagonal partitioning:
 *   *e0 = <Psi|H|Psi> / <Psi|Psi>,
 *   *e2 = sum over determinants k outside supp(Psi) of (H Psi)_k^2 / (*e0 - H_kk),
 *         divided by <Psi|Psi>;
 *   *n_external (may be NULL) = number of those k with (H Psi)_k != 0.
 * deterministic != 0: H Psi from the sort path and every sum in ascending
 * rank (bit-reproducible); else the dense tile kernel and tree reductions.
 * Needs the full H Psi as a list on the device (distinct entries x 16 B).
 * Synchronises.  SFCI_E_ARG for an empty or zero-norm Psi. */
sfci_status sfci_pt2(sfci_problem* prob, const sfci_svec* psi, int32_t deterministic, double* e0, double* e2,
                     uint64_t* n_external);

/* The energy of a vector and its integral gradients at fixed Psi (device
 * vector, strictly ascending ranks, any nonzero norm):
 *   *energy (host) = <Psi|H|Psi> / <Psi|Psi>   (Sec. 2.1, Eq. 9);
 *   dh (device n*n, may be NULL) and deri (device n^4, may be NULL) = the
 *   gradients of that quotient along symmetric perturbations of h and eri
 *   (an extension, not in the paper), i.e. sfci_sigma_backward with v = Psi
 *   and sbar = Psi / <Psi|Psi>; at an eigenvector these are the energy's
 *   Hellmann-Feynman derivatives.
 * deterministic != 0: H Psi from the sort path and the energy's sums in
 * ascending rank (bit-reproducible); else the dense tile kernel and tree
 * reductions.  The gradients need the dense array (SFCI_E_UNSUPPORTED when
 * it does not fit).  Synchronises.  SFCI_E_ARG for an empty or zero-norm Psi. */
sfci_status sfci_energy_gradients(sfci_problem* prob, const sfci_svec* psi, int32_t deterministic, double* energy,
                                  double* dh, double* deri);

/* ---- batched iteration (an extension, not in the paper) ----
 * Many instances (e.g. points along a bond-stretch curve) with uneven
 * truncations M_k, and possibly different orbital counts, iterate together:
 * each sigma application of all instances is one launch of the target-owned
 * tile kernel, and after one eager block every iteration step (its
 * preparation, the tile launch and the vector operations) is replayed from
 * one captured hipGraph.  The batch keeps those graphs: a later call with the
 * same truncations, options and start-vector sizes, made while no library
 * buffer has been freed or regrown in between, replays them from its first
 * block on.  All problems must share one device and stream. */
typedef struct sfci_batch sfci_batch;

typedef struct {
    double fwd_ms;              /* device time of the iteration (all blocks) */
    double bwd_ms;              /* device time of the gradient pass */
    double sigma_ms;            /* sum over the sigma launches: HIP events around each eager launch and
                                   event-record nodes around the launch inside each replayed step graph */
    uint64_t terms_emitted;     /* nonzero-element terms over all sigma applications and instances */
    uint64_t nnz_in_total;      /* input entries over all sigma applications and instances */
    uint64_t sigma_calls;       /* sigma applications per instance (= launches when batched_sigma) */
    uint64_t psi_nnz_total;     /* entries of the final Psi over all instances */
    int32_t graph_replayed_blocks;
    int32_t batched_sigma;      /* 1: one launch per step served every instance */
    int32_t tune_trials;        /* candidate launches timed by this call (0: none, or the batch's earlier choice) */
    uint32_t tune_b1_chunk;     /* work sizes the sigma launches used (0 = built-in default) */
    uint32_t tune_bb_chunk;
    uint32_t tune_per_cu;
    double tune_default_ms;     /* trial time of the default sizes and of the chosen ones (when tuned) */
    double tune_best_ms;
    int32_t sigma_in_graph;     /* 1: each replayed step was one graph, the tile launch inside it */
    int32_t graphs_reused;      /* 1: the step graphs came from an earlier call, every block replayed */
} sfci_batch_stats;

/* probs: n_inst problem handles (kept, not owned). */
sfci_status sfci_batch_create(int32_t n_inst, sfci_problem* const* probs, sfci_batch** out);
sfci_status sfci_batch_destroy(sfci_batch* batch);

/* The SFCI iteration (as sfci_lanczos) for every instance k from v0s[k]
 * (device vectors) with truncation Ms[k]; opts->M is ignored.
 * energies (host, n_inst * (n_iter/n_L)) receives the block energies,
 * instance-major.  dh_all / deri_all (device, may be NULL) receive, per
 * instance in order, dE/dh (n_k^2) and dE/d(pq|rs) (n_k^4) of
 * E = <Psi|H|Psi>/<Psi|Psi> at the final untruncated Psi, symmetrised as in
 * sfci_sigma_backward.  stats may be NULL. */
sfci_status sfci_batch_lanczos(sfci_batch* batch, const sfci_svec* v0s, const uint64_t* Ms,
                               const sfci_lanczos_opts* opts, double* energies, double* dh_all, double* deri_all,
                               sfci_batch_stats* stats);

/* Message for the last failing call on this thread ("" if none). */
const char* sfci_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SFCI_H */
