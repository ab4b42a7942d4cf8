// Batched SFCI: many problem instances (points along a bond-stretch curve,
// uneven truncations M_k, possibly different orbital counts) iterate
// together.  Per sigma application the work of all instances is drained by
// ONE launch of the target-owned tile kernel; the rest of an iteration (T/S
// gathers, Eq. 10, truncation, Eq. 11) is issued per instance on the shared
// stream.  After one eager block has sized and allocated every buffer, each
// iteration step (preparation, the tile launch, the vector operations) and
// the block end are captured into hipGraphs and replayed; the batch keeps
// them, and a later call with the same signature (instances, buffers,
// truncations, options, work sizes) replays them from its first block on.
// After the last block each instance's gradient of E = <Psi|H|Psi>/<Psi|Psi>
// with respect to h and (pq|rs) is computed at fixed Psi.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sfci.h"
#include "sfci_internal.h"

struct sfci_batch {
    int n = 0;
    std::vector<sfci_problem*> P;
    hipStream_t stream = nullptr;      // the problems' stream
    hipStream_t own = nullptr;         // capture-capable stream used during a batched run
    std::vector<DevBuf> descs;  // per iteration step j: the n instance descriptions
    DevBuf prefix, counter, scratch;
    DevBuf binst, bscan;        // batched vector steps: the instances (BInst), the two scans' jobs
    RowTileGradWs grad_ws;
    // per-instance chains run on these streams (forked from and joined to `own`)
    std::vector<hipStream_t> aux;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    // work sizes of the sigma tile launches (chosen by autotuning, kept across calls)
    RowTileTune tune;
    bool tuned = false;
    // Step graphs (one per iteration step) and the block-end graph, kept for
    // later calls.  A call whose instances, buffers, truncations, options and
    // work sizes (gsig) equal those of the capture, with no library buffer
    // freed since (gepoch), replays them from its first block on.
    std::vector<hipGraphExec_t> gstep;
    hipGraphExec_t gend = nullptr;
    std::vector<hipEvent_t> gev;  // recorded by event nodes inside the step graphs: [2j], [2j+1] around step j's sigma
    std::vector<u64> gsig;
    u64 gepoch = 0;
    void drop_graphs() {
        if (own) (void)hipStreamSynchronize(own);
        for (auto x : gstep) (void)hipGraphExecDestroy(x);
        gstep.clear();
        if (gend) (void)hipGraphExecDestroy(gend);
        gend = nullptr;
        for (auto e : gev)
            if (e) (void)hipEventDestroy(e);
        gev.clear();
        gsig.clear();
    }
};

namespace {

struct Inst {
    sfci_problem* P;
    u64 M, cap, tps;
    u64* Wr;
    double* Wa;
    u64* sc;       // [0..nL) nnz of w_j, [32] emitted, [33] list count, [34] psi count, [35] sigma input entries, [36] transposed Psi count
    double* T;     // one block: T then S (n_L x n_L each)
    double* S;
    double* x;
    double* lam;
    double* energies;  // n_blocks
    int* blk;
    int* status;
    u64* psi_r;
    double* psi_a;
    double* sbar;
    u64 lcap;
    u64* lr;
    double* la;
    DVec W(int j) const { return DVec{Wr + (size_t)j * cap, Wa + (size_t)j * cap, sc + j, cap}; }
};

// Largest workgroups-per-CU multiple a tuning candidate may ask for.
constexpr unsigned kTuneMaxPerCu = 4;

#define SFCI_GUARD_BEGIN try {
#define SFCI_GUARD_END                                               \
    }                                                                \
    catch (const sfci_error& e) {                                    \
        return (sfci_status)sfci_set_error(e.code, e.msg);           \
    }                                                                \
    catch (const std::exception& e) {                                \
        return (sfci_status)sfci_set_error(SFCI_E_DEVICE, e.what()); \
    }

}  // namespace

extern "C" {

sfci_status sfci_batch_create(int32_t n_inst, sfci_problem* const* probs, sfci_batch** out) {
    SFCI_GUARD_BEGIN
    if (n_inst < 1 || !probs || !out) return (sfci_status)sfci_set_error(SFCI_E_ARG, "need n_inst >= 1 problems");
    for (int k = 0; k < n_inst; ++k) {
        if (!probs[k]) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL problem");
        if (probs[k]->stream != probs[0]->stream || probs[k]->device != probs[0]->device)
            return (sfci_status)sfci_set_error(SFCI_E_ARG, "batched problems must share one device and one stream");
        for (int l = 0; l < k; ++l)
            if (probs[l] == probs[k])
                return (sfci_status)sfci_set_error(SFCI_E_ARG, "a problem appears twice (instances own their workspaces)");
    }
    sfci_batch* B = new sfci_batch();
    B->n = n_inst;
    B->P.assign(probs, probs + n_inst);
    B->stream = probs[0]->stream;
    SFCI_CHECK_HIP(hipStreamCreateWithFlags(&B->own, hipStreamNonBlocking));
    const int S = std::min(n_inst, 4);
    B->aux.assign(S, nullptr);
    B->ev_join.assign(S, nullptr);
    for (int s = 0; s < S; ++s) {
        SFCI_CHECK_HIP(hipStreamCreateWithFlags(&B->aux[s], hipStreamNonBlocking));
        SFCI_CHECK_HIP(hipEventCreateWithFlags(&B->ev_join[s], hipEventDisableTiming));
    }
    SFCI_CHECK_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    *out = B;
    return SFCI_OK;
    SFCI_GUARD_END
}

sfci_status sfci_batch_destroy(sfci_batch* B) {
    if (!B) return SFCI_OK;
    (void)hipStreamSynchronize(B->stream);
    B->drop_graphs();
    for (auto& d : B->descs) d.release();
    B->prefix.release();
    B->binst.release();
    B->bscan.release();
    B->counter.release();
    B->scratch.release();
    B->grad_ws.release();
    for (auto s : B->aux)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : B->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->own) (void)hipStreamDestroy(B->own);
    delete B;
    return SFCI_OK;
}

sfci_status sfci_batch_lanczos(sfci_batch* B, const sfci_svec* v0s, const uint64_t* Ms, const sfci_lanczos_opts* o,
                               double* energies, double* dh_all, double* deri_all, sfci_batch_stats* stats) {
    SFCI_GUARD_BEGIN
    if (!B || !v0s || !Ms || !o || !energies) return (sfci_status)sfci_set_error(SFCI_E_ARG, "NULL argument");
    if (o->n_L < 1 || o->n_L > 32 || o->n_iter < o->n_L)
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "need 1 <= n_L <= 32 and n_iter >= n_L");
    if (o->no_dense)
        return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "the batched iteration keeps dense accumulators");
    if (o->conv_eps != 0.0)
        return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED,
                                           "the batched iteration runs n_iter / n_L blocks (no conv_eps halting)");
    if (!(o->screen_eps >= 0.0) || !(o->excite_eps >= 0.0))
        return (sfci_status)sfci_set_error(SFCI_E_ARG, "screen_eps and excite_eps must be >= 0");
    const int nL = o->n_L, nblk = o->n_iter / nL, n = B->n;
    const bool det = o->deterministic != 0;
    const bool use_graph = !det && (o->dedup != SFCI_DEDUP_DENSE_ATOMIC);
    // Run on the batch's own stream (graph capture is not possible on the
    // legacy default stream); the problems' stream is restored on exit.
    SFCI_CHECK_HIP(hipStreamSynchronize(B->stream));
    hipStream_t st = B->own;
    struct Restore {
        sfci_batch* B;
        ~Restore() {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(B->own, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
                hipGraph_t g = nullptr;  // an error left a capture open: close and drop it
                if (hipStreamEndCapture(B->own, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            }
            (void)hipStreamSynchronize(B->own);
            for (auto* P : B->P) P->stream = B->stream;
        }
    } restore{B};
    for (auto* P : B->P) P->stream = st;
    // Deterministic sigma (sort path) of every instance: an equal share of a
    // quarter of the memory free now for each instance's tuple buffers, so
    // that instances set up later are not left with the remainder of the
    // earlier ones' buffers.  Cleared when the call returns.
    struct TupHint {
        sfci_batch* B;
        ~TupHint() {
            for (auto* P : B->P) P->tup_cap_hint = 0;
        }
    } tup_hint{B};
    if (det) {
        size_t freeb = 0, totb = 0;
        SFCI_CHECK_HIP(hipMemGetInfo(&freeb, &totb));
        const u64 per = std::max<u64>(4096, (u64)(freeb / 4 / (size_t)std::max(1, n)) / SFCI_SORT_TUPLE_BYTES);
        for (auto* P : B->P) P->tup_cap_hint = per;
    }
    std::vector<Inst> I(n);
    bool all_tiles = true;
    for (int k = 0; k < n; ++k) {
        sfci_problem* P = B->P[k];
        if (v0s[k].nnz == 0) return (sfci_status)sfci_set_error(SFCI_E_ARG, "empty start vector");
        validate_vec(P, v0s[k].rank, v0s[k].nnz);
        if (!ensure_dense(P))
            return (sfci_status)sfci_set_error(SFCI_E_UNSUPPORTED, "every instance needs its dense accumulator");
        if (!det && o->dedup != SFCI_DEDUP_DENSE_ATOMIC && !rowtile_available(P)) all_tiles = false;
        Inst& q = I[k];
        q.P = P;
        P->tie_band = o->tie_band ? 1 : 0;
        P->excite_eps = o->excite_eps;
        q.M = Ms[k];
        q.cap = (Ms[k] >= P->Ndet) ? P->Ndet
                                   : std::min<u64>(std::max<u64>(Ms[k] + tie_extra(P), v0s[k].nnz), P->Ndet);
        q.tps = terms_per_source(P->n, P->na, P->nb);
        q.Wr = (u64*)P->ws_lz[1].get((size_t)nL * q.cap * sizeof(u64));
        q.Wa = (double*)P->ws_lz[2].get((size_t)nL * q.cap * sizeof(double));
        q.sc = (u64*)P->ws_lz[3].get(64 * sizeof(u64));
        double* dbl = (double*)P->ws_lz[4].get((size_t)(2 * nL * nL + 64 + nblk) * sizeof(double));
        q.T = dbl;
        q.S = dbl + nL * nL;
        q.x = q.S + nL * nL;
        q.lam = q.x + 32;
        q.energies = q.lam + 8;
        int* ints = (int*)P->ws_lz[6].get(64 * sizeof(int));
        q.blk = ints;
        q.status = ints + 16;
        const u64 pcap = std::min<u64>(P->Ndet, (u64)nL * q.cap);
        q.psi_r = (u64*)P->ws_lz[5].get(pcap * sizeof(u64));
        q.psi_a = (double*)P->ws_lz[7].get(2 * pcap * sizeof(double));
        q.sbar = q.psi_a + pcap;
        if (det) {
            q.lcap = std::min<u64>(P->Ndet, q.cap * q.tps);
            q.lr = (u64*)P->ws_list_r.get(q.lcap * sizeof(u64));
            q.la = (double*)P->ws_list_a.get(q.lcap * sizeof(double));
        }
        launch_fill_u64(q.sc, 64, 0, st);
        SFCI_CHECK_HIP(hipMemsetAsync(ints, 0, 64 * sizeof(int), st));
        DVec w = q.W(0);
        SFCI_CHECK_HIP(hipMemcpyAsync(w.r, v0s[k].rank, v0s[k].nnz * sizeof(u64), hipMemcpyDeviceToDevice, st));
        SFCI_CHECK_HIP(hipMemcpyAsync(w.a, v0s[k].amp, v0s[k].nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
        launch_set_u64(P, w.nnz, v0s[k].nnz);
        launch_normalise(P, w.a, w.nnz, q.cap, det);
    }
    const bool batched_sigma = !det && o->dedup != SFCI_DEDUP_DENSE_ATOMIC && all_tiles;
    const bool autotune = o->autotune != 0 && batched_sigma;
    int tune_trials = 0;
    double tune_default_ms = 0.0, tune_best_ms = 0.0;
    // The vector steps of a tile-batched iteration (dots, Eq. 10, truncation,
    // Eq. 11, the block end) run as one launch per step for all instances
    // (SFCI_BATCH_REST=0: per instance, as the other modes do).
    bool batched_rest = batched_sigma;
    if (const char* env = getenv("SFCI_BATCH_REST")) batched_rest = batched_rest && env[0] != '0';
    const BInst* d_bi = nullptr;
    const BScanJob* d_scan_dense = nullptr;
    const BScanJob* d_scan_list = nullptr;
    u64 max_cap = 1, max_ndet = 1;
    int max_ndig = 1;
    if (batched_rest) {
        std::vector<BInst> hb(n);
        std::vector<BScanJob> hs(2 * (size_t)n);
        for (int k = 0; k < n; ++k) {
            Inst& q = I[k];
            sfci_problem* P = q.P;
            const u64 nch = select_chunks(P->Ndet);
            const u64 n2 = (u64)P->n * P->n;
            BInst& b = hb[k];
            b.Wr = q.Wr;
            b.Wa = q.Wa;
            b.sc = q.sc;
            b.cap = q.cap;
            b.D = P->d_D;
            b.Ndet = P->Ndet;
            b.T = q.T;
            b.S = q.S;
            b.x = q.x;
            b.lam = q.lam;
            b.energies = q.energies;
            b.blk = q.blk;
            b.status = q.status;
            // also the gradient pass's raw sums and the per-instance reductions
            b.red = (double*)P->ws_red.get(std::max<u64>(bstep_red_doubles(nL), 2048 + n2 + n2 * n2) * sizeof(double));
            b.st = (SelState*)P->ws_sel.get(sizeof(SelState));
            b.st2 = (SelState*)P->ws_sel2.get(sizeof(SelState));
            b.cr = (u64*)P->ws_cand_r.get(P->Ndet * sizeof(u64));
            b.ca = (double*)P->ws_cand_a.get(P->Ndet * sizeof(double));
            b.cnt = (u64*)P->ws_cnt.get(nch * sizeof(u64));
            b.bsum = (u64*)P->ws_scan.get(scan_block_sums(nch) * sizeof(u64));
            b.psi_r = q.psi_r;
            b.psi_a = q.psi_a;
            b.psi_n = q.sc + 34;
            b.M = q.M;
            b.ndet_m1 = P->kg.ndet_m1;
            b.rank_bits = P->kg.rank_bits;
            b.nL = nL;
            hs[k] = BScanJob{b.cnt, b.cnt, nch, b.bsum, &b.st->count_cand};
            hs[n + k] = BScanJob{b.cnt, b.cnt, nch, b.bsum, &b.st2->count_out};
            max_cap = std::max(max_cap, q.cap);
            max_ndet = std::max(max_ndet, P->Ndet);
            max_ndig = std::max(max_ndig, (63 + P->kg.rank_bits + 10) / 11);
        }
        BInst* dbi = (BInst*)B->binst.get((size_t)n * sizeof(BInst));
        BScanJob* dsj = (BScanJob*)B->bscan.get(2 * (size_t)n * sizeof(BScanJob));
        SFCI_CHECK_HIP(hipMemcpyAsync(dbi, hb.data(), hb.size() * sizeof(BInst), hipMemcpyHostToDevice, st));
        SFCI_CHECK_HIP(hipMemcpyAsync(dsj, hs.data(), hs.size() * sizeof(BScanJob), hipMemcpyHostToDevice, st));
        SFCI_CHECK_HIP(hipStreamSynchronize(st));  // the host arrays go out of scope
        d_bi = dbi;
        d_scan_dense = dsj;
        d_scan_list = dsj + n;
    }
    // The gradient pass's buffers at their full size before any graph is
    // captured: growing one later would free memory the graphs use.
    if (!det && (dh_all || deri_all))
        for (const Inst& q : I) {
            const u64 n2 = (u64)q.P->n * q.P->n;
            const u64 pcap = std::min<u64>(q.P->Ndet, (u64)nL * q.cap);
            (void)q.P->ws_red.get((2048 + n2 + n2 * n2) * sizeof(double));
            (void)q.P->ws_list_r.get(pcap * sizeof(u64));
            (void)q.P->ws_list_a.get(pcap * sizeof(double));
            // rowtile_prepare's per-entry words (two u32 per input entry), for Psi
            if (rowtile_available(q.P)) (void)q.P->ws_rt_beta.get(2 * std::max<u64>(1, pcap) * sizeof(u32));
        }
    // What the step graphs depend on besides device data: kept graphs serve
    // a later call only when its signature is the same.
    auto signature = [&] {
        std::vector<u64> g;
        auto bits = [](double d) {
            u64 b;
            std::memcpy(&b, &d, sizeof b);
            return b;
        };
        auto ptr = [](const void* p) { return (u64)(uintptr_t)p; };
        g.insert(g.end(), {(u64)n, (u64)nL, (u64)o->dedup, (u64)(o->tie_band != 0), bits(o->screen_eps),
                           bits(o->excite_eps), (u64)batched_sigma, (u64)batched_rest, B->tune.b1_chunk,
                           B->tune.bb_chunk, B->tune.per_cu});
        for (const Inst& q : I)
            g.insert(g.end(), {ptr(q.P), q.M, q.cap, ptr(q.Wr), ptr(q.Wa), ptr(q.sc), ptr(q.T), ptr(q.psi_r),
                               ptr(q.psi_a), ptr(q.P->d_D)});
        return g;
    };
    const bool graphs_reused = use_graph && !B->gstep.empty() && (!autotune || B->tuned) &&
                               B->gepoch == device_free_epoch() && B->gsig == signature();
    if (!graphs_reused) B->drop_graphs();

    // One sigma application for every instance, in two parts: the per-instance
    // preparation (row pointers, tile offsets, input-size bookkeeping) and the
    // single tile launch that drains the work of all instances.
    B->descs.resize(nL);
    std::vector<RowTileDesc> descs(n);
    u64 total_items = 0, nbr_cap = 0;
    RowTileGeom geom{};
    char* d_desc = nullptr;
    u64* d_pre = nullptr;
    unsigned* d_cnt = nullptr;
    void* d_scr = nullptr;
    // Per-instance work fans out over the auxiliary streams (instance k on
    // aux[k % S]) and joins back to st, so that the small kernels of
    // different instances overlap; under capture this becomes parallel graph
    // branches.  The deterministic mode stays on st (its sort path
    // synchronises the stream of the instance).
    const int S = det ? 1 : (int)B->aux.size();
    auto fan = [&](auto&& body) {
        if (S <= 1) {
            for (int k = 0; k < n; ++k) body(k);
            return;
        }
        SFCI_CHECK_HIP(hipEventRecord(B->ev_fork, st));
        for (int s = 0; s < S; ++s) SFCI_CHECK_HIP(hipStreamWaitEvent(B->aux[s], B->ev_fork, 0));
        for (int k = 0; k < n; ++k) {
            I[k].P->stream = B->aux[k % S];
            body(k);
            I[k].P->stream = st;
        }
        for (int s = 0; s < S; ++s) {
            SFCI_CHECK_HIP(hipEventRecord(B->ev_join[s], B->aux[s]));
            SFCI_CHECK_HIP(hipStreamWaitEvent(st, B->ev_join[s], 0));
        }
    };
    auto sigma_prepare = [&](int j, bool upload) {
        if (!batched_sigma) {
            for (int k = 0; k < n; ++k) launch_add_u64(I[k].P, I[k].sc + 35, I[k].sc + j);  // input entries
            return;
        }
        std::vector<u64> pre(n + 1, 0);
        fan([&](int k) {
            launch_add_u64(I[k].P, I[k].sc + 35, I[k].sc + j);
            DVec w = I[k].W(j);
            descs[k] = rowtile_prepare(I[k].P, SigmaLaunch{w.r, w.a, w.nnz, w.cap}, I[k].P->d_D,
                                       (unsigned long long*)(I[k].sc + 32), o->screen_eps, false, batched_rest);
        });
        for (int k = 0; k < n; ++k) {
            pre[k + 1] = pre[k] + descs[k].n_items;
            nbr_cap = std::max(nbr_cap, descs[k].nbr_cap);
        }
        total_items = pre[n];
        geom = rowtile_geom(descs.data(), n);
        const size_t db = rowtile_desc_bytes();
        d_desc = (char*)B->descs[j].get((size_t)n * db);
        d_pre = (u64*)B->prefix.get((size_t)(n + 1) * sizeof(u64));
        d_cnt = (unsigned*)B->counter.get(64);
        // room for the largest grid a tuning candidate may use
        const unsigned gmax = std::max(rowtile_grid(B->P[0]->num_cu, geom.lds, total_items),
                                       rowtile_grid(B->P[0]->num_cu, geom.lds, total_items, kTuneMaxPerCu));
        d_scr = B->scratch.get(rowtile_scratch_bytes(gmax, nbr_cap));
        if (upload) {
            std::vector<unsigned char> host((size_t)n * db);
            for (int k = 0; k < n; ++k) std::memcpy(host.data() + (size_t)k * db, descs[k].raw, db);
            SFCI_CHECK_HIP(hipMemcpyAsync(d_desc, host.data(), host.size(), hipMemcpyHostToDevice, st));
            SFCI_CHECK_HIP(hipMemcpyAsync(d_pre, pre.data(), pre.size() * sizeof(u64), hipMemcpyHostToDevice, st));
            SFCI_CHECK_HIP(hipStreamSynchronize(st));  // the host staging buffers go out of scope
        }
        launch_fill_u64((u64*)d_cnt, 1, 0, st);
    };
    auto sigma_launch = [&](int j) {
        if (batched_sigma) {
            // descriptions of step j (uploaded in the eager block; the
            // remaining launch parameters are the same for every step)
            rowtile_run(st, B->P[0]->num_cu, B->descs[j].p, d_pre, n, d_cnt, d_scr, nbr_cap, geom, total_items, false,
                        B->tune);
            return;
        }
        for (int k = 0; k < n; ++k) {
            Inst& q = I[k];
            DVec w = q.W(j);
            SigmaLaunch sl{w.r, w.a, w.nnz, w.cap};
            if (det) {
                sigma_sorted(q.P, sl, q.lcap, q.lr, q.la, q.sc + 33, q.sc + 32);
                launch_scatter_set(q.P, q.P->d_D, q.lr, q.la, q.sc + 33, q.lcap);
                if (o->screen_eps > 0.0) launch_screen(q.P, q.P->d_D, q.P->Ndet, o->screen_eps);
            } else {
                dense_sigma(q.P, sl, o->dedup, (unsigned long long*)(q.sc + 32), o->screen_eps);
            }
        }
    };
    // Autotuning: the sigma of step j (inputs prepared, counter zeroed) is
    // launched once per candidate work-size set, each bracketed by events;
    // every launch overwrites the same touched tiles, so the real launch that
    // follows leaves the state it would have without the trials.  The term
    // counters are saved and restored around them.  Coordinate descent:
    // beta singles per unit, then beta-beta doubles per unit, then the grid.
    auto tune_on_step = [&](int j) {
        (void)j;
        for (int k = 0; k < n; ++k)
            SFCI_CHECK_HIP(hipMemcpyAsync(I[k].sc + 40, I[k].sc + 32, sizeof(u64), hipMemcpyDeviceToDevice, st));
        const unsigned auto_per_cu =
            std::max(1u, rowtile_grid(1, geom.lds, ~0ull));  // workgroups per CU the default grid uses
        auto trial = [&](const RowTileTune& t) {
            hipEvent_t a, z;
            SFCI_CHECK_HIP(hipEventCreate(&a));
            SFCI_CHECK_HIP(hipEventCreate(&z));
            SFCI_CHECK_HIP(hipEventRecord(a, st));
            rowtile_run(st, B->P[0]->num_cu, B->descs[j].p, d_pre, n, d_cnt, d_scr, nbr_cap, geom, total_items, true,
                        t);
            SFCI_CHECK_HIP(hipEventRecord(z, st));
            SFCI_CHECK_HIP(hipEventSynchronize(z));
            float ms = 0.f;
            SFCI_CHECK_HIP(hipEventElapsedTime(&ms, a, z));
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(z);
            ++tune_trials;
            return (double)ms;
        };
        RowTileTune best{16, 4, auto_per_cu};
        double best_ms = trial(best);
        tune_default_ms = best_ms;
        auto consider = [&](RowTileTune t) {
            const double ms = trial(t);
            if (ms < best_ms) best_ms = ms, best = t;
        };
        const RowTileTune b0 = best;
        for (unsigned c : {8u, 32u}) consider(RowTileTune{c, b0.bb_chunk, b0.per_cu});
        const RowTileTune b1 = best;
        for (unsigned c : {2u, 8u}) consider(RowTileTune{b1.b1_chunk, c, b1.per_cu});
        const RowTileTune b2 = best;
        if (2 * auto_per_cu <= kTuneMaxPerCu) consider(RowTileTune{b2.b1_chunk, b2.bb_chunk, 2 * auto_per_cu});
        tune_best_ms = best_ms;
        B->tune = best;
        B->tuned = true;
        for (int k = 0; k < n; ++k)
            SFCI_CHECK_HIP(hipMemcpyAsync(I[k].sc + 32, I[k].sc + 40, sizeof(u64), hipMemcpyDeviceToDevice, st));
        launch_fill_u64((u64*)d_cnt, 1, 0, st);  // the real launch starts from item 0
    };
    const int band = o->tie_band ? 1 : 0;
    auto iteration_rest = [&](int j) {
        if (batched_rest) {
            bstep_dots(st, d_bi, n, j, nL);
            if (j + 1 < nL) {
                bstep_axpy(st, d_bi, n, j, j, 0, max_cap);
                if (j >= 1) bstep_axpy(st, d_bi, n, j - 1, j, 0, max_cap);
                // D is left as it is: the next sigma launch writes every row (full_rows)
                bstep_select(st, d_bi, n, BOUT_NEXT, j, max_ndet, B->P[0]->num_cu, band, max_ndig, d_scan_dense,
                             d_scan_list, 0, false);
                bstep_normalise(st, d_bi, n, BOUT_NEXT, j, max_cap);
            } else {
                bstep_fill_zero(st, d_bi, n, max_ndet);
            }
            return;
        }
        fan([&](int k) {
            Inst& q = I[k];
            sfci_problem* P = q.P;
            DVec wj = q.W(j);
            for (int l = 0; l <= j; ++l) {
                DVec wl = q.W(l);
                launch_dot_dense(P, wl.r, wl.a, wl.nnz, q.cap, P->d_D, q.T + l * nL + j, q.T + j * nL + l, det);
                launch_dot_sparse(P, wl.r, wl.a, wl.nnz, q.cap, wj.r, wj.a, wj.nnz, q.S + l * nL + j,
                                  q.S + j * nL + l, det);
            }
            if (j + 1 < nL) {
                launch_axpy_scatter(P, P->d_D, wj.r, wj.a, wj.nnz, q.cap, q.T + j * nL + j, -1.0);
                if (j >= 1) {
                    DVec wm = q.W(j - 1);
                    launch_axpy_scatter(P, P->d_D, wm.r, wm.a, wm.nnz, q.cap, q.T + (j - 1) * nL + j, -1.0);
                }
                DVec wn = q.W(j + 1);
                CandSrc src{};
                src.dense = P->d_D;
                select_topm(P, src, q.M, wn.r, wn.a, wn.nnz, true);
                launch_normalise(P, wn.a, wn.nnz, q.cap, det);
            } else {
                launch_fill_f64(P->d_D, P->Ndet, 0.0, P->stream);
            }
        });
    };
    auto block_end = [&](bool last) {
        if (batched_rest) {
            bstep_geneig(st, d_bi, n, nL);
            for (int j = 0; j < nL; ++j) bstep_axpy(st, d_bi, n, j, 0, 1, max_cap);
            if (!last) {
                bstep_select(st, d_bi, n, BOUT_W0, 0, max_ndet, B->P[0]->num_cu, band, max_ndig, d_scan_dense,
                             d_scan_list, 0);
                bstep_normalise(st, d_bi, n, BOUT_W0, 0, max_cap);
            } else {
                // every nonzero entry of Psi (capacity n_L * cap suffices)
                bstep_select(st, d_bi, n, BOUT_PSI, 0, max_ndet, B->P[0]->num_cu, band, max_ndig, d_scan_dense,
                             d_scan_list, 1);
            }
            bstep_inc_blk(st, d_bi, n);
            return;
        }
        fan([&](int k) {
            Inst& q = I[k];
            sfci_problem* P = q.P;
            launch_geneig_full(P, nL, q.T, q.S, q.lam, q.x, q.energies, q.status, q.blk);
            for (int j = 0; j < nL; ++j) {
                DVec wj = q.W(j);
                launch_axpy_scatter(P, P->d_D, wj.r, wj.a, wj.nnz, q.cap, q.x + j, +1.0);
            }
            CandSrc src{};
            src.dense = P->d_D;
            if (!last) {
                DVec w0 = q.W(0);
                select_topm(P, src, q.M, w0.r, w0.a, w0.nnz, true);
                launch_normalise(P, w0.a, w0.nnz, q.cap, det);
            } else {
                select_topm(P, src, UINT64_MAX, q.psi_r, q.psi_a, q.sc + 34, true);  // capacity n_L * cap suffices
            }
            launch_inc_int(P, q.blk);
        });
    };

    // events: whole run, gradients, and one pair around every eager sigma
    // launch; the pairs recorded inside the step graphs are the batch's (gev)
    const int n_sig = nblk * nL;
    std::vector<hipEvent_t> ev(3 + 2 * (size_t)n_sig, nullptr);
    struct EvFree {
        std::vector<hipEvent_t>& v;
        ~EvFree() {
            for (auto e : v)
                if (e) (void)hipEventDestroy(e);
        }
    } ev_free{ev};
    for (auto& e : ev) SFCI_CHECK_HIP(hipEventCreate(&e));
    hipEvent_t e0 = ev[0], e1 = ev[1], e2 = ev[2];
    // replayed steps: one graph per step (B->gstep, kept for later calls), or,
    // where the runtime refuses event-record nodes in a graph, the
    // preparation and the rest of the step as two graphs with the tile launch
    // between them (gprep, grest: this call only)
    std::vector<hipGraphExec_t> gprep, grest;
    struct GraphFree {
        std::vector<hipGraphExec_t>& a;
        std::vector<hipGraphExec_t>& b;
        ~GraphFree() {
            for (auto* v : {&a, &b})
                for (auto x : *v) (void)hipGraphExecDestroy(x);
        }
    } graph_free{gprep, grest};
    // kept graphs are dropped unless this call ends with them intact
    struct KeepGuard {
        sfci_batch* B;
        bool keep = false;
        ~KeepGuard() {
            if (!keep) B->drop_graphs();
        }
    } keep_guard{B};
    std::vector<hipGraphExec_t>& gstep = B->gstep;
    bool split_steps = false;
    auto capture_graph = [&](auto&& body) {
        hipGraph_t g;
        SFCI_CHECK_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        body();
        SFCI_CHECK_HIP(hipStreamEndCapture(st, &g));
        return g;
    };
    auto instantiate = [&](hipGraph_t g) {
        hipGraphExec_t ex;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        SFCI_CHECK_HIP(e);
        return ex;
    };
    auto capture = [&](auto&& body) { return instantiate(capture_graph(body)); };
    // One iteration step as one graph: the captured preparation, tile launch
    // and vector operations as child graphs, chained through event-record
    // nodes around the tile launch (the events time it on every replay).
    auto step_graph = [&](int j) {
        hipGraph_t gA = capture_graph([&] { sigma_prepare(j, false); });
        hipGraph_t gB = capture_graph([&] { sigma_launch(j); });
        hipGraph_t gC = capture_graph([&] { iteration_rest(j); });
        hipGraph_t g = nullptr;
        hipError_t e = hipGraphCreate(&g, 0);
        hipGraphNode_t nA, e1, nB, e2, nC;
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&nA, g, nullptr, 0, gA);
        if (e == hipSuccess) e = hipGraphAddEventRecordNode(&e1, g, &nA, 1, B->gev[2 * j]);
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&nB, g, &e1, 1, gB);
        if (e == hipSuccess) e = hipGraphAddEventRecordNode(&e2, g, &nB, 1, B->gev[2 * j + 1]);
        if (e == hipSuccess) e = hipGraphAddChildGraphNode(&nC, g, &e2, 1, gC);
        (void)hipGraphDestroy(gA);  // the child nodes hold their own copies
        (void)hipGraphDestroy(gB);
        (void)hipGraphDestroy(gC);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (g) (void)hipGraphDestroy(g);
            return (hipGraphExec_t) nullptr;
        }
        return instantiate(g);
    };
    double sigma_ms = 0.0;
    int replayed_blocks = 0;
    SFCI_CHECK_HIP(hipEventRecord(e0, st));
    int sig = 0;
    for (int b = 0; b < nblk; ++b) {
        const bool last = (b + 1 == nblk);
        const bool replay = use_graph && (b >= 1 || graphs_reused);
        if (replay && gstep.empty() && !split_steps) {
            // one graph per iteration step (step_graph) and one for the
            // (non-final) block end
            B->gev.assign(2 * (size_t)nL, nullptr);
            for (auto& e : B->gev) SFCI_CHECK_HIP(hipEventCreate(&e));
            for (int j = 0; j < nL && !split_steps; ++j) {
                hipGraphExec_t x = step_graph(j);
                if (x) gstep.push_back(x);
                else split_steps = true;
            }
            if (split_steps) {
                for (auto x : gstep) (void)hipGraphExecDestroy(x);
                gstep.clear();
                for (int j = 0; j < nL; ++j) {
                    gprep.push_back(capture([&] { sigma_prepare(j, false); }));
                    grest.push_back(capture([&] { iteration_rest(j); }));
                }
            }
            B->gend = capture([&] { block_end(false); });
            if (!split_steps) {
                B->gsig = signature();
                B->gepoch = device_free_epoch();
            }
        }
        if (replay) ++replayed_blocks;
        for (int j = 0; j < nL; ++j, ++sig) {
            if (replay && !split_steps) {
                SFCI_CHECK_HIP(hipGraphLaunch(gstep[j], st));
                continue;
            }
            if (replay) {
                SFCI_CHECK_HIP(hipGraphLaunch(gprep[j], st));
                SFCI_CHECK_HIP(hipEventRecord(B->gev[2 * j], st));
                sigma_launch(j);
                SFCI_CHECK_HIP(hipEventRecord(B->gev[2 * j + 1], st));
                SFCI_CHECK_HIP(hipGraphLaunch(grest[j], st));
                continue;
            }
            sigma_prepare(j, true);
            if (autotune && !B->tuned && b == 0 && j == nL - 1) tune_on_step(j);
            SFCI_CHECK_HIP(hipEventRecord(ev[3 + 2 * sig], st));
            sigma_launch(j);
            SFCI_CHECK_HIP(hipEventRecord(ev[4 + 2 * sig], st));
            iteration_rest(j);
        }
        if (replay) {
            // the step graphs' events hold this block's sigma times until the next replay
            for (int j = 0; j < nL; ++j) {
                SFCI_CHECK_HIP(hipEventSynchronize(B->gev[2 * j + 1]));
                float ms = 0.f;
                SFCI_CHECK_HIP(hipEventElapsedTime(&ms, B->gev[2 * j], B->gev[2 * j + 1]));
                sigma_ms += ms;
            }
        }
        if (replay && !last) SFCI_CHECK_HIP(hipGraphLaunch(B->gend, st));
        else block_end(last);
    }
    SFCI_CHECK_HIP(hipEventRecord(e1, st));
    // gradients of each instance's Rayleigh quotient at the final Psi:
    // sbar = Psi / <Psi|Psi>, v = Psi
    if (dh_all || deri_all) {
        bool tiles = !det;
        for (int k = 0; k < n && tiles; ++k) tiles = rowtile_grad_available(I[k].P);
        std::vector<GradJob> jobs;
        u64 off_h = 0, off_g = 0;
        for (int k = 0; k < n; ++k) {
            Inst& q = I[k];
            sfci_problem* P = q.P;
            const u64 pcap = std::min<u64>(P->Ndet, (u64)nL * q.cap);
            const u64 n2 = (u64)P->n * P->n, n4 = n2 * n2;
            double* raw = (double*)P->ws_red.get((2048 + n2 + n4) * sizeof(double));
            double* dh = dh_all ? dh_all + off_h : nullptr;
            double* dg = deri_all ? deri_all + off_g : nullptr;
            launch_div_by_sumsq(P, q.psi_a, q.sc + 34, pcap, q.sbar);
            const SigmaLaunch psi{q.psi_r, q.psi_a, q.sc + 34, pcap};
            if (tiles) {
                GradJob J{};
                J.P = P;
                J.v = psi;
                J.s_rank = q.psi_r;
                J.s_amp = q.sbar;
                J.s_nnz = q.sc + 34;
                J.s_cap = pcap;
                J.Rh = raw + 2048;
                J.Rg = raw + 2048 + n2;
                J.dh = dh;
                J.dg = dg;
                J.vt_rank = (u64*)P->ws_list_r.get(pcap * sizeof(u64));
                J.vt_amp = (double*)P->ws_list_a.get(pcap * sizeof(double));
                J.vt_nnz = q.sc + 36;
                J.pair_sym = true;  // sbar = Psi / <Psi|Psi>
                jobs.push_back(J);
            } else {
                launch_scatter_set(P, P->d_D, q.psi_r, q.sbar, q.sc + 34, pcap);
                launch_backward_dense(P, psi, P->d_D, nullptr, dh, dg, raw + 2048, raw + 2048 + n2);
                launch_scatter_zero(P, P->d_D, q.psi_r, q.sc + 34, pcap);
            }
            off_h += n2;
            off_g += n4;
        }
        if (tiles) rowtile_gradients(st, n, jobs.data(), B->grad_ws);
    }
    SFCI_CHECK_HIP(hipEventRecord(e2, st));
    // results
    std::vector<int> hstat(n);
    std::vector<u64> hsc((size_t)n * 64);
    for (int k = 0; k < n; ++k) {
        SFCI_CHECK_HIP(hipMemcpyAsync(energies + (size_t)k * nblk, I[k].energies, nblk * sizeof(double),
                                      hipMemcpyDeviceToHost, st));
        SFCI_CHECK_HIP(hipMemcpyAsync(&hstat[k], I[k].status, sizeof(int), hipMemcpyDeviceToHost, st));
        SFCI_CHECK_HIP(hipMemcpyAsync(&hsc[(size_t)k * 64], I[k].sc, 64 * sizeof(u64), hipMemcpyDeviceToHost, st));
    }
    SFCI_CHECK_HIP(hipStreamSynchronize(st));
    // the step graphs stay for later calls while every buffer they use is alive
    keep_guard.keep = !split_steps && !gstep.empty() && B->gepoch == device_free_epoch();
    if (stats) {
        float f = 0.f, bw = 0.f;
        SFCI_CHECK_HIP(hipEventElapsedTime(&f, e0, e1));
        SFCI_CHECK_HIP(hipEventElapsedTime(&bw, e1, e2));
        stats->fwd_ms = f;
        stats->bwd_ms = bw;
        double sms = sigma_ms;
        for (int i = 0; i < n_sig; ++i) {
            if (i >= (nblk - replayed_blocks) * nL) break;  // replayed steps: counted from the graphs' events above
            float ms = 0.f;
            SFCI_CHECK_HIP(hipEventElapsedTime(&ms, ev[3 + 2 * i], ev[4 + 2 * i]));
            sms += ms;
        }
        stats->sigma_ms = sms;
        u64 emitted = 0, nin = 0, psi_total = 0;
        for (int k = 0; k < n; ++k) {
            emitted += hsc[(size_t)k * 64 + 32];
            psi_total += hsc[(size_t)k * 64 + 34];
            nin += hsc[(size_t)k * 64 + 35];
        }
        stats->terms_emitted = emitted;
        stats->nnz_in_total = nin;
        stats->sigma_calls = (u64)n_sig;
        stats->psi_nnz_total = psi_total;
        stats->graph_replayed_blocks = replayed_blocks;
        stats->batched_sigma = batched_sigma ? 1 : 0;
        stats->tune_trials = tune_trials;
        stats->tune_b1_chunk = batched_sigma ? B->tune.b1_chunk : 0u;
        stats->tune_bb_chunk = batched_sigma ? B->tune.bb_chunk : 0u;
        stats->tune_per_cu = batched_sigma ? B->tune.per_cu : 0u;
        stats->tune_default_ms = tune_default_ms;
        stats->tune_best_ms = tune_best_ms;
        stats->sigma_in_graph = (replayed_blocks > 0 && !split_steps) ? 1 : 0;
        stats->graphs_reused = graphs_reused ? 1 : 0;
    }
    for (int k = 0; k < n; ++k)
        if (hstat[k]) return (sfci_status)sfci_set_error(SFCI_E_DEVICE, "generalized eigenproblem failed");
    return SFCI_OK;
    SFCI_GUARD_END
}

}  // extern "C"
