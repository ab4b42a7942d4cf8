"""Benchmark of the SFCI hot path (sigma = H v with its Lanczos iteration) on one MI355X.

Default workload (c4batch): 32 bond-stretch instances of 8 electrons (4 alpha,
4 beta) in 20 orbitals, N_det = C(20,4)^2 = 2.35e7 each, integrals
h(lam) = h0 + lam h1, L(lam) = L0 + lam L1 with lam = j/31 (seeds 40-43, rank
40), truncations M_j = round(10^(4 + 2 u_j)) (seed 44), 30 sigma applications
per instance in blocks of N_L = 10, then dE/dh and dE/d(pq|rs) for every
instance.  A step is one Lanczos iteration of all 32 instances (one batched
sigma launch plus the per-instance vector operations); the timed region is
`--steps` iterations plus the gradient pass.  The plain path (each instance
alone: one FP64 atomic per term, no graphs, then the backward) is timed after
it for the speedup and the energy comparison.

Other workloads: c2 (10 electrons in 26 orbitals, one instance, M = 1e6), c3
(12 electrons in 28 orbitals, 1.42e11 determinants, run with --M 1e7: the
list iteration, since the 1.14 TB N_det array cannot exist) and c4 (one
20-orbital instance).  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E
# value: sigma terms per second of the whole job; the roofline fraction and the
# batched-vs-plain speedup with its energy agreement ride along in the record
METRIC = "\u03c3 terms/s and HBM-roofline fraction; batched fwd+bwd speedup vs plain @1e-9 Ha"

WORKLOADS = {
    "c2": dict(n=26, na=5, nb=5, rank=52, seed=2,
               desc="10e in 26 orbitals (5a,5b), N_det=4.33e9, molecule-like integrals seed 2"),
    "c3": dict(n=28, na=6, nb=6, rank=56, seed=3,
               desc="12e in 28 orbitals (6a,6b), N_det=1.42e11 (no N_det array: list iteration, sigma in "
                    "slices of target rows), molecule-like integrals seed 3"),
    "c4": dict(n=20, na=4, nb=4, rank=40, seed=None,
               desc="8e in 20 orbitals (4a,4b), N_det=2.35e7, bond-stretch instance lambda=0"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed Lanczos iterations, rounded up to whole blocks of n_L (default 30 for c4batch, "
                         "10 otherwise)")
    ap.add_argument("--warmup", type=int, default=10,
                    help="warm-up Lanczos iterations, rounded up to whole blocks of n_L (c4batch: at least "
                         "the timed iterations, so that the warm-up call captures the step graphs the timed "
                         "call replays)")
    ap.add_argument("--workload", default="c4batch", choices=sorted(WORKLOADS) + ["c4batch"])
    ap.add_argument("--no-plain", action="store_true", help="c4batch: skip the plain-path comparison")
    ap.add_argument("--n-inst", type=int, default=32)
    ap.add_argument("--M", type=float, default=1e6)
    ap.add_argument("--n_L", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=40.0)
    ap.add_argument("--dedup", default="dense", choices=["dense", "dense_atomic", "sort"],
                    help="dense: target-owned LDS tiles; dense_atomic: one FP64 atomic per term")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c4batch: keep the tile kernel's default work sizes")
    ap.add_argument("--pt2", action="store_true",
                    help="single-problem workloads: also time the Epstein-Nesbet correction of the start vector")
    ap.add_argument("--excited", action="store_true",
                    help="single-problem workloads: also time the iteration with the start vector projected out")
    ap.add_argument("--det", action="store_true",
                    help="single-problem workloads: deterministic mode (sort dedup, ordered sums)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run three 1 GiB device-to-device copies (calibrates the HBM byte counters)")
    return ap.parse_args()


def copy_probe(torch):
    n = 1 << 27  # 2^27 doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied 3 x {n * 8} bytes", flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sigma_rowtile_c4batch_traffic.md")


def measured_traffic():
    """HBM bytes per k_sigma_rowtile_whole launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel source
    has changed since the counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith(" "):
            k, _, v = line.partition(":")
            kv[k.strip()] = v.strip()
    csrc = os.path.join(ROOT, "paper_2312_01846_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("rowtile.hip", "sfci_device.h"))
    if kv.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return dict(total=float(kv["traffic_bytes_per_launch"]), fetch=float(kv["fetch_bytes_per_launch"]),
                    write=float(kv["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """Host threads the oracle may use: the cores this process may run on,
    at most 16 (a one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(h, g, n, na, nb, ranks, amps, target_s):
    """The oracle's sigma (generate + merge, Sec. 2.2) on a bounded strided
    sample of a vector of the timed workload: on all host cores (the paper's
    shared-memory form: per-thread buckets, per-bucket stable sort and merge)
    and on one core."""
    import oracle

    P = oracle.Problem(n, na, nb, h, g)
    tps = _tps(n, na, nb)
    ranks = np.ascontiguousarray(ranks, dtype=np.uint64)
    amps = np.ascontiguousarray(amps, dtype=np.float64)

    def timed(threads, budget):
        oracle.set_threads(threads)
        take = 64
        while True:
            idx = np.unique(np.linspace(0, len(ranks) - 1, min(take, len(ranks))).astype(np.int64))
            r, a = ranks[idx], amps[idx]
            t = time.perf_counter()
            P.sigma(r, a)
            el = time.perf_counter() - t
            if el > budget / 4 or len(idx) >= len(ranks):
                return len(idx), el
            take = min(len(ranks), int(take * max(2.0, budget / 4 / max(el, 1e-3))))

    cores = host_cores()
    old = oracle.get_threads()
    try:
        k_all, t_all = timed(cores, 0.6 * target_s)
        k_one, t_one = timed(1, 0.4 * target_s)
    finally:
        oracle.set_threads(old)
    return dict(value=k_all * tps / t_all, unit="terms/s", cores=cores, kind="oracle",
                single_core_value=k_one * tps / t_one, cpu_model=_cpu_model(),
                sample=f"oracle sigma (generate, then merge by stable sort and in-order sums) of {k_all} entries "
                       f"taken at even strides across a {len(ranks)}-entry vector of the timed workload, "
                       f"{k_all * tps:.3g} terms in {t_all:.1f} s on {cores} threads (per-thread buckets of the "
                       f"rank range, Sec. 2.2); single core: {k_one} entries, {k_one * tps:.3g} terms in "
                       f"{t_one:.1f} s")


# MI355X LDS: 128 B per clock per CU, 256 CUs at 2.4 GHz; a 64-lane FP64 add
# moves 512 B, so a conflict-free ds_add_f64 stream peaks at 16 adds/clk/CU.
LDS_ADD_PEAK = 256 * 16 * 2.4e9


def tile_roofline(st, alg_bytes, traffic, roof, kernel="k_sigma_rowtile"):
    """The tile kernel's roofline.  Every emitted term is one FP64 add into the
    workgroup's LDS tile (the accumulators never go to HBM), and the targets
    are random slots of the tile: the binding roof is the device's random
    LDS FP64 add rate, measured by sfci_roof_probe.  Reported beside it: HBM
    traffic from the committed counters (FETCH_SIZE + WRITE_SIZE) against
    8 TB/s, and the 16 B/term model of a dense-accumulator sigma."""
    calls = max(1, st["sigma_calls"])
    sig_s = st["sigma_ms"] / 1e3
    t_launch = sig_s / calls
    terms_s = st["terms_emitted"] / sig_s if sig_s > 0 else 0.0
    lds_peak = roof["lds_atomic_Gops"][1] * 1e9
    out = {
        "bound": "lds",
        "kernel": kernel,
        "achieved": terms_s / 1e9,
        "peak": lds_peak / 1e9,
        "unit": "G FP64 LDS adds/s (one per emitted term; peak: random-slot ds_add_f64, measured)",
        "frac": terms_s / lds_peak if lds_peak else None,
        "peak_conflict_free_published": LDS_ADD_PEAK / 1e9,
        "frac_of_conflict_free": terms_s / LDS_ADD_PEAK,
        "traffic": traffic["total"] / 1e9 if traffic else None,
        "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "hbm": {
            "achieved_GBps": traffic["total"] / t_launch / 1e9 if traffic and t_launch > 0 else None,
            "peak_GBps": HBM_PEAK / 1e9,
            "frac": traffic["total"] / t_launch / HBM_PEAK if traffic and t_launch > 0 else None,
            "copy_GBps_measured": roof["copy_GBps"],
        },
        "model_16B_per_term": {
            "achieved_GBps": alg_bytes / sig_s / 1e9 if sig_s > 0 else 0.0,
            "frac_of_8TBps": alg_bytes / sig_s / HBM_PEAK if sig_s > 0 else 0.0,
            "note": "16 B per input entry + 16 B per term (an accumulator read-modify-write in HBM); the LDS "
                    "tiles never send those bytes to HBM, so this is no bound on this kernel",
        },
        "sigma_kernel_ms_per_launch": t_launch * 1e3,
        "sigma_terms_per_launch": st["terms_emitted"] / calls,
        "probe": roof,
    }
    return out


def _tps(n, na, nb):
    from paper_2312_01846_amd.sfci import terms_per_source

    return terms_per_source(n, na, nb)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; sharding across GPUs is a design note "
                                   "(alpha-rank-range slices), not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps is None:
        args.steps = 30 if args.workload == "c4batch" else 10
    # The iteration runs whole blocks of n_L sigma applications (Sec. 2.1's
    # restart): requested counts are rounded up to whole blocks, and the
    # counts actually run are what the record reports.
    args.steps_requested, args.warmup_requested = args.steps, args.warmup
    args.steps = max(1, -(-max(1, args.steps) // args.n_L)) * args.n_L
    args.warmup = -(-max(0, args.warmup) // args.n_L) * args.n_L
    import torch

    if args.copy_probe:
        return copy_probe(torch)
    from paper_2312_01846_amd import sfci, synth

    if args.workload == "c4batch":
        return bench_batch(args, torch, sfci, synth)
    wl = WORKLOADS[args.workload]
    n, na, nb = wl["n"], wl["na"], wl["nb"]
    if args.workload == "c4":
        _, h, g = synth.bond_stretch_batch(n, 32, wl["rank"])[0]
    else:
        h, g = synth.molecule_like(n, wl["rank"], wl["seed"])
    M = int(args.M)
    torch.cuda.set_device(0)
    P = sfci.Problem(n, na, nb, h, g)
    tps = P.tps
    print(f"# building a start vector: {args.warmup} warm-up iterations at M={M}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    warm = P.lanczos(np.array([0], dtype=np.int64), np.array([1.0]), M=M, n_L=args.n_L, n_iter=args.warmup,
                     psi_capacity=min(P.n_det, args.n_L * (M + sfci.TIE_SLACK)), dedup=args.dedup,
                     deterministic=args.det)
    v_r, v_a = P.topm(warm["psi_rank"], warm["psi_amp"], M, normalise=True)
    torch.cuda.synchronize()
    print(f"# warm-up done in {time.perf_counter() - t0:.1f} s; start vector nnz={v_r.numel()}", file=sys.stderr,
          flush=True)
    t1 = time.perf_counter()
    out = P.lanczos(v_r, v_a, M=M, n_L=args.n_L, n_iter=args.steps, want_psi=False, dedup=args.dedup,
                    deterministic=args.det)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    st = out["stats"]
    print(f"# timed {args.steps} steps in {wall:.3f} s; sigma kernels {st['sigma_ms']:.1f} ms", file=sys.stderr,
          flush=True)
    terms = st["terms_emitted"]
    value = terms / wall
    # roofline of the dominant kernel (the sigma expansion): algorithmic bytes =
    # 16 B per input entry (rank + amplitude) + 16 B per emitted term (FP64
    # read-modify-write of the accumulator slot).
    nnz_in_total = st["terms_enumerated"] // tps
    alg_bytes = 16 * nnz_in_total + 16 * terms
    sig_s = st["sigma_ms"] / 1e3
    achieved = alg_bytes / sig_s if sig_s > 0 else 0.0
    pt2 = None
    if args.pt2:
        # second-order Epstein-Nesbet correction of the (truncated, normalised) start vector
        pt2 = dict(input_nnz=int(v_r.numel()))
        for mode, det in (("fast", False), ("deterministic", True)):
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            e0, e2, ne = P.pt2(v_r, v_a, deterministic=det)
            pt2[mode] = dict(ms=(time.perf_counter() - t2) * 1e3, e0=e0, e2=e2, n_external=ne,
                             sigma_terms_per_s=int(v_r.numel()) * tps / (time.perf_counter() - t2))
        print(f"# pt2: {pt2}", file=sys.stderr, flush=True)
    excited = None
    if args.excited:
        # the next state: the same iteration with the (truncated) start vector projected out
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        xo = P.lanczos(np.array([0], dtype=np.int64), np.array([1.0]), M=M, n_L=args.n_L, n_iter=args.steps,
                       want_psi=False, dedup=args.dedup, deterministic=args.det, roots=[(v_r, v_a)])
        torch.cuda.synchronize()
        xs = time.perf_counter() - t3
        excited = dict(ms_per_step=xs * 1e3 / args.steps, energies=[float(x) for x in xo["energies"]],
                       ground_ms_per_step=wall * 1e3 / args.steps)
        print(f"# excited: {excited}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(h, g, n, na, nb, v_r.cpu().numpy().astype(np.uint64), v_a.cpu().numpy(),
                           args.cpu_seconds)
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "steps_requested": args.steps_requested,
        "warmup_requested": args.warmup_requested,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl['desc']}, M={M}, N_L={args.n_L}, "
                        + ("deterministic (sort dedup)" if args.det else f"dedup={args.dedup}"),
            "M": M,
            "n_L": args.n_L,
            "terms_per_step": terms / args.steps,
            "energies": [float(x) for x in out["energies"]],
            "pt2": pt2,
            "excited": excited,
            "parallelism": "single GPU",
        },
        # rows of at most 16 384 beta ranks are one LDS tile: the one-tile kernel runs
        "roofline": (tile_roofline(st, alg_bytes, None, sfci.roof_probe(1 << 30),
                                   kernel=("k_sigma_rowtile_whole" if math.comb(n, nb) <= 16384
                                           else "k_sigma_rowtile"))
                     if (not args.det and args.dedup == "dense") else {
            "bound": "hbm",
            "kernel": "k_rs_scatter" if args.det else "k_sigma_dense",
            "achieved": achieved / 1e9,
            "peak": HBM_PEAK / 1e9,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK,
            "traffic": None,
            "sigma_kernel_ms_per_launch": st["sigma_ms"] / max(1, st["sigma_calls"]),
            "alg_bytes_per_launch": alg_bytes / max(1, st["sigma_calls"]),
            "sigma_terms_per_s_kernel": terms / sig_s if sig_s > 0 else 0.0,
        }),
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


def bench_batch(args, torch, sfci, synth):
    n, na, nb, rank = 20, 4, 4, 40
    inst = synth.bond_stretch_batch(n, 32, rank)[:args.n_inst]
    Ms = synth.batch_truncations(32)[:args.n_inst]
    torch.cuda.set_device(0)
    probs = [sfci.Problem(n, na, nb, h, g) for _, h, g in inst]
    start = synth.perturbed_start(n, na, nb)
    r0 = probs[0].rank([s[0] for s in start], [s[1] for s in start]).cpu().numpy()
    a0 = np.array([s[2] for s in start])
    order = np.argsort(r0, kind="stable")
    v0 = (r0[order], a0[order])
    B = sfci.Batch(probs)
    if args.warmup:
        # The warm-up call has the timed call's shape (at least as many
        # iterations as the warm-up asks for): it tunes the tile kernel's work
        # sizes and captures the step graphs, both kept by the batch for the
        # timed call.
        args.warmup = max(args.warmup, args.steps)
        print(f"# warm-up: {args.warmup} batched iterations + gradients", file=sys.stderr, flush=True)
        wout = B.lanczos([v0] * len(probs), Ms, n_L=args.n_L, n_iter=args.warmup, autotune=not args.no_autotune)
        tune = wout["stats"]["tune"]
        print(f"# tuned work sizes: {tune}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = B.lanczos([v0] * len(probs), Ms, n_L=args.n_L, n_iter=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = out["stats"]
    E = out["energies"]
    print(f"# batched: {wall:.3f} s (fwd {st['fwd_ms']:.0f} ms, bwd {st['bwd_ms']:.0f} ms, sigma {st['sigma_ms']:.0f} ms; "
          f"step graphs {'kept from the warm-up' if st['graphs_reused'] else 'captured in this call'})",
          file=sys.stderr, flush=True)
    plain = None
    sample = None
    if not args.no_plain:
        t1 = time.perf_counter()
        Ep = np.zeros(len(probs))
        biggest = int(np.argmax(Ms))
        for k, P in enumerate(probs):
            o = P.lanczos(v0[0], v0[1], M=Ms[k], n_L=args.n_L, n_iter=args.steps, dedup="dense_atomic",
                          psi_capacity=min(P.n_det, args.n_L * (Ms[k] + sfci.TIE_SLACK)))
            P.energy_gradients(o["psi_rank"], o["psi_amp"])
            Ep[k] = o["energies"][-1]
            if k == biggest:
                sample = (o["psi_rank"], o["psi_amp"])
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        dE = np.abs(E[:, -1] - Ep)
        plain = dict(seconds=t_plain, speedup=t_plain / wall, energy_max_abs_diff=float(dE.max()),
                     energy_abs_diff=[float(x) for x in dE],
                     path="each instance alone: FP64-atomic sigma, per-kernel launches, then the backward")
        print(f"# plain: {t_plain:.3f} s, speedup {t_plain / wall:.2f}x, max |dE| {dE.max():.2e}", file=sys.stderr,
              flush=True)
    terms = st["terms_emitted"]
    sig_s = st["sigma_ms"] / 1e3
    alg_bytes = 16 * st["nnz_in_total"] + 16 * terms
    achieved = alg_bytes / sig_s if sig_s > 0 else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        kb = int(np.argmax(Ms))
        if sample is None:
            o = probs[kb].lanczos(v0[0], v0[1], M=Ms[kb], n_L=args.n_L, n_iter=args.n_L)
            sample = (o["psi_rank"], o["psi_amp"])
        _, hs, gs = inst[kb]
        cpu = cpu_baseline(hs, gs, n, na, nb, sample[0].cpu().numpy().astype(np.uint64), sample[1].cpu().numpy(),
                           args.cpu_seconds)
        cpu["sample"] += f" (instance {kb}, its final Psi)"
    traffic = measured_traffic()
    roof = sfci.roof_probe(188 << 20)  # the ceilings, with a third array the size of one instance's accumulator
    rec = {
        "metric": METRIC,
        "value": terms / wall,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "steps_requested": args.steps_requested,
        "warmup_requested": args.warmup_requested,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"c4batch: {len(probs)} bond-stretch instances, 8e in 20 orbitals (4a,4b), N_det=2.35e7 each, "
                        f"M log-uniform in [1e4,1e6] (seed 44), N_L={args.n_L}, {args.steps} sigma per instance "
                        f"+ dE/dh, dE/d(pq|rs); start: aufbau + 0.1 N(0,1) on its singles (seed 7)",
            "Ms": Ms,
            "n_L": args.n_L,
            "fwd_ms": st["fwd_ms"],
            "bwd_ms": st["bwd_ms"],
            "sigma_ms_total": st["sigma_ms"],
            "terms_emitted": terms,
            "psi_nnz_total": st["psi_nnz_total"],
            "graph_replayed_blocks": st["graph_replayed_blocks"],
            "graphs_reused": st["graphs_reused"],
            "tile_work_sizes": st["tune"],
            "final_energies": [float(x) for x in E[:, -1]],
            "plain_path": plain,
            "batched_speedup_vs_plain": plain["speedup"] if plain else None,
            "parallelism": "single GPU",
        },
        "roofline": tile_roofline(st, alg_bytes, traffic, roof, kernel="k_sigma_rowtile_whole"),
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
