"""Benchmark of the double-double stealthy-hyperuniform hot path on one MI355X.

Default workload: the largest single-GPU configuration, d = 3, N = 30 000,
chi = 0.45 (R2 = 721, M = 40 494) with v(k) = (1 - |k|/K)^2.  A step is a
100-iteration segment of its L-BFGS quench from a fresh seeded uniform-random
start (the paper's Poisson initial condition) toward S_max <= 1e-40: every
iteration evaluates Phi + gradient over all M N particle-wavevector pairs in
double-double (a4-a8 of the path) and runs the device-resident minimiser (a9);
the cutoff, wavevector set and weights are built once before the timed region.
A whole quench of this configuration takes minutes, so configs/s at the floor
is measured beside it on whole quenches of d = 3, N = 8000, chi = 0.45.

Printed (one JSON line): dd pair-evaluations per second over the timed steps
(M N per Phi + gradient evaluation), the roofline of the dominant pass kernel
(FP64 flops with FMA = 2 against the 78.6 TFLOP/s FP64 vector peak, launch
times from HIP events on the launch stream), and the CPU oracle timed on a
bounded sample of the same workload.  Other workloads (--workload): whole
quenches (d3_N8000_chi0.45, d3_N30000_chi0.45[_w] with --segment 0), batches,
served streams and single evaluations at the paper's production shape.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOOR = 1e-40
# FP64 operations per particle-wavevector pair in the inner loops, counted from
# the kernel source as (add, mul, fma).  The n~(k) pass forms b z^t and b conj(z^t)
# for two wavevectors from four shared lazy dd products (4 mul, 12 fma) and four
# TwoSums with their error terms (32 add), and adds each pair factor with two
# lazy dd accumulations (8 add each): per pair 16 + 16 add, 2 mul, 6 fma; the
# gradient pass does a lazy complex dd product (two lazy dd dot products of 8 add,
# 2 mul, 6 fma each), the lazy dd dot product v (S c - C s) and two lazy
# accumulations (the sum of q and the sum of its prefix sums).
OPS_PER_PAIR_MIX = {"nk": (32, 2, 6), "grad": (40, 6, 18)}
# operations counted once (issue slots) and floating-point operations with an
# FMA counted as two (the convention of the published FP64 peak)
OPS_PER_PAIR = {k: a + m + f for k, (a, m, f) in OPS_PER_PAIR_MIX.items()}
FLOPS_PER_PAIR = {k: a + m + 2 * f for k, (a, m, f) in OPS_PER_PAIR_MIX.items()}
# MI355X FP64 vector peak: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T issue slots/s,
# 78.6 TFLOP/s with an FMA counted as two
PEAK_FP64_OPS = 256 * 64 * 2.4e9
PEAK_FP64_FLOPS = 2 * PEAK_FP64_OPS
WORKLOADS = {
    "d3_N8000_chi0.45": dict(d=3, N=8000, chi=0.45, cfg_id=2),
    "d3_N30000_chi0.45": dict(d=3, N=30000, chi=0.45, cfg_id=4),
    # the same size with v(k) = (1 - |k|/K)^2, K^2 = (R2 + 1/2) (2 pi / L)^2
    # (the largest single-GPU configuration; by default a step is a 100-iteration
    # segment of its L-BFGS quench, see bench_segments)
    "d3_N30000_chi0.45_w": dict(d=3, N=30000, chi=0.45, cfg_id=4, vkind=1, segment=100),
    "d2_N128_chi0.4": dict(d=2, N=128, chi=0.4, cfg_id=1),
    # 256 independent quenches: d in {2, 3}, N log-uniform in [500, 5000], chi in {0.2, 0.35, 0.45}
    "batch256_d2-3_N500-5000": dict(batch=256, shape_seed=3, cfg_id=3),
    # 200 requests served with continuous batching: d in {2, 3}, N log-uniform in
    # [500, 5000], chi uniform in [0.1, 0.49], Poisson arrivals at 0.7 x capacity
    "serve200_d2-3_N500-5000": dict(serve=200, stream_seed=5, cfg_id=6),
    # the same stream shape at N log-uniform in [1e3, 1e5] (the large requests take
    # seconds each)
    "serve200_d2-3_N1e3-1e5": dict(serve=200, stream_seed=8, cfg_id=7, n_min=1000, n_max=100000, arena_gb=96),
    "serve24_d2-3_N1e3-1e5": dict(serve=24, stream_seed=8, cfg_id=7, n_min=1000, n_max=100000, arena_gb=96),
    # the paper's production shape, one Phi + gradient evaluation at a time (a
    # quench at this size takes hours): d = 2, N = 2e6, chi = 0.1 and 0.4
    "d2_N2e6_chi0.1": dict(d=2, N=2_000_000, chi=0.1, cfg_id=9, evals_only=True),
    "d2_N2e6_chi0.4": dict(d=2, N=2_000_000, chi=0.4, cfg_id=9, evals_only=True),
}


def kernel_source_hash() -> str:
    """Hash of the pair kernels and of the host code that shapes their launches
    (schedules, tiles): counter summaries taken on other sources are ignored."""
    h = hashlib.sha256()
    for f in ("ss_dd.h", "ss_kernels.hip", "ss_api.hip", "ss_internal.h"):
        with open(os.path.join(ROOT, "paper_2304_09139_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile(name: str) -> dict | None:
    """key: value lines of a committed rocprofv3 counter summary, or None when
    there is none or it was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                rec[key.strip()] = val.strip()
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def read_traffic(kernel: str, workload: str) -> float | None:
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, calibrated on a copy)."""
    rec = read_profile(f"{kernel}_{workload}_counters.txt")
    try:
        return float(rec["hbm_bytes_per_launch"]) if rec else None
    except (KeyError, ValueError):
        return None


def read_fp64_flops(kernel: str, workload: str) -> float | None:
    """FP64 floating-point operations per launch with an FMA counted as two, from
    the SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 wave-instruction counts (x 64 lanes)."""
    rec = read_profile(f"{kernel}_{workload}_valu.txt")
    try:
        return 64.0 * (float(rec["add_f64"]) + float(rec["mul_f64"]) + 2.0 * float(rec["fma_f64"])) if rec else None
    except (KeyError, ValueError):
        return None


def roofline(kernel: str, label: str, launches: int, ms: float, pairs: float, workload: str | None) -> dict:
    """Roofline of one pair kernel from its HIP-event launch times: algorithmic
    FP64 flops (the per-pair count of the inner loop, FMA = 2) x the pairs of
    the average launch, over the average launch duration, against the 78.6
    TFLOP/s FP64 vector peak; the same launches in issue slots (every add, mul
    and fma counted once) against 39.3 T slots/s beside it."""
    kname = {"nk": "k_nk", "grad": "k_grad"}[kernel]
    avg_s = ms / max(launches, 1) * 1e-3
    ppl = pairs / max(launches, 1)
    achieved = FLOPS_PER_PAIR[kernel] * ppl / avg_s if launches else 0.0
    issue = OPS_PER_PAIR[kernel] * ppl / avg_s if launches else 0.0
    a, m, f = OPS_PER_PAIR_MIX[kernel]
    counted = read_fp64_flops(kname, workload) if workload else None
    return {
        "bound": "alu",
        "kernel": label,
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_FLOPS / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_FLOPS,
        "traffic": read_traffic(kname, workload) if workload else None,
        "flop_count": f"{FLOPS_PER_PAIR[kernel]} FP64 flops per pair ({a} add + {m} mul + {f} fma, FMA = 2) "
                      f"x {ppl:.6g} pairs per launch; peak = 256 CU x 64 lanes x 2.4 GHz x 2",
        "launches": launches,
        "avg_launch_ms": avg_s * 1e3,
        "issue": {"achieved": issue / 1e9, "peak": PEAK_FP64_OPS / 1e9,
                  "unit": "G FP64 instructions/s per lane (add, mul, fma each counted once)",
                  "frac": issue / PEAK_FP64_OPS},
        # FP64 flops the hardware executed per launch (SQ counters of the committed
        # profile, FMA = 2; includes the per-run work outside the inner loop)
        "executed": None if counted is None else {"flops_per_launch": counted,
                                                  "tflops": counted / avg_s / 1e12,
                                                  "frac": counted / avg_s / PEAK_FP64_FLOPS},
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def mp_error_report(ctx, w, n, v, pos, count=32, seed=7, label=""):
    """n~(k) at sampled wavevectors (the smallest |k|, the outermost shell and
    random ones) from the double-double and the FP64 passes, against a 256-bit
    mpmath evaluation of the same sums (phases n.u taken exactly from the dd
    positions): the error of every reported S(k) at those k."""
    import mpmath
    import numpy as np

    mp = mpmath.mp.clone() if hasattr(mpmath.mp, "clone") else mpmath.mp
    mp.prec = 256
    nd = ctx.energy_grad(w, n, v, pos, grad=False, nk=True)["nk"].cpu().numpy()
    nf = ctx.energy_grad(w, n, v, pos, grad=False, nk=True, fp64=True)["nk"].cpu().numpy()
    nh = n.cpu().numpy()
    ph = pos.cpu().numpy()
    rng = np.random.default_rng(seed)
    ks = sorted(set([0, w.M - 1] + [int(k) for k in rng.choice(w.M, count - 2, replace=False)]))
    u = [[mp.mpf(float(ph[0, a, j])) + mp.mpf(float(ph[1, a, j])) for j in range(w.N)] for a in range(w.d)]
    rows = []
    for q, k in enumerate(ks):
        if q % 4 == 0:
            print(f"[bench] 256-bit n~ {label}: wavevector {q + 1} of {len(ks)}", file=sys.stderr, flush=True)
        C = mp.mpf(0)
        S = mp.mpf(0)
        for j in range(w.N):
            t = sum(int(nh[k, a]) * u[a][j] for a in range(w.d))
            t = t - mp.floor(t)
            C += mp.cospi(2 * t)
            S += mp.sinpi(2 * t)
        Sk = (C * C + S * S) / w.N
        e_dd = max(abs(float(mp.mpf(float(nd[0, k])) + mp.mpf(float(nd[1, k])) - C)),
                   abs(float(mp.mpf(float(nd[2, k])) + mp.mpf(float(nd[3, k])) - S)))
        e_64 = max(abs(float(mp.mpf(float(nf[0, k])) - C)), abs(float(mp.mpf(float(nf[2, k])) - S)))
        sd = (mp.mpf(float(nd[0, k])) + mp.mpf(float(nd[1, k]))) ** 2 + (mp.mpf(float(nd[2, k])) + mp.mpf(float(nd[3, k]))) ** 2
        rows.append({"k": int(k), "n": [int(x) for x in nh[k]], "S_mp256": float(Sk),
                     "abs_err_S_dd": float(abs(sd / w.N - Sk)), "abs_err_nk_dd": e_dd, "abs_err_nk_fp64": e_64})
    return {"sampled_k": rows, "max_abs_err_nk_dd_over_N": max(r["abs_err_nk_dd"] for r in rows) / w.N,
            "max_abs_err_nk_fp64_over_N": max(r["abs_err_nk_fp64"] for r in rows) / w.N}


def cpu_baseline(d, N, chi, cfg_id, vkind=0):
    """The oracle (plain double-double C, all host cores) on a bounded sample of the
    workload: the n~ pass over a slice of the wavevectors and the gradient pass over a
    slice of the particles; the rate is pairs per second for both passes together."""
    import numpy as np

    from oracle import oracle as O
    from paper_2304_09139_amd import inputs

    R2, M = O.cutoff(d, N, chi)
    n = O.wavevectors(d, R2)
    v = O.weights(n, R2, vkind) if vkind else None
    pos = inputs.config_positions(cfg_id, d, N, 0)
    threads = O.num_threads()
    k_s = max(1, min(M, int(8.0e7 / N)))           # pass-1 sample: k_s x N pairs
    t = time.perf_counter()
    nkv = O.nk(n, pos, 0, k_s)
    t1 = time.perf_counter() - t
    j_s = max(1, min(N, int(8.0e7 / M)))           # pass-2 sample: j_s x M pairs
    t = time.perf_counter()
    O.grad(n, v, pos, nkv, js=np.arange(j_s))
    t2 = time.perf_counter() - t
    per_pair = t1 / (k_s * N) + t2 / (j_s * M)     # seconds per pair, both passes
    return {"value": 1.0 / per_pair, "unit": "dd pairs/s (Phi+grad)", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"n~ pass over {k_s} of {M} wavevectors x all {N} particles ({t1:.1f} s) and gradient "
                      f"pass over {j_s} of {N} particles x all {M} wavevectors ({t2:.1f} s), seed 0"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="d3_N30000_chi0.45_w", choices=sorted(WORKLOADS))
    ap.add_argument("--segment", type=int, default=None,
                    help="L-BFGS iterations per step for workloads timed in quench segments (the default "
                         "workload: 100); 0 times whole quenches instead")
    ap.add_argument("--no-c2", action="store_true",
                    help="segment workloads: skip the whole-quench block of d=3, N=8000, chi=0.45")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--progress", type=float, default=0.0,
                    help="seconds between the library's progress lines on stderr (0: none)")
    ap.add_argument("--no-staged", action="store_true",
                    help="skip the staged-precision quenches of the same starts (single and batched workloads)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched workloads: skip timing the same configurations one at a time")
    ap.add_argument("--mp-k", type=int, default=32, help="sampled wavevectors of the 256-bit report")
    ap.add_argument("--mp-report", action="store_true",
                    help="report the 256-bit error of n~ at sampled k of the final configuration")
    ap.add_argument("--method", default="lbfgs", choices=("lbfgs", "fire"),
                    help="minimiser of the single-configuration and batched quenches")
    ap.add_argument("--serve-phase", default="all", choices=("all", "closed", "open", "sequential"),
                    help="served workloads: run every phase (default) or one: the closed run (all requests at "
                         "once: capacity), the Poisson run at 0.7 x --serve-capacity, or the one-at-a-time path")
    ap.add_argument("--serve-range", default=None,
                    help="a:b -- the chosen phase runs requests a..b-1 of the stream only (one at a time: the "
                         "time over the stream is the sum over ranges; Poisson: a window of the stream with its "
                         "own arrival gaps, from an empty server)")
    ap.add_argument("--serve-capacity", type=float, default=None,
                    help="configs/s of a closed run, for --serve-phase open")
    ap.add_argument("--history", type=int, default=8, help="L-BFGS history length of single-configuration quenches")
    ap.add_argument("--stall-window", type=int, default=None,
                    help="stall window of single-configuration quenches (default: the library's, 50; FIRE 200)")
    ap.add_argument("--precision", default="dd", choices=("dd", "staged", "fp64"),
                    help="evaluation precision of the quench (staged: FP64 until it stalls, then dd)")
    ap.add_argument("--evals", type=int, default=0,
                    help="instead of quenches, run this many Phi + gradient evaluations of the first start and "
                         "then one 1 GiB device copy (the calibration kernel for the HBM counters)")
    args = ap.parse_args()
    args.steps_set = args.steps is not None
    if args.steps is None:
        args.steps = 5
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: this build measures the single-GPU hot path; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2304_09139_amd import inputs, ss

    wl = WORKLOADS[args.workload]
    if args.segment is None:
        args.segment = wl.get("segment", 0)
    if args.segment > 0 and args.evals == 0:
        if not args.steps_set:
            args.steps = 10
        return bench_segments(args, wl)
    if wl.get("evals_only"):
        return bench_evals(args, wl)
    if "batch" in wl:
        return bench_batch(args, wl)
    if "serve" in wl:
        return bench_serve(args, wl)
    d, N, chi = wl["d"], wl["N"], wl["chi"]
    ctx = ss.Context(0)
    ctx.progress(args.progress)
    vkind = wl.get("vkind", 0)
    w = ss.Workload.from_chi(d, N, chi, vkind=vkind)
    n = ctx.wavevectors(d, w.R2)
    v = ctx.weights(w, n) if vkind else None
    mopts = dict(s_floor=FLOOR, precision=args.precision, method=args.method, history=args.history)
    if args.method == "fire":
        mopts["stall_window"] = 200
    if args.stall_window:
        mopts["stall_window"] = args.stall_window
    # all starting configurations resident in HBM before the timed region
    starts = [torch.from_numpy(inputs.config_positions(wl["cfg_id"], d, N, r)).cuda()
              for r in range(args.warmup + args.steps)]
    ctx.workspace(w, 1)
    torch.cuda.synchronize()
    if args.evals > 0:
        out = ctx.energy_grad(w, n, v, starts[0], grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.evals):
            ctx.energy_grad(w, n, v, starts[0], grad=True, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        evict = torch.full((1 << 29,), 3, dtype=torch.uint8, device="cuda")  # > the 256 MB MALL
        dst = torch.empty_like(src)
        dst.copy_(src)
        del evict
        torch.cuda.synchronize()
        print(json.dumps({"mode": "evals", "evals": args.evals, "ms_per_eval": dt / args.evals * 1e3,
                          "pairs_per_s": w.M * N * args.evals / dt, "copy_bytes": src.numel()}), flush=True)
        ctx.close()
        return
    for r in range(args.warmup):
        ctx.minimize(w, n, v, starts[r], **mopts)
    torch.cuda.synchronize()
    # inside the timed region only the roofline kernel carries timing events
    ctx.profile(True, kernels=("grad",))
    ctx.profile_read("grad", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for r in range(args.warmup, args.warmup + args.steps):
        results.append(ctx.minimize(w, n, v, starts[r], **mopts))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {"grad": ctx.profile_read("grad", reset=True)}
    staged = None
    if args.precision == "dd" and args.method == "lbfgs" and not args.no_staged:
        # the same starts quenched with staged precision (FP64 descent, dd finish)
        # to the same floor, timed on their own
        ctx.profile(False)
        xs = [torch.from_numpy(inputs.config_positions(wl["cfg_id"], d, N, r)).cuda()
              for r in range(args.warmup, args.warmup + args.steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sres = [ctx.minimize(w, n, v, x, **dict(mopts, precision="staged")) for x in xs]
        torch.cuda.synchronize()
        st_el = time.perf_counter() - t1
        st_conv = sum(1 for r in sres if r["status"] == "converged")
        staged = {"configs_per_s": st_conv / st_el, "converged": f"{st_conv}/{len(sres)}",
                  "smax_worst": max(r["smax"][0] for r in sres),
                  "iters_mean": sum(r["iters"] for r in sres) / len(sres),
                  "iters_fp64_mean": sum(r["iters_fp64"] for r in sres) / len(sres)}
        ctx.profile(True, kernels=("grad",))
    if args.precision != "dd":   # double-double gradient launches timed on their own
        ctx.profile(True, kernels=("grad",))
        ctx.profile_read("grad", reset=True)
        out_g = ctx.energy_grad(w, n, v, starts[0], grad=True)
        for _ in range(9):
            ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_g)
        torch.cuda.synchronize()
        prof["grad_dd"] = ctx.profile_read("grad", reset=True)
    # per-pass times of a plain evaluation (outside the timed region)
    ctx.profile(True)
    for k in ("nk", "table"):
        ctx.profile_read(k, reset=True)
    out_e = ctx.energy_grad(w, n, v, starts[0], grad=True)
    for _ in range(9):
        ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_e)
    torch.cuda.synchronize()
    prof["nk"] = ctx.profile_read("nk", reset=True)
    prof["table"] = ctx.profile_read("table", reset=True)
    ctx.profile_read("grad", reset=True)
    ctx.profile(False)
    # one Phi + gradient evaluation (ss_energy_grad) timed with HIP events on its
    # stream: the median of 50 after 5 warm-ups
    for _ in range(5):
        ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_e)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for a, b in ev:
        a.record()
        ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_e)
        b.record()
    torch.cuda.synchronize()
    t_eval = sorted(a.elapsed_time(b) for a, b in ev)[25] * 1e-3

    evals = sum(r["evals"] for r in results)
    evals_fp64 = sum(r["evals_fp64"] for r in results)
    pairs = w.M * N * (evals - evals_fp64)   # double-double pairs (the metric)
    value = pairs / elapsed
    converged = sum(1 for r in results if r["status"] == "converged")
    launches, ms = prof["grad"]
    # the roofline is that of the double-double gradient pass: in a staged run
    # the FP64 launches are left out of the average
    if args.precision != "dd":
        launches, ms = prof["grad_dd"]
    nk_l, nk_ms = prof["nk"]
    out = {
        "metric": "dd particle-wavevector pairs/s (Phi+grad) and configs/s at stated max S(k) floor",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"dd": "dd", "staged": "f64 then dd", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded uniform-random starts, the paper's Poisson initial condition)",
        "config": {"workload": f"{'FIRE' if args.method == 'fire' else 'L-BFGS'} quench to S_max <= {FLOOR:g}, "
                               f"d={d}, N={N}, chi={chi}, "
                               + ("v(k)=(1-|k|/K)^2" if vkind else "v(k)=1")
                               + ("" if args.precision == "dd" else f", {args.precision} precision"),
                   "d": d, "N": N, "chi": chi, "R2": w.R2, "M": w.M, "s_floor": FLOOR, "vkind": vkind,
                   "precision": args.precision, "method": args.method, "history": args.history,
                   "stall_window": mopts.get("stall_window", 50),
                   "parallelism": "single GPU"},
        "configs_per_s": converged / elapsed,
        "converged": f"{converged}/{args.steps}",
        "statuses": sorted({r["status"] for r in results}),
        "staged_precision": staged if staged is None else dict(
            staged, speedup_configs_per_s=staged["configs_per_s"] / (converged / elapsed)),
        "paper_context": "the paper reports S_max ~ 1e-51 and Phi/eps0 ~ 1e-46 at d=2, N=2e6 (double-double, "
                         "FIRE, pyCudaPack on an unnamed GPU); it gives no throughput figure",
        "smax_worst": max(r["smax"][0] for r in results),
        "iters_mean": sum(r["iters"] for r in results) / len(results),
        "iters_fp64_mean": sum(r["iters_fp64"] for r in results) / len(results),
        "evals_fp64_mean": evals_fp64 / len(results),
        "fp64_pairs_per_s": w.M * N * evals_fp64 / elapsed,
        "evals_mean": evals / len(results),
        # the whole quench against the FP64 peak: both passes' inner-loop flops per
        # pair at the measured pair rate, minimiser overhead included
        "path_frac_of_fp64_peak": value * (FLOPS_PER_PAIR["nk"] + FLOPS_PER_PAIR["grad"]) / PEAK_FP64_FLOPS,
        "nk_pass_frac_of_fp64_peak": (FLOPS_PER_PAIR["nk"] * w.M * N / (nk_ms / max(nk_l, 1) * 1e-3))
        / PEAK_FP64_FLOPS if nk_l else None,
        # one evaluation on its own: M N / t_eval, and the paper's two-sums count 2 M N / t_eval
        "eval_pairs_per_s": w.M * N / t_eval,
        "eval_two_sums_per_s": 2 * w.M * N / t_eval,
        "eval_ms_median": t_eval * 1e3,
        "eval_ms_nk_pass": nk_ms / max(nk_l, 1),
        "eval_ms_grad_pass": ms / max(launches, 1),
        "eval_ms_table": prof["table"][1] / max(prof["table"][0], 1),
        "roofline": roofline("grad", "k_grad (gradient pass)", launches, ms, w.M * N * launches,
                             args.workload if args.precision == "dd" else None),
    }
    if args.precision == "staged" or args.mp_report:
        # 256-bit error of the reported n~ / S(k) at the final positions of the last quench
        rep = {"final": mp_error_report(ctx, w, n, v, starts[args.warmup + args.steps - 1], count=args.mp_k,
                                        label="at the end")}
        if args.precision == "staged":
            # the switch point: the FP64 stage alone from the same start (the same
            # kernels and stage parameters, so the same iterates)
            xs = torch.from_numpy(inputs.config_positions(wl["cfg_id"], d, N, args.warmup + args.steps - 1)).cuda()
            r64 = ctx.minimize(w, n, v, xs, **dict(mopts, precision="fp64",
                                                   s_floor=max(FLOOR, ss.DEFAULT_MIN_OPTS["fp64_floor"]),
                                                   max_ls_fail=1))
            rep["switch"] = dict(mp_error_report(ctx, w, n, v, xs, count=args.mp_k, label="at the switch"),
                                 fp64_iters=r64["iters"], smax_fp64=r64["smax"][0])
        out["error_vs_mp256"] = rep
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, N, chi, wl["cfg_id"])
    print(json.dumps(out), flush=True)
    ctx.close()


def quench_block(ctx, count, precision_list=("dd", "staged")):
    """Whole quenches of `count` fresh seeded starts of d=3, N=8000, chi=0.45 to
    S_max <= FLOOR, one at a time through ss_minimize, per precision: configs/s
    at the floor (one warm-up quench first)."""
    import torch

    from paper_2304_09139_amd import inputs, ss

    d, N, chi = 3, 8000, 0.45
    w = ss.Workload.from_chi(d, N, chi)
    n = ctx.wavevectors(d, w.R2)
    ctx.workspace(w, 1)
    out = {"workload": f"L-BFGS quench to S_max <= {FLOOR:g}, d={d}, N={N}, chi={chi}, v(k)=1",
           "R2": w.R2, "M": w.M, "quenches": count}
    for prec in precision_list:
        xs = [torch.from_numpy(inputs.config_positions(2, d, N, r)).cuda() for r in range(count + 1)]
        torch.cuda.synchronize()
        ctx.minimize(w, n, None, xs[0], s_floor=FLOOR, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [ctx.minimize(w, n, None, x, s_floor=FLOOR, precision=prec) for x in xs[1:]]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        conv = sum(1 for r in res if r["status"] == "converged")
        dd_evals = sum(r["evals"] - r["evals_fp64"] for r in res)
        out[prec] = {"configs_per_s": conv / el, "converged": f"{conv}/{count}", "seconds": el,
                     "smax_worst": max(r["smax"][0] for r in res),
                     "iters_mean": sum(r["iters"] for r in res) / count,
                     "iters_fp64_mean": sum(r["iters_fp64"] for r in res) / count,
                     "dd_pairs_per_s": w.M * N * dd_evals / el}
        print(f"[bench] d=3 N=8000 quenches ({prec}) done", file=sys.stderr, flush=True)
    if "dd" in out and "staged" in out:
        out["staged_over_dd_configs_per_s"] = out["staged"]["configs_per_s"] / out["dd"]["configs_per_s"]
    return out


def bench_segments(args, wl):
    """A step is a segment of `args.segment` L-BFGS iterations of one quench from a
    fresh seeded uniform start (the paper's Poisson initial condition), s_floor =
    FLOOR: every iteration evaluates Phi + gradient over all M N particle-
    wavevector pairs at least once (the trial point of the line search) and runs
    the minimiser's direction, step and history update on the device.  The
    cutoff, the wavevector set and the weights (once per configuration) are built
    before the timed region; the starts are resident in HBM."""
    import torch

    from paper_2304_09139_amd import inputs, ss

    d, N, chi, vkind = wl["d"], wl["N"], wl["chi"], wl.get("vkind", 0)
    iters = args.segment
    ctx = ss.Context(0)
    ctx.progress(args.progress)
    t_setup = time.perf_counter()
    w = ss.Workload.from_chi(d, N, chi, vkind=vkind)      # cutoff
    n = ctx.wavevectors(d, w.R2)                           # wavevector set
    v = ctx.weights(w, n) if vkind else None               # weights
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    starts = [torch.from_numpy(inputs.config_positions(wl["cfg_id"], d, N, r)).cuda()
              for r in range(args.warmup + args.steps)]
    ctx.workspace(w, 1)
    mopts = dict(s_floor=FLOOR, max_iter=iters, precision=args.precision)
    torch.cuda.synchronize()
    for r in range(args.warmup):
        ctx.minimize(w, n, v, starts[r], **mopts)
    torch.cuda.synchronize()
    ctx.profile(True, kernels=("nk", "grad"))
    for k in ("nk", "grad"):
        ctx.profile_read(k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for r in range(args.warmup, args.warmup + args.steps):
        results.append(ctx.minimize(w, n, v, starts[r], **mopts))
        print(f"[bench] segment {len(results)}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {k: ctx.profile_read(k, reset=True, work=True) for k in ("nk", "grad")}
    ctx.profile(False)
    evals = sum(r["evals"] for r in results)
    evals_fp64 = sum(r["evals_fp64"] for r in results)
    iters_done = sum(r["iters"] for r in results)
    pairs = w.M * N * (evals - evals_fp64)
    value = pairs / elapsed
    # one Phi + gradient evaluation on its own (ss_energy_grad), HIP events on its
    # stream: the median of 20 after 3 warm-ups
    out_e = ctx.energy_grad(w, n, v, starts[0], grad=True)
    for _ in range(3):
        ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_e)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for a, b in ev:
        a.record()
        ctx.energy_grad(w, n, v, starts[0], grad=True, out=out_e)
        b.record()
    torch.cuda.synchronize()
    t_eval = sorted(a.elapsed_time(b) for a, b in ev)[10] * 1e-3
    rl = {k: roofline(k, {"nk": "k_nk (n~(k) pass)", "grad": "k_grad (gradient pass)"}[k], prof[k][0],
                      prof[k][1], prof[k][2], args.workload if args.precision == "dd" else None)
          for k in ("nk", "grad")}
    dom = max(("nk", "grad"), key=lambda k: prof[k][1])   # the kernel with the larger share of time
    out = {
        "metric": "dd particle-wavevector pairs/s (Phi+grad) and configs/s at stated max S(k) floor",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"dd": "dd", "staged": "f64 then dd", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded uniform-random starts, the paper's Poisson initial condition)",
        "config": {"workload": f"{iters}-iteration L-BFGS segments of a quench toward S_max <= {FLOOR:g} from fresh "
                               f"seeded starts, d={d}, N={N}, chi={chi}, "
                               + ("v(k)=(1-|k|/K)^2, K^2=(R2+1/2)(2pi/L)^2" if vkind else "v(k)=1")
                               + ("" if args.precision == "dd" else f", {args.precision} precision"),
                   "d": d, "N": N, "chi": chi, "R2": w.R2, "M": w.M, "vkind": vkind, "s_floor": FLOOR,
                   "iters_per_step": iters, "precision": args.precision, "method": "lbfgs",
                   "parallelism": "single GPU"},
        "configs_per_s": None,
        "configs_per_s_note": "a quench of this configuration takes minutes (tens of thousands of iterations); "
                              "configs/s at the floor is reported for d=3, N=8000 in whole_quenches",
        "iters_per_step": iters_done / len(results),
        "evals_per_step": evals / len(results),
        "status": sorted({r["status"] for r in results}),
        "phi_after_step_max": max(r["phi"][0] for r in results),
        "ms_per_iteration": elapsed / iters_done * 1e3,
        "setup_ms_cutoff_wavevectors_weights": t_setup * 1e3,
        "eval_ms_median": t_eval * 1e3,
        "eval_pairs_per_s": w.M * N / t_eval,
        "eval_two_sums_per_s": 2 * w.M * N / t_eval,
        "pass_ms": {k: prof[k][1] / max(prof[k][0], 1) for k in ("nk", "grad")},
        "roofline": rl[dom],
        "roofline_other_pass": rl["grad" if dom == "nk" else "nk"],
        # whole step against the peak: both passes' inner-loop flops at the step's pair rate
        "path_frac_of_fp64_peak": value * (FLOPS_PER_PAIR["nk"] + FLOPS_PER_PAIR["grad"]) / PEAK_FP64_FLOPS,
        "paper_context": "the paper reports S_max ~ 1e-51 and Phi/eps0 ~ 1e-46 at d=2, N=2e6 (double-double, "
                         "FIRE, pyCudaPack on an unnamed GPU); it gives no throughput figure",
    }
    if not args.no_c2:
        out["whole_quenches"] = quench_block(ctx, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, N, chi, wl["cfg_id"], vkind)
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_evals(args, wl):
    """Single Phi + gradient evaluations (ss_energy_grad) of one configuration,
    timed with HIP events on the call's stream after one warm-up evaluation."""
    import torch

    from paper_2304_09139_amd import inputs, ss

    d, N, chi = wl["d"], wl["N"], wl["chi"]
    ctx = ss.Context(0)
    w = ss.Workload.from_chi(d, N, chi)
    n = ctx.wavevectors(d, w.R2)
    x = torch.from_numpy(inputs.config_positions(wl["cfg_id"], d, N, 0)).cuda()
    ws_bytes = ctx.workspace_size(w, 0)
    out = ctx.energy_grad(w, n, None, x, grad=True)
    torch.cuda.synchronize()
    steps = args.steps if args.steps_set else 3
    ctx.profile(True)
    for k in ("table", "nk", "grad"):
        ctx.profile_read(k, reset=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        ctx.energy_grad(w, n, None, x, grad=True, out=out)
        b.record()
        print(f"[bench] evaluation done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    prof = {k: ctx.profile_read(k, reset=True) for k in ("table", "nk", "grad")}
    ctx.profile(False)
    t = sorted(a.elapsed_time(b) for a, b in ev)[steps // 2] * 1e-3
    pairs = w.M * N
    out = {
        "metric": "dd particle-wavevector pairs/s of one Phi + gradient evaluation",
        "value": pairs / t, "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "dd",
        "data": "synthetic (seeded uniform-random positions, the paper's Poisson initial condition)",
        "config": {"workload": f"one Phi + gradient evaluation, d={d}, N={N}, chi={chi}, v(k)=1 (the paper's "
                               f"production shape)", "d": d, "N": N, "chi": chi, "R2": w.R2, "M": w.M,
                   "parallelism": "single GPU"},
        "two_sums_per_s": 2 * pairs / t,
        "workspace_gb": ws_bytes / 1e9,
        "pass_ms": {k: v[1] / max(v[0], 1) for k, v in prof.items()},
        "nk_pass_frac_of_fp64_peak": FLOPS_PER_PAIR["nk"] * pairs / (prof["nk"][1] / max(prof["nk"][0], 1) * 1e-3)
        / PEAK_FP64_FLOPS,
        "grad_pass_frac_of_fp64_peak": FLOPS_PER_PAIR["grad"] * pairs / (prof["grad"][1] / max(prof["grad"][0], 1)
                                                                          * 1e-3) / PEAK_FP64_FLOPS,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_batch(args, wl):
    """Batched quenches: a step is one batch of `count` independent quenches from
    fresh starts, all to S_max <= FLOOR, through ss_minimize_batch.  The same
    configurations quenched one at a time with ss_minimize are timed once
    beside it (the launch-bound way of running them)."""
    import torch

    from paper_2304_09139_amd import inputs, ss

    count = wl["batch"]
    shapes = inputs.batch_shapes(count, seed=wl["shape_seed"])
    from paper_2304_09139_amd.tune import load_tiles

    ctx_tuned = bool(load_tiles())
    ctx = ss.Context(0, tiles="tuned")
    ctx.progress(args.progress)
    works = [ss.Workload.from_chi(d, N, chi) for d, N, chi in shapes]
    steps = args.steps if args.steps_set else 2
    starts = [[torch.from_numpy(inputs.config_positions(wl["cfg_id"], w.d, w.N, 1000 * r + i)).cuda()
               for i, w in enumerate(works)] for r in range(args.warmup + steps)]
    opts = dict(s_floor=FLOOR, precision=args.precision, method=args.method)
    if args.method == "fire":
        opts["stall_window"] = 200
    need = ctx.batch_workspace_size(works, [dict(ss.DEFAULT_MIN_OPTS, **opts)] * count)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for r in range(args.warmup):
        ctx.minimize_batch(works, starts[r], opts=opts, ws=ws)
    torch.cuda.synchronize()
    ctx.profile(True, kernels=("grad",))
    ctx.profile_read("grad", reset=True)
    t0 = time.perf_counter()
    results = []
    for r in range(args.warmup, args.warmup + steps):
        results.extend(ctx.minimize_batch(works, starts[r], opts=opts, ws=ws))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, gms, gpairs = ctx.profile_read("grad", reset=True, work=True)
    ctx.profile(False)
    # double-double pairs (the metric); FP64 evaluations of staged runs apart
    pairs = sum(w.M * w.N * (r["evals"] - r["evals_fp64"]) for w, r in zip(works * steps, results))
    pairs64 = sum(w.M * w.N * r["evals_fp64"] for w, r in zip(works * steps, results))
    converged = sum(1 for r in results if r["status"] == "converged")
    staged = None
    if args.precision == "dd" and not args.no_staged:
        # the last step's batch again with staged precision (FP64 descent, each
        # configuration switching to double-double on its own), same floor
        xs = [torch.from_numpy(inputs.config_positions(wl["cfg_id"], w.d, w.N, 1000 * (args.warmup + steps - 1) + i))
              .cuda() for i, w in enumerate(works)]
        sopts = dict(opts, precision="staged")
        wss = torch.empty(ctx.batch_workspace_size(works, [dict(ss.DEFAULT_MIN_OPTS, **sopts)] * count),
                          dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sres = ctx.minimize_batch(works, xs, opts=sopts, ws=wss)
        torch.cuda.synchronize()
        st_el = time.perf_counter() - t1
        st_conv = sum(1 for r in sres if r["status"] == "converged")
        dd_last = sum(1 for r in results[-count:] if r["status"] == "converged") / (elapsed / steps)
        staged = {"configs_per_s": st_conv / st_el, "converged": f"{st_conv}/{count}",
                  "smax_worst": max(r["smax"][0] for r in sres),
                  "iters_mean": sum(r["iters"] for r in sres) / count,
                  "iters_fp64_mean": sum(r["iters_fp64"] for r in sres) / count,
                  "speedup_configs_per_s": (st_conv / st_el) / dd_last}
        del wss
    seq_conv, seq_elapsed = 0, float("nan")
    if not args.no_sequential:
        # one at a time (first step's starts again, fresh copies), timed once
        seq = [torch.from_numpy(inputs.config_positions(wl["cfg_id"], w.d, w.N, 1000 * args.warmup + i)).cuda()
               for i, w in enumerate(works)]
        wsn = [ctx.wavevectors(w.d, w.R2) for w in works]
        ctx.workspace(max(works, key=lambda w: ctx.workspace_size(w, 1)), 1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the plain path: double-double, one configuration per ss_minimize call
        seq_res = [ctx.minimize(w, n, None, x, **dict(opts, precision="dd")) for w, n, x in zip(works, wsn, seq)]
        torch.cuda.synchronize()
        seq_elapsed = time.perf_counter() - t1
        seq_conv = sum(1 for r in seq_res if r["status"] == "converged")
    lat = sorted(r["seconds"] for r in results[-count:])
    out = {
        "metric": "dd particle-wavevector pairs/s (Phi+grad) and configs/s at stated max S(k) floor",
        "value": pairs / elapsed,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"dd": "dd", "staged": "f64 then dd", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded uniform-random starts, the paper's Poisson initial condition)",
        "config": {"workload": f"batched {'FIRE' if args.method == 'fire' else 'L-BFGS'} quenches to "
                               f"S_max <= {FLOOR:g}: {count} configurations, "
                               f"d in {{2,3}}, N log-uniform in [500, 5000], chi in {{0.2, 0.35, 0.45}}, v(k)=1"
                               + ("" if args.precision == "dd" else f", {args.precision} precision"),
                   "configs": count, "s_floor": FLOOR, "precision": args.precision, "method": args.method,
                   "parallelism": "single GPU"},
        "configs_per_s": converged / elapsed,
        "converged": f"{converged}/{len(results)}",
        "iters_mean": sum(r["iters"] for r in results) / len(results),
        "fp64_pairs_per_s": pairs64 / elapsed,
        "staged_precision": None if staged is None else dict(
            staged, speedup_vs_one_at_a_time_dd=None if args.no_sequential else
            staged["configs_per_s"] / (seq_conv / seq_elapsed)),
        "smax_worst": max(r["smax"][0] for r in results),
        "one_at_a_time": None if args.no_sequential else {
            "configs_per_s": seq_conv / seq_elapsed, "seconds": seq_elapsed, "converged": f"{seq_conv}/{count}",
            "precision": "dd"},
        "speedup_vs_one_at_a_time": None if args.no_sequential else (converged / elapsed) / (seq_conv / seq_elapsed),
        "tiles": "tuned table" if ctx_tuned else "built-in",
        "latency_s": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(0.99 * len(lat)))],
                      "max": lat[-1]},
        "roofline": dict(roofline("grad", "kb_grad (batched gradient pass)", launches, gms, gpairs, None),
                         flop_count=f"{FLOPS_PER_PAIR['grad']} FP64 flops per pair (FMA = 2) x the M N of every "
                                    f"configuration listed in each launch"),
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def bench_serve(args, wl):
    """Served quenches: the request stream is first submitted all at once (the
    capacity, configs/s), then again with Poisson arrivals at 0.7 x that capacity;
    latencies are from ss_submit until the result was copied out."""
    import numpy as np

    from paper_2304_09139_amd import inputs, ss
    from paper_2304_09139_amd.tune import load_tiles

    count = wl["serve"]
    n_min, n_max = wl.get("n_min", 500), wl.get("n_max", 5000)
    stream = inputs.serve_stream(count, seed=wl["stream_seed"], n_min=n_min, n_max=n_max)
    works = [ss.Workload.from_chi(d, N, chi) for d, N, chi, _ in stream]
    # a request is (d, N, chi, seed): the server draws the uniform start of the
    # seed itself (the same positions as inputs.config_positions)
    seeds = [inputs.stream_seed(wl["cfg_id"], i) for i in range(count)]
    ctx = ss.Context(0, tiles="tuned")
    ctx.progress(args.progress)  # progress lines of single quenches (one-at-a-time phase)
    arena = wl.get("arena_gb", 8) << 30
    ctx.server_start(arena, max_slots=512)

    trace = []

    def run(times, sel):
        """Submit request sel[i] at times[i] (seconds from the start), collect all;
        the server's running and queued counts are sampled every 0.25 s."""
        trace.clear()
        t0 = time.perf_counter()
        t_sample = -1.0
        tickets = []
        done = {}
        i = 0
        last = 0.0
        n = len(sel)
        while len(done) < n:
            now = time.perf_counter() - t0
            while i < n and times[i] <= now:
                r = sel[i]
                tickets.append(ctx.submit(works[r], None, seed=seeds[r], s_floor=FLOOR, precision=args.precision))
                i += 1
                if i % 25 == 0 and times[i - 1] == 0.0:
                    print(f"[serve] {i}/{n} submitted, t {time.perf_counter() - t0:.1f}s", file=sys.stderr,
                          flush=True)
            for k, t in enumerate(tickets):
                if k not in done:
                    r = ctx.poll(t)
                    if r is not None:
                        done[k] = r[0]
            if time.perf_counter() - t0 - t_sample >= 0.25:
                t_sample = time.perf_counter() - t0
                st = ctx.server_stats()
                trace.append((t_sample, st["running"], st["queued"]))
            if time.perf_counter() - t0 - last >= 10.0:  # a progress line every 10 s
                last = time.perf_counter() - t0
                print(f"[serve] {len(done)}/{n} done, {i} submitted, t {last:.1f}s", file=sys.stderr, flush=True)
            time.sleep(0.0005)
        return time.perf_counter() - t0, [done[k] for k in range(n)]

    # warm-up: a few short requests of the smallest configurations (server
    # buffers, first launches)
    small = sorted(range(count), key=lambda i: works[i].M * works[i].N)[:8]
    warm = [ctx.submit(works[i], None, seed=seeds[i], max_iter=2) for i in small]
    for t in warm:
        while ctx.poll(t) is None:
            time.sleep(0.001)
    print(f"[serve] warm-up done; {count} requests, N {min(w.N for w in works)}..{max(w.N for w in works)}",
          file=sys.stderr, flush=True)

    def occupancy(tr):
        run_counts = np.array([r for _, r, _ in tr]) if tr else np.zeros(1)
        return {"mean_running": float(run_counts.mean()), "frac_time_one_running": float((run_counts <= 1).mean()),
                "max_running": int(run_counts.max())}

    def latency(res):
        lat = np.array([r["seconds"] for r in res])
        return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "max": float(lat.max())}

    phase = args.serve_phase
    # --serve-range a:b runs the chosen phase on requests a..b-1 of the stream (a
    # window of the Poisson stream keeps its own arrival gaps, from an empty server)
    a, b = (int(v) for v in args.serve_range.split(":")) if args.serve_range else (0, count)
    sel = list(range(a, min(b, count)))
    sel_works = [works[i] for i in sel]
    out_extra = {"requests": [sel[0], sel[-1] + 1]} if args.serve_range else {}
    closed, opened, cap, closed_s, open_s, lam = None, None, args.serve_capacity, None, None, None
    if phase in ("all", "closed"):
        closed_s, closed = run([0.0] * len(sel), sel)
        print(f"[serve] closed run: {closed_s:.1f}s", file=sys.stderr, flush=True)
        cap = sum(1 for r in closed if r["status"] == "converged") / closed_s
        out_extra["occupancy_closed"] = occupancy(trace)
        out_extra["server_counters_closed"] = ctx.server_stats()
        out_extra["closed_batch_latency_s"] = latency(closed)
        # where the time goes: the share of the pair work in the requests with N >= 2e4
        out_extra["pair_work_share_N_ge_2e4"] = (
            sum(w.M * w.N * r["evals"] for w, r in zip(sel_works, closed) if w.N >= 20000)
            / max(1, sum(w.M * w.N * r["evals"] for w, r in zip(sel_works, closed))))
    if phase in ("all", "open"):
        if not cap:
            raise SystemExit("--serve-phase open needs --serve-capacity (configs/s of the closed run)")
        lam = 0.7 * cap
        t_start = stream[sel[0] - 1][3] if sel[0] > 0 else 0.0
        open_s, opened = run([(stream[i][3] - t_start) / lam for i in sel], sel)
        out_extra["occupancy_poisson"] = occupancy(trace)
        out_extra["latency_s"] = latency(opened)
    out_extra["server_counters_total"] = ctx.server_stats()
    ctx.server_stop()
    seq_conv, seq_s = 0, float("nan")
    if phase in ("all", "sequential") and not args.no_sequential:
        # the same requests quenched one at a time with ss_minimize (same floor and
        # precision)
        import torch

        xs = [torch.from_numpy(inputs.uniform_positions(works[i].d, works[i].N, seeds[i])).cuda() for i in sel]
        ns = [ctx.wavevectors(works[i].d, works[i].R2) for i in sel]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for q, (w, n, x) in enumerate(zip([works[i] for i in sel], ns, xs)):
            tq = time.perf_counter()
            r = ctx.minimize(w, n, None, x, s_floor=FLOOR, precision=args.precision)
            seq_conv += r["status"] == "converged"
            # one line per request: a window cut short still says what it finished
            print(f"[serve] one at a time: request {sel[q]} d={w.d} N={w.N} {r['status']} "
                  f"{time.perf_counter() - tq:.2f}s ({q + 1}/{len(sel)}, t {time.perf_counter() - t1:.1f}s)",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t1
        out_extra["one_at_a_time"] = {"configs_per_s": seq_conv / seq_s, "seconds": seq_s,
                                      "converged": f"{seq_conv}/{len(sel)}", "requests": [a, a + len(sel)],
                                      "precision": args.precision}
        if cap:
            out_extra["capacity_vs_one_at_a_time"] = cap / (seq_conv / seq_s)
    # the line's value: the Poisson run when there is one, else the closed run
    res, el = (opened, open_s) if opened is not None else (closed, closed_s)
    if res is None:
        res, el = [], float("nan")
    pairs = sum(w.M * w.N * (r["evals"] - r["evals_fp64"]) for w, r in zip(sel_works, res))
    conv = sum(1 for r in res if r["status"] == "converged")
    out = {
        "metric": "dd particle-wavevector pairs/s (Phi+grad) and configs/s at stated max S(k) floor",
        "value": pairs / el if res else None,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": el * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"dd": "dd", "staged": "f64 then dd", "fp64": "f64"}[args.precision],
        "data": "synthetic (seeded uniform-random starts, the paper's Poisson initial condition)",
        "config": {"workload": f"{count} served L-BFGS quenches to S_max <= {FLOOR:g}, d in {{2,3}}, "
                               f"N log-uniform in [{n_min}, {n_max}], chi uniform in [0.1, 0.49]"
                               + (", Poisson arrivals at 0.7 x capacity" if opened is not None else
                                  ", all submitted at once" if closed is not None else "")
                               + ("" if args.precision == "dd" else f", {args.precision} precision")
                               + (f", requests {sel[0]}..{sel[-1]} of the stream" if args.serve_range else ""),
                   "requests": count, "s_floor": FLOOR, "precision": args.precision, "phase": phase,
                   "parallelism": "single GPU"},
        "configs_per_s": conv / el if res else None,
        "converged": f"{conv}/{len(res)}",
        "capacity_configs_per_s": cap,
        "arrival_rate_per_s": lam,
        "tiles": "tuned table" if load_tiles() else "built-in",
    }
    out.update(out_extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
