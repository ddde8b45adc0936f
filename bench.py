"""Benchmark of the hot path on one MI355X.

One bench step = one full adaptive integration of the single large instance
(M = 65536, rank-3 kernel (i/j)^a + (j/i)^a + 2 with a = 0.45, lam = 0.005,
monodisperse start, Dormand-Prince 5(4) with PI control, rtol 1e-6,
atol 1e-12, t = 0 -> 1e4): every right-hand side, stage combination, error
norm and controller decision of the run.  value = accepted RK steps per
second over the timed runs; ms_per_step = time-to-t_end of one run.

Prints ONE JSON line.  Inputs are synthetic and built on the host, then
moved to HBM before the timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peak HBM3E bandwidth (bytes/s)
HBM_PEAK = 8.0e12

# sources of the right-hand-side kernels; hardware byte counts recorded in
# profiles/ are used only while these files are unchanged
KERNEL_SOURCES = ["common.h", "ff.h", "fft.h", "rhs.h", "integrate.h", "kernels.h", "sched.h",
                  "schedule_table.h", "phases_a.hip", "phases_b.hip", "phases_c.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_M65536_R3.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_16559_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a copy of known size), or None
    if the summary is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    import re
    m = re.search(r"source hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"^\| " + kernel + r" \|[^\n]*\| (\d+) \|\s*$", text, re.M)
    return int(m.group(1)) if m else None


def rhs_bytes(M, R, L):
    """Algorithmic HBM bytes of the three right-hand-side kernels (FP64):
    column pass reads y, U, V and writes R packed spectra; the row-pair pass
    reads them and writes the packed half-length inverse input; the inverse
    column pass reads that plus y and U and writes S."""
    a = 8 * M + 16 * M * R + 16 * L * R
    b = 16 * L * R + 8 * L
    c = 8 * L + 8 * M + 8 * M * R + 8 * M
    return {"phase_a": a, "phase_b": b, "phase_c": c, "rhs": a + b + c}


def step_bytes(M, R, L):
    """Algorithmic HBM bytes of the integrator's stage kernels in a DP5(4)
    attempt (FP64):
      int_a        column pass of stage 2: reads n, k_1, U, V; writes y_2 and
                   R packed spectra (it also reads the previous attempt's
                   error rows for its decision, 16 KiB, not counted);
      int_b        row-pair pass: reads the spectra, writes the packed inverse
                   input;
      int_c_fused  finish of stage 3 fused with the next column pass: reads the
                   packed input, y_3, n, k_1, k_2, U, V; writes k_3, y_4 and the
                   next spectra;
      int_c_last   finish of stage 7: reads the packed input, n_new, n, the five
                   stage vectors with nonzero error weights, U; writes k_7."""
    return {"int_a": 24 * M + 16 * M * R + 16 * L * R,
            "int_b": 16 * L * R + 8 * L,
            "int_c_fused": 8 * L + 48 * M + 16 * M * R + 16 * L * R,
            "int_c_last": 8 * L + 64 * M + 8 * M * R}


def fft_length(M):
    """Transform length the library uses for M sizes: the smallest power of
    two >= 2 M - 2 (the linear convolution of two length-(M-1) inputs fits),
    at least 2^6."""
    return 1 << max(6, max(2 * M - 3, 1).bit_length())


def min_bytes(M, R):
    """Compulsory HBM bytes of one right-hand side (FP64): read n, U and V
    once and write S, with no intermediate spectra."""
    return 8 * M * (2 + 2 * R)


# launches of each stage kernel per DP5(4) attempt (stages 2..7)
STEP_LAUNCHES = {"int_a": 1, "int_b": 6, "int_c_fused": 5, "int_c_last": 1}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(U, V, lam, n0, per_step_rhs, run_rhs=None):
    """The FP64 oracle (plain O(M^2) direct sums) timed on the host: one full
    right-hand side at the start state on all host threads (up to 16) and
    one on a single thread, converted to DP5 steps/s; with run_rhs (the GPU
    run's evaluations to t_end) also the oracle's time to t_end, extrapolated
    as run_rhs times its seconds per right-hand side."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.rhs(U, V, lam, n0, threads=threads)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.rhs(U, V, lam, n0, threads=1)
    dt1 = time.perf_counter() - t0
    model = cpu_model()
    res = {"value": 1.0 / (per_step_rhs * dt), "unit": "accepted steps/s", "cores": threads,
           "kind": "oracle",
           "sample": f"one direct O(M^2 R) right-hand side at M={n0.size} "
                     f"({dt:.2f} s on {threads} threads of {os.cpu_count()} x {model}), "
                     f"times {per_step_rhs} per DP5 step",
           "rhs_evals_per_s": 1.0 / dt,
           "single_thread": {"value": 1.0 / (per_step_rhs * dt1), "rhs_evals_per_s": 1.0 / dt1,
                             "cores": 1, "rhs_s": dt1}}
    if run_rhs:
        res["time_to_t_end_extrapolated_s"] = run_rhs * dt
        res["single_thread"]["time_to_t_end_extrapolated_s"] = run_rhs * dt1
    return res


def plain_small(smol, W, torch, dev):
    """The plain-small workload (M = 512, rank-3 kernel a = 1/3, lam = 0.01,
    monodisperse start, BS3 with PI, rtol 1e-6, atol 1e-12, t_end = 50): one
    GPU run and the oracle's whole trajectory on the host (all threads up to
    16, then one thread), with their end-state difference."""
    import oracle
    c = W.WORKLOADS["plain-small"]
    U, V, lam, n0 = W.workload_instance("plain-small")
    Ud, Vd, nd = (torch.from_numpy(x).to(dev) for x in (U, V, n0))
    args = (lam, nd, c["t_end"], c["rtol"], c["atol"])
    smol.integrate(Ud, Vd, *args, method="bs3", raise_on_error=True)  # plan and graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out, st = smol.integrate(Ud, Vd, *args, method="bs3", raise_on_error=True)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    threads = min(16, os.cpu_count() or 1)
    res = {"gpu": {"time_to_t_end_s": tg, "accepted_steps_per_s": st["n_accept"] / tg,
                   "rhs_evals_per_s": st["n_rhs"] / tg, "n_accept": st["n_accept"],
                   "n_rhs": st["n_rhs"]}}
    for name, th in (("oracle", threads), ("oracle_single_thread", 1)):
        t0 = time.perf_counter()
        ref, rst, _ = oracle.integrate(U, V, lam, n0, c["t_end"], c["rtol"], c["atol"],
                                       method=oracle.BS32, threads=th)
        dt = time.perf_counter() - t0
        res[name] = {"time_to_t_end_s": dt, "cores": th, "accepted_steps_per_s": rst["n_accept"] / dt,
                     "rhs_evals_per_s": rst["n_rhs"] / dt, "n_accept": rst["n_accept"],
                     "n_rhs": rst["n_rhs"]}
    o = out.cpu().numpy()
    res["rel_diff_gpu_vs_oracle"] = float(abs(o - ref).max() / abs(ref).max())
    return res


def copy_ceiling(torch, dev, nbytes, iters=200):
    """Mean time of one device-to-device copy of nbytes (nbytes / 2 read and
    nbytes / 2 written: the same footprint as a kernel that moves nbytes),
    one launch each, timed with events on torch's current stream."""
    n = max(1, nbytes // 16)
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(iters):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / iters
    moved = 16 * n
    return {"bytes": moved, "ms": ms, "GB/s": moved / (ms * 1e-3) / 1e9,
            "frac": moved / (ms * 1e-3) / HBM_PEAK}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--t-end", type=float, default=None, help="shorter runs (profiling)")
    ap.add_argument("--workload", choices=["single", "batch", "learned", "kernels", "precision",
                                           "sizes"],
                    default="single",
                    help="single: the M=65536 DP5 instance (default); batch: the 256-instance "
                         "sweep; learned: train the step proposer, then learned vs PI at "
                         "M=262144; kernels: --steps launches of each RHS kernel plus a 64 MiB "
                         "device copy (for hardware-counter runs); precision: the float-float "
                         "convolutions against the oracle's trajectory windows and FP64 to t=1e3; "
                         "sizes: the right-hand side and the stage kernels at M = 2^12..2^19")
    ap.add_argument("--no-accuracy-check", action="store_true",
                    help="skip the tight reference run that selects rtol (profiling)")
    ap.add_argument("--train-instances", type=int, default=512)
    ap.add_argument("--train-t-end", type=float, default=1e3)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--err-target", type=float, default=None,
                    help="learned workload: error norm the hindsight training targets aim at "
                         "(default: the median accepted norm of the PI training runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); multi-GPU "
              "sharding is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2407_16559_amd as smol
    import workloads as W

    dev = torch.device("cuda:0")
    if args.workload == "batch":
        return bench_batch(args, smol, W, torch, dev)
    if args.workload == "learned":
        return bench_learned(args, smol, W, torch, dev)
    if args.workload == "kernels":
        return bench_kernels(args, smol, W, torch, dev)
    if args.workload == "precision":
        return bench_precision(args, smol, W, torch, dev)
    if args.workload == "sizes":
        return bench_sizes(args, smol, W, torch, dev)
    c = W.WORKLOADS["single-large"]
    t_end = args.t_end if args.t_end else c["t_end"]
    U, V, lam, n0 = W.workload_instance("single-large")
    M, R = U.shape[1], U.shape[0]
    Ud = torch.from_numpy(U).to(dev)
    Vd = torch.from_numpy(V).to(dev)
    n0d = torch.from_numpy(n0).to(dev)
    out = torch.empty_like(n0d)

    def run(rtol=None, atol=None):
        return smol.integrate(Ud, Vd, lam, n0d, t_end, rtol or c["rtol"], atol or c["atol"],
                              method="dp5", out=out, raise_on_error=True)

    # time-to-t_end "at 1e-6 relative error": the loosest rtol in
    # 1e-6, 3e-7, 1e-7, ... whose end state is within 1e-6 (max-norm,
    # relative) of a tight run (rtol 1e-10, atol 1e-16); untimed
    rtol, err_tight = c["rtol"], None
    if not args.no_accuracy_check:
        ref = run(1e-10, 1e-16)[0].clone()
        for rtol in (1e-6, 3e-7, 1e-7, 3e-8, 1e-8):
            got = run(rtol)[0]
            err_tight = ((got - ref).abs().max() / ref.abs().max()).item()
            if err_tight <= 1e-6:
                break
        print(f"bench: rtol {rtol:g}, error vs tight run {err_tight:.2e}", file=sys.stderr,
              flush=True)
    c = dict(c, rtol=rtol)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(run()[1])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_acc = sum(s["n_accept"] for s in stats)
    n_rhs = sum(s["n_rhs"] for s in stats)

    # live per-kernel timing (HIP events on the stream the kernels run on) of
    # the integrator's stage kernels at the run's final state; the dominant
    # kernel is the one with the largest share of an attempt
    L = fft_length(M)
    prof = smol.profile_step(Ud, Vd, lam, out.clone(), method="dp5", iters=200)
    nbytes = step_bytes(M, R, L)
    dom = max(STEP_LAUNCHES, key=lambda k: prof[k] * STEP_LAUNCHES[k])
    achieved = nbytes[dom] / (prof[dom] * 1e-3)
    attempt_ms = sum(prof[k] * STEP_LAUNCHES[k] for k in STEP_LAUNCHES)
    rhs = smol.profile_rhs(Ud, Vd, lam, out.clone(), iters=200)
    rb = rhs_bytes(M, R, L)
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": recorded_traffic(dom),
            "alg_bytes": nbytes[dom],
            "ms_per_launch": prof,
            "launches_per_attempt": STEP_LAUNCHES,
            "stage_kernels_ms_per_attempt": attempt_ms,
            "share_of_stage_kernels": prof[dom] * STEP_LAUNCHES[dom] / attempt_ms,
            "standalone_rhs": {"ms_per_launch": rhs, "alg_bytes": rb,
                               "frac": rb["rhs"] / (rhs["rhs"] * 1e-3) / HBM_PEAK,
                               "min_bytes": min_bytes(M, R),
                               "frac_min_bytes": min_bytes(M, R) / (rhs["rhs"] * 1e-3) / HBM_PEAK}}

    line = {
        "metric": "accepted RK steps/s (time-to-t_end at rtol 1e-6), M=2^16 R=3",
        "value": n_acc / elapsed,
        "unit": "accepted steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single-large-oscillatory: M=65536, R=3 kernel (i/j)^a+(j/i)^a+2, "
                               f"a=0.45, lam=0.005, monodisperse start, DP5(4) PI, "
                               f"rtol={c['rtol']:g}, atol=1e-12, t_end={t_end:g}",
                   "M": M, "R": R, "fft_length": L, "parallelism": "1 GPU"},
        "time_to_t_end_s": elapsed / args.steps,
        "rtol": c["rtol"],
        "rel_err_vs_tight_run": err_tight,
        "accepted_steps_per_run": stats[-1]["n_accept"],
        "rejected_steps_per_run": stats[-1]["n_reject"],
        "rhs_evals_per_s": n_rhs / elapsed,
        "roofline": roof,
    }
    roof["copy_same_footprint"] = copy_ceiling(torch, dev, nbytes[dom])
    roof["copy_rhs_footprint"] = copy_ceiling(torch, dev, rb["rhs"])
    # the kernel's rate against a plain copy that moves the same bytes in one launch
    roof["frac_of_copy"] = roof["frac"] / roof["copy_same_footprint"]["frac"]
    line["rhs_precision"] = rhs_precision_times(smol, torch, Ud, Vd, lam, out.clone())
    # the transform's round-off leaves tiny negative values in the tail; not clamped
    line["min_n_at_t_end"] = float(out.min().item())
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(U, V, lam, n0, 6, stats[-1]["n_rhs"])
        line["plain_small"] = plain_small(smol, W, torch, dev)
    print(json.dumps(line), flush=True)


def rhs_precision_times(smol, torch, U, V, lam, n, iters=200):
    """Mean time of one whole right-hand side (three kernels, launched by
    smol_rhs on torch's current stream, timed with events there) in FP64 and
    in float-float, at the same state."""
    res = {}
    for prec in ("fp64", "fp32x2"):
        out = torch.empty_like(n)
        for _ in range(5):
            smol.rhs(U, V, lam, n, out=out, precision=prec)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(iters):
            smol.rhs(U, V, lam, n, out=out, precision=prec)
        b.record()
        b.synchronize()
        res[prec] = {"ms_per_rhs": a.elapsed_time(b) / iters}
    res["fp32x2_over_fp64"] = res["fp32x2"]["ms_per_rhs"] / res["fp64"]["ms_per_rhs"]
    return res


def bench_batch(args, smol, W, torch, dev):
    """Batched sweep: 256 seeded instances (M log-uniform in [2^12, 2^17],
    a in [0.05, 0.5], lam log-uniform in [1e-3, 1e-1], exponential starts),
    BS3, rtol 1e-6, atol 1e-12, t_end 1e3, in one batched run per bench step;
    compared with one-by-one single-instance runs of every 16th instance,
    extrapolated to all 256."""
    c = W.WORKLOADS["batched-sweep"]
    t_end = args.t_end if args.t_end else c["t_end"]
    draws = W.batch_draws(c["n_inst"], seed=c["seed"])
    insts = []
    for d in draws:
        U, V, lam, n0 = W.batch_instance(d)
        insts.append(dict(U=torch.from_numpy(U).to(dev), V=torch.from_numpy(V).to(dev), lam=lam,
                          n0=torch.from_numpy(n0).to(dev), t_end=t_end, rtol=c["rtol"],
                          atol=c["atol"]))
    for _ in range(args.warmup):
        smol.integrate_batch(insts, method="bs3")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs, stats = smol.integrate_batch(insts, method="bs3")
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    n_acc = sum(s["n_accept"] for s in stats)
    n_rhs = sum(s["n_rhs"] for s in stats)
    # the algorithmic bytes of every instance's right-hand sides (FP64
    # three-kernel figure at its own M and transform length), per second of
    # the batched run: how close the batch as a whole comes to HBM peak
    alg = 0
    for d, st in zip(insts, stats):
        Mi, Ri = d["U"].shape[1], d["U"].shape[0]
        Li = fft_length(Mi)
        alg += st["n_rhs"] * rhs_bytes(Mi, Ri, Li)["rhs"]
    t0 = time.perf_counter()
    sample = list(range(0, len(insts), 16))
    for i in sample:
        d = insts[i]
        smol.integrate(d["U"], d["V"], d["lam"], d["n0"], t_end, d["rtol"], d["atol"],
                       method="bs3", raise_on_error=True)
    torch.cuda.synchronize()
    single = (time.perf_counter() - t0) * len(insts) / len(sample)
    line = {
        "metric": "accepted RK steps/s over all instances (batched sweep)",
        "value": n_acc / elapsed,
        "unit": "accepted steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched-sweep: 256 instances, M log-uniform 2^12..2^17, BS3(2) PI, "
                               f"rtol=1e-6, atol=1e-12, t_end={t_end:g}", "parallelism": "1 GPU"},
        "batch_time_s": elapsed,
        "single_instance_runs_extrapolated_s": single,
        "speedup_vs_single_runs": single / elapsed,
        "accepted_steps_total": n_acc,
        "rhs_evals_per_s": n_rhs / elapsed,
        "rhs_alg_GBps": alg / elapsed / 1e9,
        "rhs_alg_frac_of_hbm_peak": alg / elapsed / HBM_PEAK,
        "max_accepted_steps_one_instance": max(s["n_accept"] for s in stats),
        "all_ok": all(s["status"] == 0 for s in stats),
    }
    print(json.dumps(line), flush=True)


def bench_kernels(args, smol, W, torch, dev):
    """The three right-hand-side kernels of the large instance (M = 65536,
    at its start state), --steps launches of each and --steps whole RHS,
    --steps launches of each of the integrator's DP5(4) stage kernels at the
    same state, then --steps copies of a 64 MiB device buffer: the reference a hardware
    byte counter is scaled by (each copy reads and writes 64 MiB)."""
    import numpy as np
    U, V, lam, n0 = W.workload_instance("single-large")
    M, R = U.shape[1], U.shape[0]
    L = fft_length(M)
    Ud, Vd, nd = (torch.from_numpy(x).to(dev) for x in (U, V, W.exponential_start(M, 300.0)))
    prof = smol.profile_rhs(Ud, Vd, lam, nd, iters=args.steps)
    prof_step = smol.profile_step(Ud, Vd, lam, nd, method="dp5", iters=args.steps)
    # the same right-hand side in float-float (the k_phase* kernels over cff)
    ff = rhs_precision_times(smol, torch, Ud, Vd, lam, nd, iters=args.steps)
    ceil = {k: copy_ceiling(torch, dev, b, iters=args.steps)
            for k, b in (("int_c_fused", step_bytes(M, R, L)["int_c_fused"]),
                         ("rhs", rhs_bytes(M, R, L)["rhs"]))}
    nbytes = 64 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "kernels", "M": M, "R": R, "fft_length": L,
                      "launches": args.steps, "ms_per_launch": dict(prof, **prof_step),
                      "alg_bytes": dict(rhs_bytes(M, R, L), **step_bytes(M, R, L)),
                      "rhs_evals_per_s": 1e3 / prof["rhs"],
                      "rhs_precision": ff,
                      "copy_same_footprint": ceil,
                      "copy_bytes_each_way": nbytes}),
          flush=True)


def bench_sizes(args, smol, W, torch, dev):
    """The hot path against the size: for M = 2^12 .. 2^19 (transform
    lengths 2^13 .. 2^20; the single-large kernel, rank 3, a = 0.45,
    lam = 0.005, at an exponential state), the standalone right-hand side
    and the integrator's DP5 stage kernels timed live (200 launches each),
    their fraction of HBM peak on the algorithmic bytes, a plain copy of the
    right-hand side's bytes as the ceiling at that footprint, and DP5 step
    attempts per second (a run of 400 attempts from the monodisperse start)."""
    import numpy as np
    c = W.WORKLOADS["single-large"]
    rows = []
    for logM in range(12, 20):
        M = 1 << logM
        L = fft_length(M)
        U, V = W.brownian_rank3(M, c["a"])
        Ud, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev)
        nd = torch.from_numpy(W.exponential_start(M, M / 200.0)).to(dev)
        rhs = smol.profile_rhs(Ud, Vd, c["lam"], nd, iters=200)
        step = smol.profile_step(Ud, Vd, c["lam"], nd, method="dp5", iters=200)
        rb, sb = rhs_bytes(M, 3, L), step_bytes(M, 3, L)
        n0 = torch.from_numpy(W.monodisperse(M)).to(dev)
        smol.integrate(Ud, Vd, c["lam"], n0, 1e9, 1e-6, 1e-12, method="dp5", max_steps=16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = smol.integrate(Ud, Vd, c["lam"], n0, 1e9, 1e-6, 1e-12, method="dp5",
                               max_steps=400)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        attempts = st["n_accept"] + st["n_reject"]
        row = {"M": M, "fft_length": L,
               "rhs_ms": rhs["rhs"], "rhs_frac": rb["rhs"] / (rhs["rhs"] * 1e-3) / HBM_PEAK,
               "rhs_evals_per_s": 1e3 / rhs["rhs"],
               "copy_rhs_footprint_frac": copy_ceiling(torch, dev, rb["rhs"])["frac"],
               "int_c_fused_ms": step["int_c_fused"],
               "int_c_fused_frac": sb["int_c_fused"] / (step["int_c_fused"] * 1e-3) / HBM_PEAK,
               "stage_kernels_ms_per_attempt": sum(step[k] * STEP_LAUNCHES[k]
                                                   for k in STEP_LAUNCHES),
               "attempts_per_s": attempts / dt, "ms_per_attempt": 1e3 * dt / attempts}
        print(f"bench: sizes M=2^{logM}: {row}", file=sys.stderr, flush=True)
        rows.append(row)
        del Ud, Vd, nd, n0
        smol.release_plans()
    print(json.dumps({"workload": "sizes", "kernel": "rank-3 (i/j)^a+(j/i)^a+2, a=0.45, "
                      "lam=0.005", "rows": rows}), flush=True)


def bench_precision(args, smol, W, torch, dev):
    """The precision workload: the single-large instance (rank 3, a = 0.45,
    lam = 0.005) and the rank-4 product kernel (a = 0.3, lam = 0.02), both at
    M = 65536 from the monodisperse start with DP5(4), rtol 1e-6, atol 1e-12.
    (1) The first 16 attempts in FP64 and in float-float against the oracle's
    FP64 windows stored under tests/golden (written by
    tests/golden/make_oracle_windows.py from the oracle alone); (2) whole runs
    to t = 1e3 in both precisions, timed, with their max-norm relative
    difference (the oracle's whole trajectory, about 10^4 direct
    right-hand sides, is out of reach of a host)."""
    import numpy as np
    golden = os.path.join(ROOT, "tests", "golden")
    c = W.WORKLOADS["single-large"]
    p = W.WORKLOADS["precision"]
    cases = {"rank3": (W.brownian_rank3(c["M"], c["a"]), c["lam"], c["t_end"],
                       "single_large_dp5_w16.npz"),
             "rank4": (W.product_rank4(p["M"], p["a"]), p["lam"], p["t_eval"],
                       "precision_rank4_dp5_w16.npz")}
    res = {}
    for name, ((U, V), lam, t_w, fixture) in cases.items():
        Ud, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev)
        n0 = torch.from_numpy(W.monodisperse(U.shape[1])).to(dev)
        ref = np.load(os.path.join(golden, fixture))
        r = {}
        for prec in ("fp64", "fp32x2"):
            out, st = smol.integrate(Ud, Vd, lam, n0, t_w, 1e-6, 1e-12, method="dp5",
                                     precision=prec, max_steps=16)
            r["window_rel_err_vs_oracle_" + prec] = float(
                np.abs(out.cpu().numpy() - ref["n"]).max() / np.abs(ref["n"]).max())
        outs = {}
        for prec in ("fp64", "fp32x2"):
            smol.integrate(Ud, Vd, lam, n0, 1.0, 1e-6, 1e-12, method="dp5", precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out, st = smol.integrate(Ud, Vd, lam, n0, p["t_eval"], 1e-6, 1e-12, method="dp5",
                                     precision=prec, raise_on_error=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            outs[prec] = out
            r[prec] = {"time_to_t_s": dt, "n_accept": st["n_accept"], "n_reject": st["n_reject"],
                       "rhs_evals_per_s": st["n_rhs"] / dt}
        r["rel_diff_fp32x2_vs_fp64_at_t"] = ((outs["fp32x2"] - outs["fp64"]).abs().max()
                                            / outs["fp64"].abs().max()).item()
        res[name] = r
        print(f"bench: precision {name}: {r}", file=sys.stderr, flush=True)
    line = {"metric": "float-float convolutions: max relative error vs the FP64 oracle "
                      "(16-attempt windows) and vs FP64 at t=1e3",
            "value": max(res[k]["rel_diff_fp32x2_vs_fp64_at_t"] for k in res),
            "unit": "relative error", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1e3 * res["rank3"]["fp32x2"]["time_to_t_s"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 state, fp32x2 convolutions", "data": "synthetic",
            "config": {"workload": "precision: M=65536 rank-3 a=0.45 lam=0.005 and rank-4 "
                                   "a=0.3 lam=0.02, monodisperse, DP5(4), rtol=1e-6, "
                                   "atol=1e-12, t=1e3", "parallelism": "1 GPU"},
            "cases": res}
    print(json.dumps(line), flush=True)


def bench_learned(args, smol, W, torch, dev):
    """Learned step proposer against PI on the large instance (M = 262144,
    a = 0.4, lam = 0.01, monodisperse start, DP5(4), rtol 1e-6, t_end 1e4).

    Training data: per-attempt logs of PI runs (DP5, rtol 1e-6, to the batched
    sweep's t_end = 1e3) on 512 instances drawn from the batched sweep's
    distribution (seed 1), run in batches of 128; hindsight targets for the error norm the PI runs accept
    at (their median accepted norm, unless --err-target is given);
    weighted-MSE training with Adam (lr 1e-3, overshoot weight 4) from
    seed-12345 initial weights, all in the library's kernels.  Then one run
    with each controller, timed, and both compared with a tight run
    (rtol 1e-10, atol 1e-16)."""
    import numpy as np
    c = W.WORKLOADS["learned-proposer"]
    t_end = args.t_end if args.t_end else c["t_end"]
    t_train_end = args.train_t_end
    cap = 40000
    draws = W.batch_draws(args.train_instances, seed=1)
    logs_all = []
    t_runs = 0.0
    for lo in range(0, len(draws), 128):
        insts, logs = [], []
        for d in draws[lo:lo + 128]:
            U, V, lam, n0 = W.batch_instance(d)
            log = torch.zeros((cap, 9), dtype=torch.float64, device=dev)
            insts.append(dict(U=torch.from_numpy(U).to(dev), V=torch.from_numpy(V).to(dev),
                              lam=lam, n0=torch.from_numpy(n0).to(dev), t_end=t_train_end,
                              rtol=c["rtol"], atol=c["atol"], log=log))
            logs.append(log)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, stats = smol.integrate_batch(insts, method="dp5")
        torch.cuda.synchronize()
        t_runs += time.perf_counter() - t0
        for log, st in zip(logs, stats):
            logs_all.append((log, min(cap, st["n_accept"] + st["n_reject"])))
        print(f"bench: training runs {lo + len(insts)}/{len(draws)} ({t_runs:.1f} s)",
              file=sys.stderr, flush=True)
        del insts
    err_target = args.err_target
    if err_target is None:
        acc = torch.cat([lg[:n][lg[:n, 3] == 1.0, 2] for lg, n in logs_all])
        err_target = float(acc.median().item())
    Xs, Ts = [], []
    for log, n in logs_all:
        X, tg = smol.proposer_dataset(log, n, "dp5", err_target)
        Xs.append(X)
        Ts.append(tg)
    del logs_all
    X = torch.cat(Xs).contiguous()
    tg = torch.cat(Ts).contiguous()
    params = torch.from_numpy(W.mlp_init(12345).astype(np.float32)).to(dev)
    t0 = time.perf_counter()
    loss = smol.proposer_train(X, tg, params, epochs=args.epochs, batch=1024, lr=1e-3,
                               over_weight=4.0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"bench: trained on {X.shape[0]} rows in {t_train:.1f} s, loss "
          f"{loss[0].item():.4f} -> {loss[-1].item():.4f}", file=sys.stderr, flush=True)
    smol.proposer_set(params)

    U, V = W.brownian_rank3(c["M"], c["a"])
    Ud, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev)
    n0d = torch.from_numpy(W.monodisperse(c["M"])).to(dev)
    ref, _ = smol.integrate(Ud, Vd, c["lam"], n0d, t_end, 1e-10, 1e-16, method="dp5",
                            raise_on_error=True)
    res = {}
    for ctrl in ("pi", "learned"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, st = smol.integrate(Ud, Vd, c["lam"], n0d, t_end, c["rtol"], c["atol"],
                                 method="dp5", controller=ctrl, raise_on_error=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = ((out - ref).abs().max() / ref.abs().max()).item()
        res[ctrl] = {"time_to_t_end_s": dt, "n_accept": st["n_accept"],
                     "rhs_evals_per_s": st["n_rhs"] / dt,
                     "n_reject": st["n_reject"], "n_rhs": st["n_rhs"],
                     "reject_rate": st["n_reject"] / max(1, st["n_accept"] + st["n_reject"]),
                     "n_fallback": st["n_fallback"], "rel_err_vs_tight_run": err}
        print(f"bench: {ctrl}: {res[ctrl]}", file=sys.stderr, flush=True)
    sweep = bench_sweep_learned(args, smol, W, torch, dev)
    line = {
        "metric": "time-to-t_end with the learned step proposer, M=2^18 R=3",
        "value": res["learned"]["time_to_t_end_s"],
        "unit": "s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * res["learned"]["time_to_t_end_s"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (network f32)", "data": "synthetic",
        "config": {"workload": f"learned-proposer: M=262144, R=3, a=0.4, lam=0.01, monodisperse, "
                               f"DP5(4), rtol=1e-6, atol=1e-12, t_end={t_end:g}; trained on "
                               f"{len(draws)} sweep-distributed runs to t={t_train_end:g}, "
                               f"error target {err_target:.3g}", "parallelism": "1 GPU"},
        "learned": res["learned"], "pi": res["pi"],
        "speedup_vs_pi": res["pi"]["time_to_t_end_s"] / res["learned"]["time_to_t_end_s"],
        "rhs_ratio_vs_pi": res["learned"]["n_rhs"] / res["pi"]["n_rhs"],
        "training": {"runs_s": t_runs, "rows": int(X.shape[0]), "epochs": args.epochs,
                     "err_target": err_target, "instances": len(draws), "t_end": t_train_end,
                     "train_s": t_train, "loss_first": loss[0].item(),
                     "loss_last": loss[-1].item()},
        "batched_sweep": sweep,
    }
    print(json.dumps(line), flush=True)


def bench_sweep_learned(args, smol, W, torch, dev):
    """The batched form with the trained proposer against the plain
    single-instance PI solver, each at its time-to-t_end at 1e-6 relative
    error: the 256 sweep instances of the batched workload (seed 0, held out
    from the training seed), DP5(4) (the pair the proposer was trained on),
    atol 1e-12, t = 0 -> 1e3.  For each form the loosest rtol in 1e-6, 3e-7,
    1e-7, 3e-8 whose end states on every 32nd instance are within 1e-6
    (max-norm relative) of tight single runs (rtol 1e-10, atol 1e-16) is
    taken, as for the single-large workload.  Batched runs are timed whole;
    single-instance PI runs on the sampled instances, extrapolated to all 256
    (a batched instance equals its single run bitwise, so both PI forms meet
    the bar at the same rtol)."""
    c = W.WORKLOADS["batched-sweep"]
    t_end = c["t_end"]
    draws = W.batch_draws(c["n_inst"], seed=c["seed"])
    insts = []
    for d in draws:
        U, V, lam, n0 = W.batch_instance(d)
        insts.append(dict(U=torch.from_numpy(U).to(dev), V=torch.from_numpy(V).to(dev), lam=lam,
                          n0=torch.from_numpy(n0).to(dev), t_end=t_end, rtol=c["rtol"],
                          atol=c["atol"]))
    sample = list(range(0, len(insts), 32))
    refs = {}
    for i in sample:
        d = insts[i]
        refs[i], _ = smol.integrate(d["U"], d["V"], d["lam"], d["n0"], t_end, 1e-10, 1e-16,
                                    method="dp5", raise_on_error=True)

    def err_on_sample(outs):
        return max(((outs[i] - refs[i]).abs().max() / refs[i].abs().max()).item() for i in sample)

    res = {}
    for ctrl in ("pi", "learned"):
        for rtol in (1e-6, 3e-7, 1e-7, 3e-8):
            run = [dict(d, rtol=rtol) for d in insts]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o, stats = smol.integrate_batch(run, method="dp5", controller=ctrl)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            e = err_on_sample(o)
            res["batched_" + ctrl] = {
                "rtol": rtol, "time_s": dt, "max_rel_err_vs_tight_on_sample": e,
                "n_rhs": sum(st["n_rhs"] for st in stats),
                "n_reject": sum(st["n_reject"] for st in stats),
                "rhs_evals_per_s": sum(st["n_rhs"] for st in stats) / dt,
                "all_ok": all(st["status"] == 0 for st in stats)}
            print(f"bench: sweep batched {ctrl} rtol {rtol:g}: {res['batched_' + ctrl]}",
                  file=sys.stderr, flush=True)
            if e <= 1e-6:
                break
    rtol_pi = res["batched_pi"]["rtol"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in sample:
        d = insts[i]
        smol.integrate(d["U"], d["V"], d["lam"], d["n0"], t_end, rtol_pi, d["atol"],
                       method="dp5", raise_on_error=True)
    torch.cuda.synchronize()
    res["single_pi"] = {"rtol": rtol_pi,
                        "time_s_extrapolated": (time.perf_counter() - t0) * len(insts) / len(sample)}
    res["speedup_batched_learned_vs_single_pi"] = (res["single_pi"]["time_s_extrapolated"]
                                                  / res["batched_learned"]["time_s"])
    res["speedup_batched_pi_vs_single_pi"] = (res["single_pi"]["time_s_extrapolated"]
                                             / res["batched_pi"]["time_s"])
    print(f"bench: batched sweep: {res}", file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
