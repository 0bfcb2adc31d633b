#!/usr/bin/env python
"""Throughput of QAOA expectation + adjoint gradient on one MI355X.

Workload: 0-1 QUBO on n = 32 variables with an Erdos-Renyi(0.1) coupling
pattern, J_ij ~ N(0,1), h_i ~ N(0,1) (seed 2), depth p = 3, angles = linear
ramp + N(0, 0.05) noise; complex128 state (64 GiB) + adjoint vector (64 GiB)
+ fp64 cost diagonal (32 GiB), all resident in HBM.  One step = one call of
qaoa_gradient: E and all 2p partial derivatives.

Prints one JSON line.  Besides the headline throughput it reports the
roofline of the dominant kernel (HIP events bracketing every pass launch on the
library's stream, divided into the pass's algorithmic bytes) and the CPU
oracle's throughput on a bounded sample of the same workload.  Under "extra":
the complex64 variant, 10^6-shot sampling, the batched engine on 4096 graphs of
n ~ U{10..20} (p = 4, 100 Adam steps each, one persistent launch), and the
time-to-ratio of learned versus linear-ramp starts on held-out ER(24, 0.5)
graphs (p = 8, a sample of the evaluation set).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grad evals/s + HBM GB/s at n=32 p=3; time-to-ratio learned vs plain init"
HBM_PEAK_GBS = 8000.0


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_pass_traffic_qubo32_p3_c128.md")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2407_13012_amd", "csrc", f)
                   for f in ("kernels.hip", "passes.hip", "tile_device.h", "plan.cpp", "api.cpp", "qaoa_internal.h")]


# template instance that runs each pass kind (passes.hip; one instance per
# spectator class S of the pass, S = 0 for a layer's first group)
KERNEL_OF = {"forward": "k_pass<{}, kFwd, S>", "turn": "k_pass<{}, kTurn, S>", "backward": "k_pass<{}, kBwd, S>",
             "boundary_forward": "k_pass_fuse<{}, kFwdFuse, S>", "boundary_backward": "k_pass_fuse<{}, kBwdFuse, S>"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kind: str):
    """HBM bytes per launch of one pass kind from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on different kernel sources."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256") != kernel_source_hash():
        return None
    try:
        return float(vals[f"{kind} HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def model_bytes_per_amp(n: int, p: int, s: int, c: int) -> float:
    """Per-amplitude bytes of one E+G under the pass model p(6 P s + 2 c) + c - 2 s
    with P = ceil(n / kmax) passes per mixer layer (kmax = 13 for 16-byte
    amplitudes, 14 for 8-byte ones)."""
    kmax = 13 if s == 16 else 14
    P = math.ceil(n / kmax)
    return p * (6 * P * s + 2 * c) + c - 2 * s


def time_gradients(q, gamma, beta, steps, warmup):
    import torch
    for _ in range(warmup):
        q.gradient(gamma, beta)
    torch.cuda.synchronize()
    q.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        q.gradient(gamma, beta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = q.profile_read()
    q.profile_enable(False)
    return t1 - t0, prof


def copy_ceiling(gib: float) -> float:
    """Practical HBM ceiling: GB/s (bytes read + written) of a plain device copy,
    the faster of torch's copy (a DMA-style blit) and an elementwise x * 1 kernel."""
    import torch
    nel = int(gib * (1 << 30)) // 8
    x = torch.empty(nel, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    best = 0.0
    for op in (lambda: y.copy_(x), lambda: torch.mul(x, 1.0, out=y)):
        op()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            op()
        torch.cuda.synchronize()
        best = max(best, 2 * nel * 8 / ((time.perf_counter() - t0) / 3) / 1e9)
    del x, y
    torch.cuda.empty_cache()
    return best


def small_workloads() -> dict:
    """The two smaller configurations: E+G latency of the n=12, p=2 MaxCut and
    E+G time of the n=26 3-regular weighted MaxCut (p=6) in both precisions,
    the latter against its byte model (P_min = 2)."""
    import torch

    import qaoa_inputs as qi
    from paper_2407_13012_amd import QaoaHandle
    out = {}
    w = qi.workload_small()
    with QaoaHandle.from_instance(w["instance"]) as q:
        for _ in range(5):
            q.gradient(w["gamma"], w["beta"])
        t0 = time.perf_counter()
        for _ in range(100):
            q.gradient(w["gamma"], w["beta"])
        out["maxcut12_p2_grad_us"] = (time.perf_counter() - t0) / 100 * 1e6
    w = qi.workload_regular26()
    for prec, s, c in (("c128", 16, 8), ("c64", 8, 4)):
        with QaoaHandle.from_instance(w["instance"], prec) as q:
            q.gradient(w["gamma"], w["beta"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                q.gradient(w["gamma"], w["beta"])
            dt = (time.perf_counter() - t0) / 10
        out[f"regular26_p6_{prec}_grad_ms"] = dt * 1e3
        out[f"regular26_p6_{prec}_model_roofline_frac"] = (model_bytes_per_amp(26, 6, s, c) * 2.0 ** 26 / dt
                                                           / (HBM_PEAK_GBS * 1e9))
    return out


def batch_bytes_per_amp(n: int, p: int, kmax: int = 10) -> float:
    """Algorithmic bytes per amplitude of one batched-engine E+G (complex128, fp64 C).
    With P mixer sweeps per layer the engine runs, forward, an init + phase sweep
    (s + c), plain sweeps (2s) and, for P >= 2, p - 1 layer-boundary sweeps
    (2s + c; for P = 1 every later layer's sweep applies its phase: 2s + c), up
    to the last group; the turn sweep (last group, E, lam = C phi: 2s + c, only c
    when it is the whole evolution); backward the mirror image (plain 4s,
    boundary or phase sweeps 4s + c, the last one storing nothing: 2s + c)."""
    s, c = 16, 8
    if n <= 12:  # one sweep per layer
        if p == 1:
            return float(c)
        return (s + c) + (p - 2) * (2 * s + c) + (2 * s + c) + (p - 2) * (4 * s + c) + (2 * s + c)
    P = 1 + -(-(n - 12) // kmax)
    sweeps = P + (p - 1) * (P - 1)            # forward sweeps, the turn included
    plain = sweeps - 2 - (p - 1)
    fwd = (s + c) + (p - 1) * (2 * s + c) + plain * 2 * s
    bwd = (p - 1) * (4 * s + c) + (2 * s + c) + plain * 4 * s
    return fwd + (2 * s + c) + bwd


def batch_leg(count: int, p: int, steps: int, log) -> dict:
    """The batched engine on the n ~ U{10..20} MaxCut family: `count` graphs,
    depth p, `steps` Adam steps each, all in one persistent launch."""
    import numpy as np
    import torch

    import qaoa_inputs as qi
    from paper_2407_13012_amd import QaoaBatch
    from paper_2407_13012_amd import batch_tune as bt

    graphs = qi.batched_family(count)
    t0 = time.perf_counter()
    choice = bt.tune(graphs, p, log=log)
    t_tune = time.perf_counter() - t0
    opts = bt.options_of(choice)
    g0, b0 = bt.ramp_angles(count, p)
    with QaoaBatch(graphs, p, steps=steps, **opts) as b:
        b.run(g0, b0)  # warm-up: first graph launch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gam, bet, e0, e1 = b.run(g0, b0)
        dt = time.perf_counter() - t0
        t_start, t_end, which = b.timeline()
    ns = np.array([g.n for g in graphs])
    kmax = {int(k): int(v) for k, v in choice["group_by_n"].items()}
    amps = float(np.sum(2.0 ** ns))
    res_n = opts["resident_max_n"]
    # LDS-resident instances move only their cost entries through memory
    algo = sum((8.0 * (2 * p - 1) if n <= res_n else batch_bytes_per_amp(int(n), p, kmax.get(int(n), 10)))
               * 2.0 ** n for n in ns) * steps
    evals = count * steps
    log(f"[bench] batch {count} graphs x {steps} steps: {dt:.2f} s ({evals / dt:.0f} E+G/s)")
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    launches = {}
    for k, name in ((0, "streamed"), (1, "resident")):
        sel = which == k
        if not np.any(sel):
            continue
        grid = min(opts["workgroups"], int(sel.sum())) if k == 0 else min(cus, opts["workgroups"], int(sel.sum()))
        span = float(t_end[sel].max() - t_start[sel].min())
        busy = float(np.sum(t_end[sel] - t_start[sel]))
        launches[name] = {"instances": int(sel.sum()), "workgroups": grid, "span_s": span,
                          "busy_fraction": busy / (grid * span) if span > 0 else None,
                          "first_start_s": float(t_start[sel].min())}
    big = ns == ns.max()
    launches["largest_n"] = {"n": int(ns.max()), "mean_s": float(np.mean(t_end[big] - t_start[big])),
                             "last_end_s": float(t_end[big].max())}
    return {
        "graphs": count, "p": p, "adam_steps": steps, "seconds": dt,
        "grad_evals_per_s": evals / dt,
        "amplitude_layer_updates_per_s": amps * 2 * p * steps / dt,
        "algorithmic_GBps": algo / dt / 1e9,
        "mean_E_gain": float(np.mean(e1 - e0)),
        "improved_fraction": float(np.mean(e1 > e0)),
        "tuned": {k: choice[k] for k in ("group_by_n", "waves_per_simd", "workgroups", "resident_max_n")},
        "tune_s": t_tune,
        "timeline": launches,
    }


WARMSTART_PARAMS = os.path.join(ROOT, "paper_2407_13012_amd", "tuning", "mpnn_p8.npy")


def warmstart_leg(count: int, log) -> dict:
    """Time-to-ratio of learned vs plain starts: L-BFGS (one qaoa_gradient per
    evaluation) from the linear ramp and from the trained network's angles on
    held-out ER(24, 0.5) graphs, p = 8; evaluations and wall time until the
    plain run's final approximation ratio minus 0.005 is reached (the plain run
    goes on to convergence, which sets that target; the learned run stops there)."""
    import numpy as np

    import qaoa_inputs as qi
    from paper_2407_13012_amd import warmstart as ws

    if not os.path.exists(WARMSTART_PARAMS):
        return {"skipped": "no trained parameters"}
    params = np.load(WARMSTART_PARAMS, allow_pickle=False)
    graphs = qi.warmstart_eval_graphs(count)
    res = ws.evaluate(params, graphs, 8, learned_until_target=True, log=log)
    res.pop("rows")
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_THREAD_SNIPPET = """
import sys, time
sys.path.insert(0, {root!r})
import oracle, qaoa_inputs as qi
w = qi.workload_qubo32({n})
inst = w["instance"]
C = oracle.cost_of(inst)
t0 = time.perf_counter()
oracle.gradient(inst.n, C, w["gamma"], w["beta"])
print(time.perf_counter() - t0, oracle.num_threads())
"""


def one_thread_oracle_seconds(n: int):
    """One oracle E+G of the n-variable member of the headline family in a child
    process restricted to one OpenMP thread: (seconds, threads used)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", _ONE_THREAD_SNIPPET.format(root=ROOT, n=n)],
                         env=env, capture_output=True, text=True, timeout=600, check=True)
    dt, thr = out.stdout.split()[-2:]
    return float(dt), int(thr)


def cpu_baseline(inst_fn, sample_n, full_n, gamma, beta, batch_sample: int = 64,
                 slope_n: int = 26, one_thread_n: int = 22):
    """The CPU oracle (OpenMP over the host's cores) on bounded samples of the
    workloads: the headline E+G at n = sample_n (and slope_n, to show the 2^n
    scaling the extrapolation assumes), scaled by 2^(full_n - sample_n); one
    thread at n = one_thread_n; the two smaller configurations in full; 64
    graphs of the batched family."""
    import numpy as np

    import oracle
    import qaoa_inputs as qi

    def timed(n):
        inst = inst_fn(n)["instance"]
        C = oracle.cost_of(inst)
        t0 = time.perf_counter()
        oracle.gradient(n, C, gamma, beta)
        return time.perf_counter() - t0

    dt = timed(sample_n)
    scale = 2.0 ** (full_n - sample_n)
    out = {
        "value": 1.0 / (dt * scale),
        "unit": "grad_evals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"one oracle E+G ({dt:.2f} s) of the n={sample_n} member of the same QUBO family "
                   f"(p={len(gamma)}), scaled by 2^{full_n - sample_n} to n={full_n} (extrapolated)"),
        "cpu_model": cpu_model(),
        "logical_cpus_visible": len(os.sched_getaffinity(0)),
        f"qubo{sample_n}_grad_s": dt,
    }
    if slope_n and slope_n != sample_n:
        ds = timed(slope_n)
        out[f"qubo{slope_n}_grad_s"] = ds
        out["time_ratio_per_qubit"] = (dt / ds) ** (1.0 / (sample_n - slope_n))
    if one_thread_n:
        d1, thr = one_thread_oracle_seconds(one_thread_n)
        out["single_thread"] = {
            "value": 1.0 / (d1 * 2.0 ** (full_n - one_thread_n)), "unit": "grad_evals/s", "cores": thr,
            "sample": (f"one oracle E+G ({d1:.2f} s) at n={one_thread_n}, one OpenMP thread, "
                       f"scaled by 2^{full_n - one_thread_n} to n={full_n} (extrapolated)")}
    # the two smaller configurations, timed in full: MaxCut ER(12, 0.5) at p = 2 and the
    # n = 26 weighted 3-regular MaxCut at p = 6 (complex128)
    for key, wl in (("maxcut12_p2", qi.workload_small), ("regular26_p6", qi.workload_regular26)):
        w = wl()
        g = w["instance"]
        Cw = oracle.cost_of(g)
        reps = 20 if g.n <= 12 else 1
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.gradient(g.n, Cw, w["gamma"], w["beta"])
        out[key + "_grad_s"] = (time.perf_counter() - t0) / reps
    if batch_sample:
        # batched-engine workload: every 64th graph of the 4096-graph family, p = 4, one E+G each
        graphs = qi.batched_family(4096)[::4096 // batch_sample]
        g, b = qi.linear_ramp(4)
        t0 = time.perf_counter()
        for gr in graphs:
            oracle.gradient(gr.n, oracle.cost_of(gr), g, b)
        tb = time.perf_counter() - t0
        out["batch"] = {"value": len(graphs) / tb, "unit": "grad_evals/s",
                        "sample": f"one oracle E+G of each of {len(graphs)} evenly spaced graphs of the "
                                  f"n ~ U{{10..20}} family at p=4 ({tb:.2f} s)"}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--precision", default="c128", choices=["c128", "c64"])
    ap.add_argument("--cpu-sample-n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--warmstart-graphs", type=int, default=512)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="first run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X only: the simulator runs each instance on a single "
              "GPU and no multi-GPU path is built; run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import qaoa_inputs as qi
    from paper_2407_13012_amd import QaoaHandle

    torch.cuda.set_device(0)
    if args.copy_probe_gib > 0:
        nel = int(args.copy_probe_gib * (1 << 30)) // 8
        x = torch.empty(nel, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(f"[copy-probe] {nel * 8} bytes read, {nel * 8} bytes written", file=sys.stderr, flush=True)
        del x, y
        torch.cuda.empty_cache()

    copy_gbs = None
    if not args.no_extras:
        copy_gbs = copy_ceiling(8.0)
        print(f"[bench] device copy 8 GiB: {copy_gbs:.0f} GB/s (read + write)", file=sys.stderr, flush=True)

    w = qi.workload_qubo32(args.n)
    inst, gamma, beta = w["instance"], w["gamma"], w["beta"]
    p = len(gamma)
    s = 16 if args.precision == "c128" else 8
    c = 8 if args.precision == "c128" else 4
    print(f"[bench] n={args.n} p={p} m={inst.m} precision={args.precision}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    q = QaoaHandle.from_instance(inst, args.precision)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    dt, prof = time_gradients(q, gamma, beta, args.steps, args.warmup)
    ms_per_step = 1e3 * dt / args.steps
    value = args.steps / dt
    print(f"[bench] {args.steps} steps in {dt:.3f} s ({ms_per_step:.1f} ms/step)", file=sys.stderr, flush=True)

    kinds = {k: {"launches": v[0], "ms": v[1], "bytes": v[2],
                 "gbs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
             for k, v in prof.items() if v[0] > 0}
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    dk = kinds[dom]
    achieved = dk["gbs"]
    total_bytes = sum(v["bytes"] for v in kinds.values()) / args.steps
    kernel_ms = sum(v["ms"] for v in kinds.values()) / args.steps
    roofline = {
        "bound": "hbm",
        "kernel": KERNEL_OF[dom].format("double" if s == 16 else "float"),
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": recorded_traffic(dom) if (args.n == 32 and args.precision == "c128") else None,
        "bytes_per_launch": dk["bytes"] / max(dk["launches"], 1),
        "avg_launch_ms": dk["ms"] / max(dk["launches"], 1),
    }
    N = 2.0 ** args.n
    extra = {
        "passes": kinds,
        "algorithmic_bytes_per_step": total_bytes,
        "pass_time_ms_per_step": kernel_ms,
        "step_GBps": total_bytes / (ms_per_step * 1e-3) / 1e9,
        "model_bytes_per_amp": model_bytes_per_amp(args.n, p, s, c),
        "implemented_bytes_per_amp": total_bytes / N,
        "model_roofline_frac": model_bytes_per_amp(args.n, p, s, c) * N / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        # the same step against one sweep per layer (312 B/amp at c128): the ideal a single-pass mixer would need
        "ideal_p1_roofline_frac": (p * (6 * s + 2 * c) + c - 2 * s) * N / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "copy_GBps": copy_gbs,
        "create_s": t_create,
    }
    E, dg, db = q.gradient(gamma, beta)
    extra["E"] = E
    extra["grad_norm_inf"] = float(max(np.abs(dg).max(), np.abs(db).max()))

    if not args.no_extras:
        # cost diagonal rebuild time and 10^6-shot sampling on the same handle
        q.statevector(gamma, beta, copy=False)
        torch.cuda.synchronize()
        zt = torch.empty(w["shots"], dtype=torch.int64, device="cuda")
        ct = torch.empty(w["shots"], dtype=torch.float64, device="cuda")
        q.sample(w["shots"], w["sample_seed"], z_out=zt, cost_out=ct)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q.sample(w["shots"], w["sample_seed"], z_out=zt, cost_out=ct)
        torch.cuda.synchronize()
        extra["sample_1e6_ms"] = 1e3 * (time.perf_counter() - t0)
        t0 = time.perf_counter()
        E_ev = q.evaluate(gamma, beta)
        extra["evaluate_ms"] = 1e3 * (time.perf_counter() - t0)
        extra["evaluate_E"] = E_ev
    q.close()
    del q
    torch.cuda.empty_cache()

    if not args.no_extras and args.precision == "c128":
        q64 = QaoaHandle.from_instance(inst, "c64")
        dt64, prof64 = time_gradients(q64, gamma, beta, args.steps, 1)
        E64, _, _ = q64.gradient(gamma, beta)
        q64.close()
        mb64 = model_bytes_per_amp(args.n, p, 8, 4)
        extra["c64"] = {"grad_evals_per_s": args.steps / dt64, "ms_per_step": 1e3 * dt64 / args.steps,
                        "model_bytes_per_amp": mb64,
                        "model_roofline_frac": mb64 * 2.0 ** args.n / (dt64 / args.steps) / (HBM_PEAK_GBS * 1e9),
                        "E": E64, "E_rel_diff_vs_c128": abs(E64 - E) / max(abs(E), 1.0),
                        "passes": {k: {"launches": v[0], "ms": v[1], "bytes": v[2],
                                       "gbs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
                                   for k, v in prof64.items() if v[0] > 0}}
        print(f"[bench] c64 {extra['c64']['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)

    if not args.no_extras:
        extra.update(small_workloads())
        print(f"[bench] n=12 E+G {extra['maxcut12_p2_grad_us']:.0f} us; n=26 p=6 E+G "
              f"{extra['regular26_p6_c128_grad_ms']:.1f} ms (c128), {extra['regular26_p6_c64_grad_ms']:.1f} ms (c64)",
              file=sys.stderr, flush=True)

    if not args.no_batch:
        extra["batch"] = batch_leg(args.batch_graphs, 4, args.batch_steps,
                                   lambda m: print(m, file=sys.stderr, flush=True))

    if not args.no_warmstart:
        extra["warmstart"] = warmstart_leg(args.warmstart_graphs,
                                           lambda m: print(m, file=sys.stderr, flush=True))

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle at n={args.cpu_sample_n}", file=sys.stderr, flush=True)
        cpu = cpu_baseline(qi.workload_qubo32, args.cpu_sample_n, args.n, gamma, beta)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grad_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "c128" else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"QUBO n={args.n}, ER(0.1) couplings, J,h~N(0,1) seed 2, p={p}, "
                         f"{'complex128' if s == 16 else 'complex64'} expectation + adjoint gradient"),
            "n": args.n, "p": p, "terms": inst.m + args.n,
            "state_bytes": int(N * s), "precision": args.precision,
        },
        "roofline": roofline,
        # whole E+G: the bytes its passes actually move (each vector read or written once
        # per sweep, plus the cost reads) over the step time; the model-equivalent figure
        # prices the step at the pass model p(6 P s + 2c) + c - 2s per amplitude with
        # P = ceil(n / kmax) (kmax 13 for 16-byte amplitudes, 14 for 8-byte ones)
        "step_roofline": {"bound": "hbm",
                          "implemented_bytes_per_amp": extra["implemented_bytes_per_amp"],
                          "achieved": extra["step_GBps"],
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": extra["step_GBps"] / HBM_PEAK_GBS,
                          "model_bytes_per_amp": extra["model_bytes_per_amp"],
                          "model_equivalent_GBps": extra["model_bytes_per_amp"] * N / (ms_per_step * 1e-3) / 1e9,
                          "model_equivalent_frac": extra["model_roofline_frac"]},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
