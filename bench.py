#!/usr/bin/env python3
"""Benchmark of the restarted PDHG hot path on one MI355X.

Headline workload: the largest single-GPU LP, m=5M, n=20M, nnz=110M (5
nonzeros per column at random rows among the first m-50, plus 50 coupling
rows of 200k entries; values N(0,1); planted optimum), FP64, Ruiz 10 passes,
reflected Halpern iteration, target relative KKT 1e-8.  One step = one batch
of eval_every (64) PDHG iterations (fused primal step + extrapolated dual
step) and its FP64 KKT evaluation with the restart / snapshot / stop
decisions, i.e. every stage of the hot path, replayed as one HIP graph.
value = PDHG iterations per second over the timed steps, all data resident
in HBM.

Also reported, outside the timed region:
  - per-kernel HIP-event durations and the algorithmic HBM bandwidth of the
    dominant kernel (roofline), its gather rate against the random-gather
    ceiling measured live by the library's probe (pdhg_gather_probe);
  - the averaged variant (PDLP-style restarts) and FP32 bulk steps on the
    same LP;
  - the CPU oracle on a bounded sample of the same LP (cpu_baseline);
  - time to relative KKT 1e-8, FP64 vs FP32 bulk + FP64 refinement, on the
    headline LP and on the power-law and multicommodity LPs, each run capped
    so the whole benchmark fits its time budget (status and maxresid at the
    cap are reported when 1e-8 is not reached);
  - the multi-threaded CPU PDHG: iterations/s against the thread count;
  - Algorithm 1's harness: PDHG iterations/s with crossover threads running
    beside it, against the same iterations without them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("PDHG iters/s + HBM GB/s; time to rel KKT 1e-8, FP32+refine vs "
          "FP64, 1 GPU")
HBM_PEAK_GBS = 8000.0
T_START = time.time()


def log(msg: str):
    print(f"[bench {time.time() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def alg_bytes(m: int, n: int, nnz: int, fp: int = 8, has_l: bool = False):
    """Algorithmic HBM bytes of one primal and one dual step.

    Each step streams its CSR (values fp bytes + 4-byte column index per
    nonzero, 4-byte row pointers), gathers the other side's vector once, and
    reads / writes its own vectors once.
    Averaged iteration:
      primal (rows of A^T): x, c, xbar read; x, xbar written (+ l read)
      dual   (rows of A):   y, b, A~x, ybar read; y, A~x, ybar written
    Reflected Halpern iteration (same counts):
      primal: x, c, anchor x0 read; x^ = T_x(z) and the new x written
      dual:   y, b, A~x, anchor y0, A~x0 read; y, A~x written
    """
    primal = (fp + 4) * nnz + 4 * (n + 1) + fp * m + 5 * fp * n + (fp * n if has_l else 0)
    dual = (fp + 4) * nnz + 4 * (m + 1) + fp * n + 7 * fp * m
    return primal, dual


def _kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    # the kernels, their launch shapes and the row-block planner
    for f in ("kernels.hip", "internal.h", "host_csr.cpp"):
        with open(os.path.join(ROOT, "paper_2510_24429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, or None when it was taken on other sources."""
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(tfile):
        return None
    tr = {}
    with open(tfile) as f:
        for line in f:
            if not line.startswith("#") and ":" in line:
                k, v = line.split(":", 1)
                tr[k.strip()] = v.strip()
    if tr.get("kernel_source_hash") != _kernel_hash():
        return None
    return int(tr["bytes_per_launch"])


def rate_and_kernels(s, lp, steps, warmup, N=64, fp=8, profile_steps=None):
    """Time `steps` batches of N iterations after `warmup` (graphs), then the
    per-kernel HIP-event durations of a few more batches."""
    import torch
    restarts = [0]

    def step():
        st = s.iterate(N)
        if st != 0:        # converged inside the window: start over
            restarts[0] += 1
            s.set_iterate(None, None)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - ta
    s.profile(True)
    s.kernel_times(reset=True)
    for _ in range(profile_steps or max(3, min(10, steps))):
        step()
    kt = s.kernel_times(reset=True)
    s.profile(False)
    bp, bd = alg_bytes(lp.m, lp.n, lp.nnz, fp=fp)
    tp = kt["primal_step"]["total_ms"] / max(kt["primal_step"]["launches"], 1)
    td = kt["dual_step"]["total_ms"] / max(kt["dual_step"]["launches"], 1)
    return dict(elapsed=elapsed, iters_s=steps * N / elapsed, tp=tp, td=td,
                bp=bp, bd=bd, restarts=restarts[0],
                gbs_p=bp / (tp * 1e-3) / 1e9, gbs_d=bd / (td * 1e-3) / 1e9,
                iter_gbs=(bp + bd) / ((tp + td) * 1e-3) / 1e9)


def kernels_dict(r):
    return {"primal_step": {"us": round(r["tp"] * 1e3, 2), "alg_bytes": r["bp"],
                            "GB_s": round(r["gbs_p"], 1)},
            "dual_step": {"us": round(r["td"] * 1e3, 2), "alg_bytes": r["bd"],
                          "GB_s": round(r["gbs_d"], 1)},
            "iteration_GB_s": round(r["iter_gbs"], 1),
            "steps_only_iters_s": round(1e3 / (r["tp"] + r["td"]), 1),
            "iteration_frac": round(r["iter_gbs"] / HBM_PEAK_GBS, 4)}


TTK_LEVELS = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6]


def _level_times(s):
    """Seconds from the start of the iterations (after Ruiz and the power
    iteration) and iterations to the first snapshot at each level.  The
    refinement measures its refined point before every round and at the end,
    so its times are those of the round boundaries."""
    out = {}
    for i in range(s.snapshot_count()):
        inf = s.snapshot_info(i)
        out[f"{inf['level']:.0e}"] = {"t_s": round(inf["t_wall"], 3), "iters": inf["iter"]}
    return out


def time_to_kkt(s, lp, cap, variant, tag):
    """Wall time from data resident on the GPU (after load) to FP64 relative
    KKT <= 1e-8, including Ruiz scaling and the power iteration: the FP64
    path, then FP32 bulk iterations with FP64 refinement, on the loaded
    context `s`, each within `cap` seconds.  Each path also reports when it
    first reached the levels 1e-2 .. 1e-6 (snapshots), which compares the
    two paths on an LP that neither finishes within the cap."""
    import numpy as np
    import torch
    res = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.configure(eps_rel=1e-8, time_limit_s=cap, variant=variant, levels=TTK_LEVELS)
    st = s.solve()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    inf = s.info()
    log(f"ttk {tag} fp64: {t:.2f}s status {st} iters {inf['iters']} restarts "
        f"{inf['restarts']} maxresid {inf['kkt']['maxresid']:.2e}")
    res["fp64"] = {"seconds": round(t, 3), "status": st, "cap_s": round(cap, 1),
                   "iters": inf["iters"], "restarts": inf["restarts"],
                   "maxresid": inf["kkt"]["maxresid"], "pobj": inf["kkt"]["pobj"],
                   "levels": _level_times(s)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.configure(eps_rel=1e-8, time_limit_s=cap, variant=variant, levels=TTK_LEVELS)
    r = s.solve_refined(outer_eps=1e-8, inner_eps=1e-4, max_rounds=12,
                        max_inner_iters=5_000_000)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log(f"ttk {tag} fp32+refine: {t:.2f}s status {r['status']} rounds "
        f"{r['rounds']} inner iters {r['inner_iters']} maxresid "
        f"{r['kkt']['maxresid']:.2e}")
    res["fp32_refine"] = {"seconds": round(t, 3), "status": r["status"],
                          "cap_s": round(cap, 1), "rounds": r["rounds"],
                          "inner_iters": r["inner_iters"],
                          "maxresid": r["kkt"]["maxresid"], "pobj": r["kkt"]["pobj"],
                          "levels": _level_times(s)}
    if res["fp64"]["status"] == 1 and res["fp32_refine"]["status"] == 1:
        res["speedup_fp32_refine"] = round(res["fp64"]["seconds"] /
                                           res["fp32_refine"]["seconds"], 3)
    # objective error of each result: against the planted optimum c^T x*
    # when the generator planted one, and between the two paths
    p64 = res["fp64"]["pobj"]
    if lp.x_star is not None:
        pstar = float(np.dot(lp.c, lp.x_star))
        for k in ("fp64", "fp32_refine"):
            res[k]["obj_rel_err_vs_planted"] = abs(res[k]["pobj"] - pstar) / (1 + abs(pstar))
    res["fp32_refine"]["obj_rel_diff_vs_fp64"] = (
        abs(res["fp32_refine"]["pobj"] - p64) / (1 + abs(p64)))
    return res


def alg1_harness_rate(s, variant, K=16384):
    """Algorithm 1 (Section 3.1) with a stand-in crossover: PDHG iterations/s
    over K iterations while the harness launches a crossover thread per
    snapshot (each sleeps 0.2 s and reports no success), against the same K
    iterations without the harness.  Rates from the library's own iteration
    time (t_iter), so the wait for the last crossover is not counted."""
    import threading
    levels = [1e-2, 1e-3, 1e-4, 1e-5]
    s.configure(eps_rel=1e-12, variant=variant, max_iters=K)
    s.solve()
    plain = s.info()
    started, lock = [], threading.Lock()

    def crossover(idx, info, x, y, z, cancelled):
        with lock:
            started.append(idx)
        time.sleep(0.2)
        return False

    s.configure(eps_rel=1e-12, variant=variant, max_iters=K, levels=levels)
    winner, status = s.concurrent_crossover(crossover)
    harn = s.info()
    r_plain = plain["iters"] / plain["t_iter"]
    r_harn = harn["iters"] / harn["t_iter"]
    log(f"alg1 harness: {r_harn:.1f} iters/s with {len(started)} crossovers, "
        f"{r_plain:.1f} without")
    return {"iters": K, "iters_s_plain": round(r_plain, 1),
            "iters_s_with_harness": round(r_harn, 1),
            "ratio": round(r_harn / r_plain, 4), "snapshots": s.snapshot_count(),
            "crossovers_started": len(started), "winner": winner, "status": status,
            "crossover": "stand-in: sleeps 0.2 s, never succeeds"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(lp, iters, variant):
    """The FP64 oracle, serial, on the same LP: `iters` iterations after its
    evaluation at k = 0, timed by the difference of two runs (0 and `iters`
    iterations), so the rate counts iterations alone.  Both runs skip Ruiz
    scaling and the power iteration (fixed step and primal weight), whose
    cost is setup, not iteration."""
    from oracle import oracle
    kw = dict(eps_rel=1e-8, eta=0.5, omega0=1.0, variant=variant, ruiz_passes=0,
              eval_every=1 << 30)
    t0 = time.time()
    r0 = oracle.solve(lp, max_iters=0, **kw)
    r1 = oracle.solve(lp, max_iters=iters, **kw)
    wall = time.time() - t0
    dt = r1.info["t_iter"] - r0.info["t_iter"]
    ips = r1.info["iters"] / dt
    log(f"cpu oracle: {r1.info['iters']} iters in {dt:.2f}s (evaluation "
        f"{r0.info['t_iter']:.2f}s, wall {wall:.1f}s)")
    return {"value": round(ips, 4), "unit": "iters/s", "cores": 1,
            "kind": "oracle", "host_cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{r1.info['iters']} PDHG iterations "
                      f"({['averaged', 'Halpern'][variant]}, FP64, serial "
                      f"C oracle) of the same LP, timed as the difference of "
                      f"runs of {iters} and 0 iterations so that the evaluation "
                      f"at k=0 is excluded; Ruiz and power iteration skipped "
                      f"(fixed step), 1 thread"}


def cpu_platform(lp, budget_s, variant):
    """The CPU PDHG (the same method on the host's cores, FP64) on one LP:
    iterations/s and algorithmic GB/s against the thread count, next to the
    host's streaming read bandwidth at the same thread count, and the thread
    count from which the rate stays within 10% of its best (saturation).
    Each point times iterations only (after the evaluation at k = 0), with a
    fixed step and no Ruiz passes (setup, not iteration)."""
    from paper_2510_24429_amd.cpu import CpuSolver, stream_bandwidth
    bp, bd = alg_bytes(lp.m, lp.n, lp.nnz)
    bytes_iter = bp + bd + 4 * (lp.m + lp.n + 2)   # 8-byte row pointers on the host
    cap = min(os.cpu_count() or 1, 64)
    ts, t = [], 1
    while t < cap:
        ts.append(t)
        t *= 2
    ts.append(cap)
    rows = []
    t_end = time.time() + budget_s
    s = CpuSolver.from_lp(lp, threads=1)
    for t in ts:
        if time.time() > t_end:
            break
        s.set_threads(t)
        s.configure(eps_rel=1e-12, ruiz_passes=0, eta=0.5, omega0=1.0,
                    variant=variant, eval_every=1 << 30)
        t0 = time.perf_counter()
        s.iterate(1)                     # the evaluation at k = 0 and one step
        t1 = time.perf_counter() - t0
        K = int(min(5000, max(2, 1.5 / max(t1 / 4.0, 1e-6))))   # ~1.5 s
        t0 = time.perf_counter()
        s.iterate(K)
        ips = K / (time.perf_counter() - t0)
        bw = stream_bandwidth(t, 1 << 30, 3)
        rows.append({"threads": t, "iters_s": round(ips, 2),
                     "GB_s": round(bytes_iter * ips / 1e9, 1),
                     "stream_read_GB_s": round(bw, 1),
                     "frac_of_stream": round(bytes_iter * ips / 1e9 / bw, 3)})
        log(f"cpu pdhg, {t} threads: {ips:.1f} iters/s, "
            f"{bytes_iter * ips / 1e9:.1f} GB/s (stream read {bw:.1f} GB/s)")
    s.close()
    best = max(r["iters_s"] for r in rows) if rows else 0.0
    sat = next((r["threads"] for r in rows if r["iters_s"] >= 0.9 * best), None)
    return {"kind": "cpu pdhg (FP64, same method and decisions)",
            "workload": lp.name, "bytes_per_iter": bytes_iter,
            "host_cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "saturation_threads": sat, "scaling": rows}


def gather_sweep(Solver):
    """The probe's random-gather rate by table size and panel count."""
    from paper_2510_24429_amd import lpgen
    lp = lpgen.make("uniform_m500_n1k")
    s = Solver.from_lp(lp, device=0)
    rows = []
    for mb in (1, 2, 4, 8, 16, 32, 64, 128, 160):
        ent = mb * 1048576 // 8
        for P in (1, 2, 4, 8):
            for nt in (0, 1):
                g = s.gather_probe(ent, panels=P, stream_nt=nt, n_gathers=1 << 26, reps=5)
                rows.append((mb, P, nt, g))
                print(f"table {mb:4d} MB  panels {P}  per-XCD {mb / P:7.2f} MB  "
                      f"stream_nt {nt}  {g / 1e9:7.1f} G gathers/s", flush=True)
    s.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="coupled_m5m_n20m")
    ap.add_argument("--budget", type=float, default=480.0,
                    help="seconds for the whole run: the time-to-KKT caps "
                         "shrink to fit it")
    ap.add_argument("--ttk-cap", type=float, default=150.0,
                    help="largest cap per time-to-KKT run (seconds)")
    ap.add_argument("--no-ttk", action="store_true", help="skip time-to-KKT runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU legs")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline workload only (no variant / FP32 rates, no "
                         "other workloads)")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle iterations for cpu_baseline (0: by size)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--variant", type=int, default=1,
                    help="0: averaged iterates with PDLP-style restarts; "
                         "1: reflected Halpern iteration (default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device copy of 256 MiB (reference for "
                         "the profiler's byte counters)")
    ap.add_argument("--gather-sweep", action="store_true",
                    help="print the probe's gather rates by table size and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not "
              "supported (the multi-GPU sharding is a design note only)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_24429_amd import lpgen
    from paper_2510_24429_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.gather_sweep:
        gather_sweep(Solver)
        return
    if args.copy_probe:
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def left():
        return args.budget - (time.time() - T_START)

    t0 = time.time()
    lp = lpgen.make(args.workload)
    log(f"generated {args.workload}: m={lp.m} n={lp.n} nnz={lp.nnz} "
        f"({time.time() - t0:.1f}s)")
    N = 64
    t0 = time.time()
    s = Solver.from_lp(lp, device=0)
    t_load = time.time() - t0
    s.configure(eps_rel=1e-8, eval_every=N, use_graph=0 if args.no_graph else 1,
                variant=args.variant)
    log(f"loaded ({t_load:.1f}s), configured ({s.info()['t_setup']:.2f}s setup), "
        f"panels A {s.panel_count(0)} A^T {s.panel_count(1)}")

    r = rate_and_kernels(s, lp, args.steps, args.warmup, N)
    value = r["iters_s"]
    log(f"timed {args.steps} steps: {r['elapsed']:.3f}s, {value:.1f} iters/s; "
        f"primal {r['tp']*1e3:.1f}us {r['gbs_p']:.0f}GB/s  dual {r['td']*1e3:.1f}us "
        f"{r['gbs_d']:.0f}GB/s  iteration {r['iter_gbs']:.0f}GB/s")
    dominant = "primal_step" if r["tp"] >= r["td"] else "dual_step"
    ach = r["gbs_p"] if dominant == "primal_step" else r["gbs_d"]
    # the same kernel's gathers (one per nonzero) against the probe's rate for
    # the table it gathers from (y of m entries for the primal step, x of n
    # for the dual step, each XCD holding 1/P of it when panelled)
    if dominant == "primal_step":
        cols, P, side = lp.m, s.panel_count(1), 1
        t_dom = r["tp"]
    else:
        cols, P, side = lp.n, s.panel_count(0), 0
        t_dom = r["td"]
    table_xcd = 8.0 * cols / P
    nt = 1 if table_xcd > 3 * 1048576 else 0     # the library's load-kind rule
    g_cap = s.gather_probe(cols, panels=P, stream_nt=nt, n_gathers=lp.nnz, reps=3)
    g_ach = lp.nnz / (t_dom * 1e-3)
    log(f"{dominant}: {g_ach / 1e9:.1f} G gathers/s against the probe's "
        f"{g_cap / 1e9:.1f} G/s ({table_xcd / 1048576:.1f} MB per XCD)")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["elapsed"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator, planted optimum)",
        "config": {"workload": args.workload, "m": lp.m, "n": lp.n,
                   "nnz": lp.nnz, "precision": "fp64", "eval_every": N,
                   "ruiz_passes": 10, "eps_rel": 1e-8,
                   "variant": ["averaged", "halpern"][args.variant],
                   "graphs": not args.no_graph,
                   "panels": [s.panel_count(0), s.panel_count(1)]},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": _traffic(dominant, args.workload),
                     "kernel": dominant},
        "kernels": kernels_dict(r),
        "gather_rate": {"kernel": dominant, "achieved": round(g_ach / 1e9, 1),
                        "ceiling": round(g_cap / 1e9, 1), "unit": "G gathers/s",
                        "ceiling_source": "pdhg_gather_probe, measured in this run",
                        "table_MB_per_xcd": round(table_xcd / 1048576.0, 2),
                        "frac": round(g_ach / g_cap, 4)},
        "restarts_of_run": r["restarts"],
    }

    if not args.no_extra:
        # the averaged variant and FP32 bulk steps on the same loaded LP
        s.configure(eps_rel=1e-8, eval_every=N, variant=0)
        r0 = rate_and_kernels(s, lp, max(5, args.steps // 2), 2, N)
        log(f"averaged variant: {r0['iters_s']:.1f} iters/s, primal {r0['tp']*1e3:.1f}us "
            f"dual {r0['td']*1e3:.1f}us")
        out["averaged_variant"] = {"iters_s": round(r0["iters_s"], 2),
                                   "kernels": kernels_dict(r0)}
        s.configure(eps_rel=1e-8, eval_every=N, variant=args.variant, precision=1)
        r32 = rate_and_kernels(s, lp, max(5, args.steps // 2), 2, N, fp=4)
        log(f"fp32 steps: {r32['iters_s']:.1f} iters/s, primal {r32['tp']*1e3:.1f}us "
            f"dual {r32['td']*1e3:.1f}us")
        out["fp32_steps"] = {"iters_s": round(r32["iters_s"], 2),
                             "kernels": kernels_dict(r32)}

    if not args.no_cpu:
        # about 15 s of serial iterations (the oracle runs 1.0-1.5 s per
        # iteration on 110M nonzeros), plus two evaluations at k = 0
        iters = args.cpu_iters or max(2, min(64, int(1.4e9 / max(lp.nnz, 1))))
        out["cpu_baseline"] = cpu_baseline(lp, iters, args.variant)

    ttk = {}
    if not args.no_extra:
        # the power-law LP (m = 200k, n = 1M): its rate, and both paths
        # to 1e-8 (they finish in about 45 s and 15 s)
        lp1 = lpgen.make("powerlaw_m200k_n1m")
        with Solver.from_lp(lp1, device=0) as s1:
            s1.configure(eps_rel=1e-8, eval_every=N, variant=args.variant)
            r1 = rate_and_kernels(s1, lp1, 40, 5, N)
            log(f"powerlaw_m200k_n1m: {r1['iters_s']:.1f} iters/s")
            out["powerlaw_m200k_n1m"] = {"iters_s": round(r1["iters_s"], 2),
                                         "kernels": kernels_dict(r1)}
            out["alg1_harness"] = alg1_harness_rate(s1, args.variant)
            if not args.no_ttk and left() > 150:
                ttk["powerlaw_m200k_n1m"] = time_to_kkt(
                    s1, lp1, min(args.ttk_cap, 90.0), args.variant, "powerlaw")
        if not args.no_cpu:
            out["cpu_platform"] = cpu_platform(lp1, min(40.0, max(left() - 300, 5.0)),
                                               args.variant)
            cp = out["cpu_platform"]["scaling"]
            if cp:
                out["cpu_platform"]["gpu_over_best_cpu"] = round(
                    r1["iters_s"] / max(r["iters_s"] for r in cp), 1)
        del lp1
        if not args.no_ttk and left() > 260:
            lp2 = lpgen.make("mcf_150knodes_600karcs_k8")
            with Solver.from_lp(lp2, device=0) as s2:
                cap = min(args.ttk_cap, (left() - 120) / 2)
                ttk["mcf_150knodes_600karcs_k8"] = time_to_kkt(
                    s2, lp2, cap, args.variant, "multicommodity")
            del lp2
    if not args.no_ttk:
        cap = min(args.ttk_cap, max(left() - 20, 20.0) / 2)
        ttk[args.workload] = time_to_kkt(s, lp, cap, args.variant, "headline")
        out["time_to_kkt"] = ttk
    s.close()
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
