#!/usr/bin/env python3
"""Throughput of the ion-flow step on one MI355X.

Workload: two 5 um grains on the axis 0.5 r_De apart, Mach 1 argon flow with
charge exchange (nu = 0.1 omega_pi), N = 2^20 ion superparticles in a
cylinder of radius 3 r_De and height 8 r_De, dt = 0.01/omega_pi; synthetic,
seeded initial state.  A step is the whole hot path: all-pairs forces, push
with collisions/absorption/exit/reinjection, charge and force bookkeeping.

Prints one JSON line: ion-steps/s (value), pair interactions/s, the FP32
roofline fraction of the pair kernel (per-launch HIP-event time), the HBM
rate of the push kernel, and the FP64 CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 23            # algorithmic FP32 flop per ordered pair
# FP32 flop the symmetric kernel executes per unordered pair: the 17 operations
# of the pair term with its transcendental steps (difference 3, r^2 5, rsqrt 1,
# r 1, exponent argument 1, exp 1, 1/r^2 1, (1 + r)/r^3 2, times e^-r 1) plus
# 3 fused multiply-adds into the target's sum (6) and 3 into the source's
# reaction (6): 28, against 2 x 23 = 46 for the two ordered pairs it covers.
FLOP_PER_UNIQUE_PAIR = 28
PEAK_FP32 = 157.3e12          # MI355X published FP32 vector peak (counts packed FP32)
PEAK_FP64 = 78.6e12           # MI355X published FP64 vector peak
PEAK_HBM = 8.0e12             # MI355X HBM3E, B/s


def measured_traffic(kernel: str, n_ions: int):
    """HBM bytes per launch of `kernel` from the committed memory-counter
    summary, or None if it is absent, for another size, or the kernel sources
    have changed since the counters were taken."""
    from paper_2205_06557_amd import pmc_summary as P
    path = os.path.join(ROOT, "profiles", "step_kernels_traffic.json")
    if not os.path.exists(path):
        return None
    s = json.load(open(path))
    if s.get("source_sha256") != P.kernel_sources_hash() or s.get("n_ions") != n_ions:
        return None
    k = s.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes"]


def measured_issue(n_ions: int):
    """VALU issue utilisation of the pair kernel (quad-cycles of issued VALU
    instructions over the SIMDs' available quad-cycles) from the committed
    instruction-counter summary, or None if absent, for another size, or the
    kernel sources have changed since."""
    from paper_2205_06557_amd import pmc_summary as P
    path = os.path.join(ROOT, "profiles", "pair_sym_counters.json")
    if not os.path.exists(path):
        return None
    s = json.load(open(path))
    if s.get("source_sha256") != P.kernel_sources_hash() or s.get("n_ions") != n_ions:
        return None
    return s.get("valu_issue_frac")


def copy_rate(nbytes: int, reps: int = 20) -> float:
    """GB/s of a plain device-to-device copy moving `nbytes` in total (read
    plus write), timed with events: what a transfer of the push kernel's
    size reaches on this device."""
    import torch
    half = max(nbytes // 2, 1)
    src = torch.empty(half, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2 * half * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def push_bytes_per_ion(prec: int) -> int:
    """Algorithmic bytes per ion of the step's tail kernel: with the symmetric
    FP32 pair sum it reads x, v and the int64 pair totals and writes the
    cleared totals, the acceleration, x, v and the event byte; with the
    one-sided (FP64) sum it reads x, v, a and writes x, v and the event byte."""
    if prec == 0:
        return 12 + 12 + 24 + 24 + 12 + 12 + 12 + 1
    e = 8
    return 3 * e * 3 + 2 * 3 * e + 1


def cpu_baseline(w, sysm, target_s: float):
    """The FP64 oracle's force evaluation on a sample of target ions of the
    same 2^20-ion state (every ion a source), scaled to ion-steps/s; and the
    error of the GPU's accelerations at that state on the sampled targets."""
    import numpy as np
    from oracle import oracle as O
    o = O.Oracle(w, init=False)
    x, v, q, step = sysm.get_state()
    lam, cs, wpi = o.derived["lam"], o.derived["cs"], o.derived["wpi"]
    o.set_state(x.T.astype(np.float64) * lam, v.T.astype(np.float64) * cs, q, step)
    sysm.step(1)                      # the GPU's forces at the same state (untimed)
    a_gpu = sysm.accelerations().T.astype(np.float64) * lam * wpi * wpi
    rng = np.random.default_rng(0)
    o.accel_subset(rng.choice(w.n_ions, size=16, replace=False))      # threads up, caches warm
    order = rng.permutation(w.n_ions)
    m2, chunk, dt = 0, 256, 0.0
    a_orc = []
    while dt < target_s and m2 + chunk <= w.n_ions:
        t0 = time.perf_counter()
        a_orc.append(o.accel_subset(order[m2:m2 + chunk]))
        dt += time.perf_counter() - t0
        m2 += chunk
    pairs = m2 * (w.n_ions - 1)
    pps = pairs / dt
    a_orc = np.concatenate(a_orc)
    a_g = a_gpu[order[:m2]]
    d = np.linalg.norm(a_g - a_orc, axis=1)
    mag = np.linalg.norm(a_orc, axis=1)
    rel = d / np.maximum(mag, math.sqrt(np.mean(mag ** 2)))
    err = {"targets": int(m2), "rel_l2": float(np.linalg.norm(a_g - a_orc) / np.linalg.norm(a_orc)),
           "p99_9": float(np.percentile(rel, 99.9)), "max": float(rel.max()),
           "note": "GPU FP32 accelerations vs the FP64 oracle at the timed run's final state; per-ion "
                   "error over max(|a_i|, rms |a|)"}
    return {
        "value": pps / (w.n_ions - 1),
        "unit": "ion-steps/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": f"FP64 ion accelerations (ion-ion + ion-dust + drive) for {m2} random target ions of "
                  f"the {w.n_ions}-ion state, all ions as sources ({pairs:.3e} pairs in {dt:.1f} s); "
                  f"ion-steps/s = pairs/s / (N-1); push, charging and reinjection are O(N) and omitted",
        "pairs_per_s": pps,
    }, err


FLOP_PER_CUT_PAIR = 40       # algorithmic FP32 flop per evaluated pair of the switched force


def cutoff_bench(args):
    """Constant-concentration series with the ion-ion cutoff (r_cut = 4,
    switched from 3 Debye lengths): the domain grows with N (2^16 ions per
    6 r_De of height), one grain at the origin.  Times K steps at each N,
    fits t ~ N^beta, and reports the largest N's rate as the value."""
    import numpy as np
    import torch
    from paper_2205_06557_amd import binding as B
    from paper_2205_06557_amd import workloads as W

    torch.cuda.set_device(0)
    series = []
    sizes = sorted(int(v) for v in args.cutoff_sizes.split(","))
    max_lg = sizes[-1]
    for lg in sizes:
        w = W.long_domain(1 << lg)
        s = B.System(w)
        s.set_cutoff(W.CUTOFF_SWITCH, W.CUTOFF_RADIUS)
        s.step(args.warmup)
        s.sync()
        s.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = s.kernel_times()
        s.set_timing(False)
        ns, npairs = s.cutoff_info()
        within = pairs_within_cutoff(s, w, W.CUTOFF_RADIUS) if lg == max_lg else None
        s.close()
        pair_ms = kt["pair"][0] / max(kt["pair"][1], 1)
        row = {"n_ions": w.n_ions, "H_over_lambda": w.H / w.lam, "slabs": ns,
               "ms_per_step": 1e3 * wall / args.steps, "pair_ms": pair_ms,
               "pairs_evaluated": npairs, "sources_per_ion": npairs / w.n_ions,
               "ion_steps_per_s": w.n_ions * args.steps / wall}
        if within is not None:
            row["pairs_within_cutoff"] = within
        series.append(row)
        print(f"[bench] cutoff N=2^{lg}: {row['ms_per_step']:.2f} ms/step, "
              f"{row['sources_per_ion']:.0f} sources per ion", file=sys.stderr, flush=True)
    n = np.array([r["n_ions"] for r in series], dtype=float)
    t = np.array([r["ms_per_step"] for r in series])
    beta = float(np.polyfit(np.log(n), np.log(t), 1)[0]) if len(series) > 1 else None
    last = series[-1]
    achieved = FLOP_PER_CUT_PAIR * last["pairs_evaluated"] / (last["pair_ms"] * 1e-3)
    within = last["pairs_within_cutoff"]
    achieved_within = FLOP_PER_CUT_PAIR * within["ordered_pairs"] / (last["pair_ms"] * 1e-3)
    res = {
        "metric": "ion-steps/s with the ion-ion cutoff, constant-concentration series",
        "value": last["ion_steps_per_s"],
        "unit": "ion-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": last["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one 5 um grain, R = 3 r_De, H = 6 r_De N/2^16, Mach 1, "
                               "nu = 0.1 omega_pi, cutoff 4 r_De switched from 3 r_De",
                   "n_ions": last["n_ions"]},
        "time_exponent_beta": beta,
        "series": series,
        "roofline": {"bound": "alu", "achieved": achieved_within / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved_within / PEAK_FP32, "traffic": None,
                     "kernel": "slab sort + pair_cut",
                     "flop_per_pair": FLOP_PER_CUT_PAIR,
                     "flop_convention": "ordered ion pairs closer than r_cut (the method's work), "
                                        "estimated from sampled targets",
                     "covered_pairs_frac": achieved / PEAK_FP32,
                     "covered_convention": "every ordered pair of the 256-ion sorted blocks the "
                                           "kernel covers, padding and pairs beyond r_cut included",
                     "launch_ms": last["pair_ms"]},
    }
    print(json.dumps(res), flush=True)


def pairs_within_cutoff(sysm, w, r_cut, n_targets=256, seed=0):
    """Ordered ion pairs closer than r_cut at the system's current state,
    estimated from n_targets random target ions (each against every other
    ion, exact distances in FP64): N times the mean count, with its standard
    error."""
    import numpy as np
    x = sysm.get_state()[0].astype(np.float64)           # [3][N], units of r_De
    rc = r_cut / w.lam
    rng = np.random.default_rng(seed)
    counts = []
    for i in rng.choice(x.shape[1], size=n_targets, replace=False):
        d2 = ((x - x[:, i:i + 1]) ** 2).sum(axis=0)
        counts.append(int(np.count_nonzero(d2 < rc * rc)) - 1)
    c = np.asarray(counts, dtype=np.float64)
    n = x.shape[1]
    return {"ordered_pairs": float(n * c.mean()), "std_error": float(n * c.std(ddof=1) / math.sqrt(len(c))),
            "targets_sampled": n_targets}


def crossover_bench(args):
    """Pair-phase time per launch of the one-sided and the symmetric all-pairs
    kernels on the single-grain workload at 2^12 .. 2^20 ions (HIP events on
    the launch stream, K steps after the warm-up)."""
    import torch
    from paper_2205_06557_amd import binding as B
    from paper_2205_06557_amd import workloads as W

    torch.cuda.set_device(0)
    rows = []
    for lg in range(12, 21, 2):
        w = W.single_grain_small().with_(n_ions=1 << lg)
        row = {"n_ions": w.n_ions}
        for name, kind in (("one_sided", B.PAIR_ONE_SIDED), ("symmetric", B.PAIR_SYMMETRIC)):
            s = B.System(w)
            s.set_pair_kernel(kind)
            s.step(args.warmup)
            s.sync()
            s.set_timing(True)
            s.step(args.steps)
            s.sync()
            kt = s.kernel_times()
            s.close()
            row[name + "_pair_ms"] = kt["pair"][0] / max(kt["pair"][1], 1)
        row["speedup"] = row["one_sided_pair_ms"] / row["symmetric_pair_ms"]
        rows.append(row)
        print(f"[bench] crossover N=2^{lg}: one-sided {row['one_sided_pair_ms']:.4f} ms, "
              f"symmetric {row['symmetric_pair_ms']:.4f} ms", file=sys.stderr, flush=True)
    big = rows[-1]
    achieved = FLOP_PER_PAIR * big["n_ions"] * (big["n_ions"] - 1) / (big["symmetric_pair_ms"] * 1e-3)
    res = {
        "metric": "pair-phase time per launch, one-sided vs symmetric all-pairs kernel",
        "value": big["symmetric_pair_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one 5 um grain, R = 3 r_De, H = 6 r_De, Mach 1, nu = 0.1 omega_pi",
                   "n_ions": big["n_ions"]},
        "series": rows,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": "pair_sym_kernel at the largest N", "flop_per_pair": FLOP_PER_PAIR},
    }
    print(json.dumps(res), flush=True)


def graph_bench(args):
    """Step time of small single systems launched kernel by kernel against
    the same steps replayed as HIP graphs of 10 steps (od_set_graph)."""
    import torch
    from paper_2205_06557_amd import binding as B
    from paper_2205_06557_amd import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    K = 200
    rows = []
    for n in (2000, 1 << 12, 1 << 14, 1 << 16):
        w = W.single_grain_small().with_(n_ions=n)
        row = {"n_ions": n}
        for name, g in (("single_launch_ms", 0), ("graph_ms", 10)):
            s = B.System(w, stream=stream.cuda_stream)
            s.set_graph(g)
            s.step(20)
            s.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(K)
            s.sync()
            row[name] = 1e3 * (time.perf_counter() - t0) / K
            s.close()
        row["speedup"] = row["single_launch_ms"] / row["graph_ms"]
        rows.append(row)
        print(f"[bench] graph N={n}: {row['single_launch_ms']:.4f} ms/step single launches, "
              f"{row['graph_ms']:.4f} ms/step graph", file=sys.stderr, flush=True)
    res = {
        "metric": "ms per step of small single systems, single launches vs HIP-graph replay",
        "value": rows[0]["graph_ms"], "unit": "ms", "n_gpus": 1, "steps": K, "warmup": 20,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one 5 um grain, R = 3 r_De, H = 6 r_De, Mach 1, nu = 0.1 omega_pi",
                   "n_ions": rows[0]["n_ions"], "steps_per_graph": 10},
        "series": rows,
    }
    print(json.dumps(res), flush=True)


def batch_bench(args):
    """Batched sweep: 64 single-grain systems, log2 N ~ U(14, 17), Mach, radius
    and collision frequency drawn per system; one launch per phase for all
    systems (autotuned decomposition, HIP-graph replay) against the same
    systems run one after another."""
    import torch
    from paper_2205_06557_amd import binding as B
    from paper_2205_06557_amd import workloads as W

    ws = W.sweep_systems(64)
    Ns = [w.n_ions for w in ws]
    tot = sum(Ns)
    pairs_step = sum(n * (n - 1) for n in Ns)
    K = args.steps
    print(f"[bench] batched sweep: {len(ws)} systems, N in [{min(Ns)}, {max(Ns)}], sum N = {tot}",
          file=sys.stderr, flush=True)
    b = B.Batch(ws)
    tune_ms = b.autotune(None)
    cfg = b.config()
    cfg["pair_kernel"] = "symmetric" if b.pair_kernel() == B.PAIR_SYMMETRIC else "one-sided"
    if cfg["pair_kernel"] == "symmetric":
        cfg["symmetric"] = b.sym_config()
    graph = 10 if K % 10 == 0 else 0
    b.set_graph(graph)
    b.step(max(args.warmup, 1) * (graph or 1))
    b.sync()
    b.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.sync()
    kt = b.kernel_times()
    b.close()
    print(f"[bench] batched: {1e3 * wall / K:.2f} ms/step; now the systems one after another",
          file=sys.stderr, flush=True)
    seq = 0.0
    for k, w in enumerate(ws):
        if k % 16 == 0:
            print(f"[bench] sequential runs {k}..{min(k + 15, len(ws) - 1)}", file=sys.stderr, flush=True)
        s = B.System(w)
        s.step(1)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        s.close()
    res = {
        "metric": "aggregate ion-steps/s, batched sweep of 64 systems",
        "value": tot * K / wall,
        "unit": "ion-steps/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 single-grain systems, log2 N ~ U(14,17) in multiples of 256, "
                               "Mach ~ U(0.3,2), radius ~ U(2,10) um, nu ~ U(0.02,0.3) omega_pi",
                   "sum_n_ions": tot, "decomposition": cfg, "graph_steps": graph,
                   "autotune_pair_ms": tune_ms},
        "pair_interactions_per_s": pairs_step * K / wall,
        "sequential_ion_steps_per_s": tot * K / seq,
        "speedup_vs_sequential": seq / wall,
        "roofline": {"bound": "alu", "achieved": FLOP_PER_PAIR * pairs_step * K / wall / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": FLOP_PER_PAIR * pairs_step * K / wall / PEAK_FP32, "traffic": None,
                     "kernel": "whole step (graph replay)"},
        "graph_ms": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
    }
    print(json.dumps(res), flush=True)


def surrogate_bench(args):
    """The surrogate against the plain method on the 8-grain chain (0.4 r_De
    spacing, Mach 1): the network trained on the packaged batched-solver runs,
    its errors on the held-out inputs beside the noise of their reference runs,
    and the wall time to the converged charge (200-step block means of the
    chain's mean charge within the band, 2 % by default, of an independent
    reference run; the steps until every grain is within 5 % beside it) from a
    cold start, from the isolated-grain OML charge and from the network's
    charges."""
    import numpy as np
    from paper_2205_06557_amd import surrogate as S

    def log(m):
        print(m, file=sys.stderr, flush=True)

    d = S.load_dataset()
    t0 = time.perf_counter()
    sur = S.Surrogate.train(d["X"], d["T"], epochs=600, seed=11)
    train_s = time.perf_counter() - t0
    P, inside = sur.predict_targets(d["Xh"])
    held = S.heldout_errors(P, d["Th"])
    Pl, _ = sur.predict_learned(d["Xh"])
    drag = S.heldout_errors(Pl, np.stack([S.to_learned(d["Xh"], t) for t in d["Th"]]))
    log(f"[bench] surrogate trained on {len(d['X'])} runs in {train_s:.2f} s; held-out: "
        f"{json.dumps(held)}")
    n = args.surrogate_ions
    rep = S.warm_start_study(S.STUDY_X, n, args.surrogate_ref_steps, args.surrogate_steps, sur, log=log,
                             band=args.surrogate_band)
    speed = rep.get("speedup_vs_cold")
    res = {
        "metric": "surrogate vs plain: wall-clock speed-up to the converged charge",
        "value": speed if speed is not None else rep.get("speedup_vs_cold_at_least"),
        "unit": "x (cold-start time / surrogate-start time)",
        "n_gpus": 1, "steps": args.surrogate_steps, "warmup": 0,
        "ms_per_step": 1e3 * rep["surrogate"]["seconds_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"8-grain chain, inputs {list(S.STUDY_X)} (Mach, radius um, spacing r_De, "
                               f"nu/omega_pi, Te/Ti), N = {n}, dt = {S.DT_WPI}/omega_pi, field-driven "
                               f"injection + confinement field",
                   "reference_steps": args.surrogate_ref_steps, "candidate_steps": args.surrogate_steps,
                   "band": args.surrogate_band, "block_steps": S.BLOCK,
                   "train_rows": int(len(d["X"])), "train_run_n_ions": d["n_ions"],
                   "heldout_inputs": int(len(d["Xh"])), "heldout_streams": int(d["Th"].shape[0])},
        "speedup_is_lower_bound": speed is None,
        "surrogate": {"charge_err_median": held["charge_rel_err"]["median"],
                      "charge_err_p90": held["charge_rel_err"]["p90"],
                      "charge_reference_se_median": held["charge_reference_se"]["median"],
                      "charge_rms_excess": held["charge_rms_excess"],
                      "force_err_median": held["force_rel_err"]["median"],
                      "force_err_p90": held["force_rel_err"]["p90"],
                      "force_reference_se_median": held["force_reference_se"]["median"],
                      "force_rms_excess": held["force_rms_excess"],
                      "ion_drag_err_median": drag["force_rel_err"]["median"],
                      "ion_drag_reference_se_median": drag["force_reference_se"]["median"],
                      "ion_drag_rms_excess": drag["force_rms_excess"],
                      "inside_box": int(inside.sum()), "train_s": train_s,
                      "start_charge_err_vs_reference": rep["surrogate"]["initial_max_rel_err"]},
        "warm_start": {k: {kk: rep[k][kk] for kk in ("initial_chain_rel_err", "initial_max_rel_err", "steps_to_band",
                                                      "steps_settled_in_band", "steps_settled_3pct",
                                                      "steps_every_grain_5pct", "steps_every_grain_3pct",
                                                      "seconds_to_band", "seconds_per_step")}
                       for k in ("cold", "oml", "surrogate")},
        "speedup_vs_cold_settled": rep.get("speedup_vs_cold_settled"),
        "reference_block_dev_chain_median": rep["reference_block_dev_chain_median"],
        "reference_block_dev_every_grain_median": rep["reference_block_dev_every_grain_median"],
        "reference_half_window_drift": rep["reference_half_window_drift"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-ions", type=int, default=1 << 20)
    ap.add_argument("--fp64", action="store_true", help="FP64 state and pair forces")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for memory counters)")
    ap.add_argument("--confinement", action="store_true",
                    help="add the confinement field of the outer plasma (Appendix A)")
    ap.add_argument("--cutoff", action="store_true",
                    help="the constant-concentration series with the ion-ion cutoff")
    ap.add_argument("--cutoff-sizes", default="17,18,19,20,21,22",
                    help="log2 N of the cutoff series (comma-separated)")
    ap.add_argument("--batch", action="store_true",
                    help="the batched 64-system sweep instead of the 2^20-ion two-grain workload")
    ap.add_argument("--crossover", action="store_true",
                    help="pair-phase times of the one-sided and symmetric kernels, 2^12 .. 2^20 ions")
    ap.add_argument("--graph", action="store_true",
                    help="small single systems: single launches against HIP-graph replay")
    ap.add_argument("--surrogate", action="store_true",
                    help="the surrogate against the plain method on the 8-grain chain")
    ap.add_argument("--surrogate-ions", type=int, default=1 << 16)
    ap.add_argument("--surrogate-ref-steps", type=int, default=24000)
    ap.add_argument("--surrogate-steps", type=int, default=8000)
    ap.add_argument("--surrogate-band", type=float, default=0.02,
                    help="relative band of the converged chain charge (200-step block means)")
    args = ap.parse_args()
    if args.surrogate and args.gpus == 1:
        sys.path.insert(0, ROOT)
        surrogate_bench(args)
        return
    if args.graph and args.gpus == 1:
        graph_bench(args)
        return
    if args.crossover and args.gpus == 1:
        crossover_bench(args)
        return
    if args.batch and args.gpus == 1:
        sys.path.insert(0, ROOT)
        batch_bench(args)
        return
    if args.cutoff and args.gpus == 1:
        cutoff_bench(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path here "
              "(the symmetric pair sum would shard by work item, with a reduce-scatter of its "
              "fixed-point totals, but no run uses a second GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_06557_amd import binding as B
    from paper_2205_06557_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(2)   # evicts the 256 MB MALL
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 268435456 B read, 268435456 B written", file=sys.stderr,
              flush=True)
        del src, dst, flush
    w = W.two_grain_wake().with_(n_ions=args.n_ions)
    if args.confinement:
        w = w.with_(flags=int(w.flags) | W.FLAG_CONFINEMENT)
    prec = B.PREC_FP64 if args.fp64 else B.PREC_FP32
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    sysm = B.System(w, precision=prec)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_setup)
    N = sysm.N
    print(f"[bench] {w.name}: N={N} grains={len(w.dust)} precision={'fp64' if prec else 'fp32'}",
          file=sys.stderr, flush=True)
    sysm.step(args.warmup)
    sysm.sync()
    torch.cuda.synchronize()
    if torch.distributed.is_available() and torch.distributed.is_initialized():
        torch.distributed.barrier()
    sysm.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sysm.sync()
    kt = sysm.kernel_times()
    sysm.set_timing(False)
    ms_step = 1e3 * wall / args.steps
    ion_steps = N * args.steps / wall
    pairs = N * (N - 1) * args.steps / wall
    pair_ms = kt["pair"][0] / max(kt["pair"][1], 1)
    push_ms = kt["tail"][0] / max(kt["tail"][1], 1)
    rein_ms = kt["reinject"][0] / max(kt["reinject"][1], 1)
    achieved = FLOP_PER_PAIR * N * (N - 1) / (pair_ms * 1e-3)
    executed = FLOP_PER_UNIQUE_PAIR * N * (N - 1) / 2 / (pair_ms * 1e-3)
    peak = PEAK_FP64 if prec else PEAK_FP32
    push_gbs = push_bytes_per_ion(prec) * N / (push_ms * 1e-3)
    q, _ = sysm.charges()
    res = {
        "metric": "ion-steps/s and pair-interactions/s at 2^20 ions",
        "value": ion_steps,
        "unit": "ion-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec else "f32",
        "data": "synthetic",
        "config": {"workload": f"two-grain wake pair, N={N} ions, 2 grains (r=5um, z=-/+0.25 r_De), "
                               "Mach 1, nu=0.1 omega_pi, R=3 r_De, H=8 r_De, dt=0.01/omega_pi"
                               + (", confinement field on" if args.confinement else ""),
                   "n_ions": N, "n_dust": len(w.dust), "precision": "fp64" if prec else "fp32",
                   "confinement": bool(args.confinement)},
        "setup_ms": setup_ms,
        "pair_interactions_per_s": pairs,
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None if prec else measured_traffic("pair", N),
            "kernel": "pair_forces_f64" if prec else "pair_sym_kernel",
            "flop_per_pair": FLOP_PER_PAIR,
            "flop_convention": "algorithmic: 23 flop per ordered pair, N(N-1) pairs per launch",
            "launch_ms": pair_ms,
        },
        "tail_roofline": {
            "bound": "hbm",
            "achieved": push_gbs / 1e9,
            "peak": PEAK_HBM / 1e9,
            "unit": "GB/s",
            "frac": push_gbs / PEAK_HBM,
            "traffic": None if prec else measured_traffic("tail", N),
            "bytes_per_ion": push_bytes_per_ion(prec),
            "kernel": "step_tail_kernel",
            "launch_ms": push_ms,
        },
        "kernel_ms": {"pair": pair_ms, "tail": push_ms, "reinject": rein_ms},
        "dust_charge_e": [float(x) / 1.602176634e-19 for x in q],
    }
    if not prec:
        # the work the symmetric kernel executes: each unordered pair once
        res["roofline"]["executed"] = {
            "flop_per_unique_pair": FLOP_PER_UNIQUE_PAIR, "unique_pairs": N * (N - 1) // 2,
            "achieved": executed / 1e12, "unit": "TFLOP/s", "frac": executed / PEAK_FP32,
            "valu_issue_frac": measured_issue(N)}
    res["tail_roofline"]["copy_reference_gbs"] = copy_rate(push_bytes_per_ion(prec) * N)
    if not args.no_cpu:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        res["cpu_baseline"], res["gpu_vs_oracle_accel_error"] = cpu_baseline(w, sysm, args.cpu_seconds)
    sysm.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
