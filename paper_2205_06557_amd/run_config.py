"""Runs a named workload on the GPU and reports its time-averaged dust charges
and forces (Eqs. (1)-(4)) with block standard errors, plus throughput.

    python -m paper_2205_06557_amd.run_config single-grain-production --mach 1.0 [--steps 10000]
    python -m paper_2205_06557_amd.run_config two-grain-wake --steps 2000

The charges and forces of every step are recorded (one device-to-host copy
per block of steps) so that block averages give a standard error of the
time averages.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

NAMES = {
    "single-grain-small": lambda a: W.single_grain_small(a.seed or 1),
    "single-grain-production": lambda a: W.single_grain_production(a.mach, a.seed or 11),
    "two-grain-wake": lambda a: W.two_grain_wake(a.seed or 2),
    "chain8": lambda a: W.chain8(seed=a.seed or 4),
}


def run(w, steps: int, n_discard: int, block: int = 100, log=None, precision: int = 0):
    from . import binding as B
    w = w.with_(n_discard=n_discard)
    s = B.System(w, precision=precision)
    s.set_timing(True)
    nb = steps // block
    qs, fs = [], []
    t0 = time.time()
    for b in range(nb):
        s.step(block)
        s.sync()
        if (b + 1) * block > n_discard:
            q, _ = s.charges()
            qs.append(q)
            fs.append(s.forces(0))
        if log and (b + 1) % max(1, nb // 20) == 0:
            log(f"  step {(b + 1) * block}/{steps} ({time.time() - t0:.1f} s)")
    wall = time.time() - t0
    kt = s.kernel_times()
    qa, _ = s.charges()
    _, qavg = s.charges()
    favg = s.forces(1)
    s.close()
    # block statistics of the per-block samples (one sample per block of steps)
    qs = np.array(qs)
    fs = np.array(fs)
    nblk = max(2, min(10, len(qs) // 2))
    def se(a):
        if len(a) < 4:
            return np.full(a.shape[1:], float("nan"))
        k = len(a) // nblk
        m = a[: k * nblk].reshape(nblk, k, *a.shape[1:]).mean(axis=1)
        return m.std(axis=0, ddof=1) / math.sqrt(nblk)
    N = w.n_ions
    res = {
        "workload": w.name, "n_ions": N, "steps": steps, "n_discard": n_discard,
        "q_avg_e": (qavg / W.QE).tolist(), "q_avg_se_e": (se(qs) / W.QE).tolist(),
        "F_avg_N": favg.tolist(),
        "F_parts": ["orbit (Eq. 1)", "dust-dust (Eq. 2)", "collection (Eq. 3)", "external (Eq. 4)"],
        "ion_drag_z_N": (favg[:, 0, 2] + favg[:, 2, 2]).tolist(),
        "ion_drag_z_se_N": (se(fs[:, :, 0, 2] + fs[:, :, 2, 2]) if len(fs) else np.zeros(0)).tolist(),
        "total_z_N": favg[:, :, 2].sum(axis=1).tolist(),
        "wall_s": wall,
        "ion_steps_per_s": N * steps / wall,
        "pair_interactions_per_s": N * (N - 1) * steps / wall,
        "kernel_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
    }
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(NAMES))
    ap.add_argument("--mach", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--discard", type=int, default=None)
    ap.add_argument("--n-ions", type=int, default=None)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--field-driven", action="store_true",
                    help="inject from the field-driven flow's stationary distribution")
    ap.add_argument("--confinement", action="store_true",
                    help="add the confinement field of the outer plasma")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    w = NAMES[a.name](a)
    if a.n_ions:
        w = w.with_(n_ions=a.n_ions)
    flags = int(w.flags) | (W.FLAG_FIELD_DRIVEN if a.field_driven else 0) | \
        (W.FLAG_CONFINEMENT if a.confinement else 0)
    w = w.with_(flags=flags, name=w.name + (" field-driven" if a.field_driven else "") +
                (" confinement" if a.confinement else ""))
    steps = a.steps or w.n_steps
    disc = a.discard if a.discard is not None else min(w.n_discard, steps // 2)
    print(f"[run] {w.name}: N={w.n_ions}, {steps} steps, averages after {disc}", flush=True)
    res = run(w, steps, disc, log=lambda m: print(m, flush=True), precision=1 if a.fp64 else 0)
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
