"""Precision report: FP32 pair tiles against the full-FP64 GPU run and the
FP64 oracle, on the two-grain wake pair.

From one common state (the FP32 system's, loaded exactly into the FP64
system) both GPU modes take one step; accelerations are compared on every
ion between the two modes and, for a random 2^14-ion target subsample (all
ions as sources), against the oracle; grain forces and charges are compared
against the oracle.  Both modes then run freely for a few hundred steps and
the time-averaged charges and forces are compared, with block standard
errors (trajectories decorrelate, so only statistical agreement is
expected).  The nonreciprocal total force on each grain is reported.

Environment: ODUST_PRECISION_N (default 2^16 ions), ODUST_PRECISION_STEPS
(default 300), ODUST_REPORT (path of a JSON report to write).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import accel_errors, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


def _block_stats(trace, nb=6):
    trace = np.asarray(trace)
    bl = len(trace) // nb
    m = trace[: nb * bl].reshape(nb, bl, *trace.shape[1:]).mean(axis=1)
    return m.mean(axis=0), m.std(axis=0, ddof=1) / math.sqrt(nb)


def test_precision_report(B):
    N = int(os.environ.get("ODUST_PRECISION_N", 1 << 16))
    steps = int(os.environ.get("ODUST_PRECISION_STEPS", 300))
    w = W.two_grain_wake().with_(n_ions=N, n_discard=0)
    say("precision report", w.name, "N", N, "steps", steps)
    rep = {"workload": w.name, "n_ions": N}
    with B.System(w) as s32, B.System(w, precision=B.PREC_FP64) as s64:
        s32.step(20)
        x, v, q, st = s32.get_state()
        s64.set_state(x.astype(np.float64), v.astype(np.float64), q, st)
        o = O.Oracle(w, init=False)
        lam, cs, wpi = o.derived["lam"], o.derived["cs"], o.derived["wpi"]
        o.set_state(x.T.astype(np.float64) * lam, v.T.astype(np.float64) * cs, q, st)
        s32.step(1)
        s64.step(1)
        s32.sync()
        s64.sync()
        acc = lam * wpi * wpi
        a32 = s32.accelerations().T.astype(np.float64) * acc
        a64 = s64.accelerations().T * acc
        rng = np.random.default_rng(3)
        idx = np.sort(rng.choice(N, size=min(N, 1 << 14), replace=False))
        ao = o.accel_subset(idx)
        e32 = accel_errors(a32[idx], ao)
        e64 = accel_errors(a64[idx], ao)
        e3264 = accel_errors(a32, a64)
        say("  accel fp32 vs oracle", e32, " fp64 vs oracle", e64, " fp32 vs fp64 (all ions)", e3264)
        rep["step_accel_err"] = {"fp32_vs_oracle": e32, "fp64_vs_oracle": e64, "fp32_vs_fp64": e3264}
        assert e32[0] <= 1e-5 and e32[1] <= 1e-5
        assert e64[0] <= 1e-10
        Fo = o.dust_forces()
        F32 = s32.forces(0)
        F64 = s64.forces(0)
        ferr = {}
        for name, F in (("fp32", F32), ("fp64", F64)):
            ferr[name] = [float(np.linalg.norm(F[d, 0] - Fo[d, 0]) / np.linalg.norm(Fo[d, 0]))
                          for d in range(2)]
        say("  Eq.(1) force rel err", ferr)
        rep["step_orbit_force_err"] = ferr
        assert max(ferr["fp32"]) <= 1e-5 and max(ferr["fp64"]) <= 1e-9
        # free-running time averages
        tr = {"fp32": [], "fp64": []}
        for k in range(steps):
            s32.step(1)
            s64.step(1)
            if (k + 1) % 20 == 0:
                s64.sync()
                say(f"  free-running steps {k + 1}/{steps}")
            for name, s in (("fp32", s32), ("fp64", s64)):
                if k % 5 == 0:
                    qn, _ = s.charges()
                    F = s.forces(0)
                    tr[name].append(np.concatenate([qn, F[:, :, 2].sum(axis=1), F[:, 0, 2]]))
        avg = {}
        for name in tr:
            m, se = _block_stats(tr[name])
            avg[name] = {"Q_C": m[:2].tolist(), "Q_se": se[:2].tolist(), "Fz_total_N": m[2:4].tolist(),
                         "Fz_total_se": se[2:4].tolist(), "Fz_orbit_N": m[4:6].tolist()}
        dq = np.abs(np.array(avg["fp32"]["Q_C"]) / np.array(avg["fp64"]["Q_C"]) - 1)
        rep["time_avg"] = avg
        rep["time_avg_charge_rel_diff_fp32_vs_fp64"] = dq.tolist()
        Ftot = np.array(avg["fp32"]["Fz_total_N"])
        rep["nonreciprocal_Fz_sum_N"] = float(Ftot.sum())
        say("  time averages", json.dumps(avg))
        say("  charge rel diff fp32/fp64", dq, " nonreciprocal F1z+F2z =", Ftot.sum())
        se = np.maximum(np.array(avg["fp32"]["Q_se"]), np.array(avg["fp64"]["Q_se"]))
        assert np.all(np.abs(np.array(avg["fp32"]["Q_C"]) - np.array(avg["fp64"]["Q_C"]))
                      <= 5 * math.sqrt(2) * se + 0.01 * np.abs(avg["fp64"]["Q_C"]))
    path = os.environ.get("ODUST_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(rep, f, indent=1, default=float)
