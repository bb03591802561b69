"""Precision study (E1): FP32 pair tiles against the full-FP64 GPU mode and the
FP64 oracle, on the two-grain wake pair under the paper's boundary model
(Section 2 and Appendix A: the confinement field of the outer plasma, and
injection from the field-driven flow's stationary distribution).

Protocol:
  * one FP32 run from the initial state; at each snapshot step k the forces
    at its state x_k are taken three ways: the FP32 run's own step k, a
    FP64-mode system loaded with x_k (exactly) and stepped once, and the
    oracle on a random 2^14-ion target subsample (all ions as sources).
    Ion accelerations and the grain forces of Eq. (1) carry their error
    against the oracle;
  * the per-step charges and forces of the FP32 run come from the on-device
    history; their time averages over the second half of the run are
    reported with block-bootstrap standard errors, and so is the sum of the
    two grains' total axial forces (the nonreciprocal force; zero if the
    grains' interaction were reciprocal);
  * a FP64-mode run from the same initial state gives time averages over the
    same window of its shorter run; FP32 and FP64 must agree within five
    combined standard errors (N-body trajectories are chaotic, so only
    statistical agreement is expected).

Environment: ODUST_PRECISION_N (default 2^16 ions), ODUST_PRECISION_STEPS
(FP32 run, default 300), ODUST_PRECISION_FP64_STEPS (default 100; 0 skips
the FP64 run), ODUST_PRECISION_SNAPSHOTS (comma-separated steps, default
0,100,300; empty for none),
ODUST_PRECISION_PLAIN=1 for the plain boundary model (shifted-Maxwellian
injection, no confinement field), ODUST_REPORT (path of a JSON report).
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


def _bootstrap(series, nblocks=10, nboot=2000, seed=0):
    """(mean, block-bootstrap standard error) of a time series along axis 0."""
    x = np.asarray(series, dtype=np.float64)
    b = len(x) // nblocks
    blocks = x[: b * nblocks].reshape(nblocks, b, *x.shape[1:]).mean(axis=1)
    rng = np.random.default_rng(seed)
    means = blocks[rng.integers(0, nblocks, size=(nboot, nblocks))].mean(axis=1)
    return x.mean(axis=0), means.std(axis=0, ddof=1)


def _rel(f, r):
    """|f - r| / |r|; an uncharged grain has no Eq. (1) force, and then f must be 0 too."""
    d, n = float(np.linalg.norm(f - r)), float(np.linalg.norm(r))
    return d / n if n > 0 else (0.0 if d == 0 else math.inf)


def _averages(h, w0):
    """Time averages of a history [steps, grains, 14] from record w0 on:
    charges (C), total axial force per grain and its orbit part (N), and the
    nonreciprocal sum of the totals."""
    tail = h[w0:]
    q, q_se = _bootstrap(tail[:, :, 0])
    fz = tail[:, :, 3:13:3]                      # z components of the four parts
    tot, tot_se = _bootstrap(fz.sum(axis=2))
    orb, orb_se = _bootstrap(fz[:, :, 0])
    nr, nr_se = _bootstrap(fz.sum(axis=2).sum(axis=1))
    return {"Q_C": q.tolist(), "Q_se": q_se.tolist(), "Fz_total_N": tot.tolist(), "Fz_total_se": tot_se.tolist(),
            "Fz_orbit_N": orb.tolist(), "Fz_orbit_se": orb_se.tolist(),
            "nonreciprocal_Fz_sum_N": float(nr), "nonreciprocal_se": float(nr_se), "window_steps": len(tail)}


def test_precision_study(B):
    N = int(os.environ.get("ODUST_PRECISION_N", 1 << 16))
    steps = int(os.environ.get("ODUST_PRECISION_STEPS", 300))
    steps64 = int(os.environ.get("ODUST_PRECISION_FP64_STEPS", 100))
    snaps = sorted(int(v) for v in os.environ.get("ODUST_PRECISION_SNAPSHOTS", "0,100,300").split(",") if v.strip())
    snaps = [k for k in snaps if k <= steps]
    plain = os.environ.get("ODUST_PRECISION_PLAIN") == "1"
    flags = 0 if plain else W.FLAG_FIELD_DRIVEN | W.FLAG_CONFINEMENT
    w = W.two_grain_wake().with_(n_ions=N, n_discard=0, flags=flags)
    say("precision study", w.name, "N", N, "FP32 steps", steps, "FP64 steps", steps64, "snapshots", snaps,
        "boundary model", "plain" if plain else "field-driven injection + confinement field")
    rep = {"workload": w.name, "n_ions": N, "steps_fp32": steps, "steps_fp64": steps64,
           "boundary_model": "plain" if plain else "field-driven injection + confinement field", "snapshots": []}
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(N, size=min(N, 1 << 14), replace=False))
    with B.System(w) as s32:
        s32.set_history(steps + 1)
        x0, v0, q0, st0 = s32.get_state()
        o = O.Oracle(w, init=False)
        lam, cs, wpi = o.derived["lam"], o.derived["cs"], o.derived["wpi"]
        acc = lam * wpi * wpi
        coef = None
        if int(flags) & W.FLAG_CONFINEMENT:
            # the oracle's field: the GPU's fitted coefficients (the fit itself is pinned separately)
            coef, _ = s32.confinement()
            o.set_confinement(coef)
        done = 0
        for k in snaps:
            while done < k:                               # progress lines every 250 steps
                m = min(250, k - done)
                s32.step(m)
                s32.sync()
                done += m
                say(f"  FP32 run at step {done}")
            x, v, q, st = s32.get_state()
            s32.step(1)                                   # forces at x_k
            done += 1
            a32 = s32.accelerations().T.astype(np.float64) * acc
            F32 = s32.forces(0)
            with B.System(w, precision=B.PREC_FP64) as s64:
                s64.set_state(x.astype(np.float64), v.astype(np.float64), q, st)
                s64.step(1)
                a64 = s64.accelerations().T * acc
                F64 = s64.forces(0)
                coef64 = s64.confinement()[0] if int(flags) & W.FLAG_CONFINEMENT else None
            o.set_state(x.T.astype(np.float64) * lam, v.T.astype(np.float64) * cs, q, st)
            ao = o.accel_subset(idx)
            Fo = o.dust_forces()
            ao64, Fo64 = ao, Fo
            if coef64 is not None:
                # the FP64 system fitted its field to its own (FP64) initial ions:
                # the oracle takes those coefficients for the FP64 comparison
                o.set_confinement(coef64)
                ao64, Fo64 = o.accel_subset(idx), o.dust_forces()
                o.set_confinement(coef)
            e32 = accel_errors(a32[idx], ao)
            e64 = accel_errors(a64[idx], ao64)
            e3264 = accel_errors(a32, a64)
            ferr = {name: [_rel(F[d, 0], R[d, 0]) for d in range(2)]
                    for name, F, R in (("fp32", F32, Fo), ("fp64", F64, Fo64))}
            snap = {"step": k, "accel_fp32_vs_oracle": e32, "accel_fp64_vs_oracle": e64,
                    "accel_fp32_vs_fp64_all_ions": e3264, "eq1_force_rel_err": ferr,
                    "grain_charge_C": q.tolist()}
            rep["snapshots"].append(snap)
            say("  snapshot", json.dumps(snap, default=float))
            assert e32[0] <= 1e-5 and e32[1] <= 1e-5
            assert e64[0] <= 1e-10
            assert max(ferr["fp32"]) <= 1e-5 and max(ferr["fp64"]) <= 1e-9
        while done < steps:
            m = min(250, steps - done)
            s32.step(m)
            s32.sync()
            done += m
            say(f"  FP32 run at step {done}")
        h32 = s32.history()
    rep["time_avg_fp32"] = _averages(h32, len(h32) // 2)
    say("  FP32 time averages (second half):", json.dumps(rep["time_avg_fp32"]))
    _write(rep)
    if steps64 == 0:
        return
    # FP64 run from the same initial state, its own history
    w64 = w
    with B.System(w64, precision=B.PREC_FP64) as s64:
        s64.set_state(x0.astype(np.float64), v0.astype(np.float64), q0, st0)
        s64.set_history(steps64 + 1)
        for k in range(0, steps64, 25):
            s64.step(min(25, steps64 - k))
            s64.sync()
            say(f"  FP64 run at step {min(k + 25, steps64)}/{steps64}")
        h64 = s64.history()
    w0 = len(h64) // 2
    a32w = _averages(h32[: len(h64)], w0)
    a64w = _averages(h64, w0)
    rep["time_avg_fp32_fp64_window"] = a32w
    rep["time_avg_fp64"] = a64w
    verdict = []
    for key, sek in (("Q_C", "Q_se"), ("Fz_total_N", "Fz_total_se")):
        d = np.abs(np.array(a32w[key]) - np.array(a64w[key]))
        se = np.hypot(np.array(a32w[sek]), np.array(a64w[sek]))
        rel = d / np.maximum(np.abs(np.array(a64w[key])), 1e-300)
        verdict.append({"quantity": key, "abs_diff": d.tolist(), "combined_se": se.tolist(), "rel_diff": rel.tolist()})
        say(f"  FP32 vs FP64 {key}: diff {d} combined se {se} rel {rel}")
        assert np.all(d <= 5 * se + 1e-9 * np.abs(np.array(a64w[key]))), (key, d, se)
    rep["fp32_vs_fp64_time_avg"] = verdict
    _write(rep)


def _write(rep):
    path = os.environ.get("ODUST_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(rep, f, indent=1, default=float)
