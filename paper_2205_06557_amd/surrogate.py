"""Learned surrogate of the self-consistent dust-chain result.

A network (trained and evaluated by the library's kernels, ``binding.Mlp``)
maps five inputs -- Mach number, grain radius (um), spacing of the grains
(Debye lengths), collision frequency (units of omega_pi), T_e/T_i -- to the
time-averaged charge and axial force of each grain of a vertical chain of
eight grains.  Training data come from the batched solver (``binding.Batch``)
run on inputs drawn uniformly in the input box.  Uses:

* warm start: the predicted charges start a full simulation near its
  self-consistent state;
* fast evaluator: charges and forces without simulating, with the full
  method as the fallback outside the input box and as the reference for its error.

Targets are made dimensionless before training: charge by
4 pi eps0 a k_B T_e / e (grain potential in units of k_B T_e / e) and force
by a^2 n k_B T_e.

Command line (GPU):
    python -m paper_2205_06557_amd.surrogate generate --out DIR --tag train --start 0 --count 512
    python -m paper_2205_06557_amd.surrogate evaluate --data DIR --out DIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Optional, Sequence

import numpy as np

from . import workloads as W

FEATURES = ("mach", "radius_um", "spacing_debye", "nu_over_wpi", "te_over_ti")
BOX_LO = np.array([0.3, 2.0, 0.25, 0.02, 10.0])
BOX_HI = np.array([2.0, 10.0, 1.0, 0.3, 100.0])
N_GRAINS = 8
TE_EV = 1.0
N_INF = 1e14


def sweep_inputs(n: int, seed: int, lo=BOX_LO, hi=BOX_HI) -> np.ndarray:
    """n input points uniform in the box (seeded Philox stream)."""
    rng = np.random.Generator(np.random.Philox(key=[seed, 4]))
    return lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(n, 5))


DT_WPI = 0.04      # time step of the surrogate protocol, units of 1/omega_pi
AVG_STEPS = 2000   # trailing steps averaged for the targets


def chain_workload(x5: Sequence[float], n_ions: int, steps: int, seed: int, system_id: int,
                   q0: Optional[Sequence[float]] = None, n_discard: Optional[int] = None,
                   dt_wpi: float = DT_WPI, avg_steps: int = AVG_STEPS) -> W.Workload:
    """The 8-grain vertical chain for one input point: grains of radius a on the
    axis at z_k = (k - 3.5) d, cylinder R = 3 r_De, H = 7 d + 5 r_De, argon at
    T_e = 1 eV, n = 1e14 m^-3, self-consistent charging, dt = dt_wpi/omega_pi
    (0.04 by default: the grain charging time is ~70/omega_pi, so a 6,000-step
    run spans ~3.4 charging times).  q0: initial charges (C), default 0;
    n_discard: default steps - avg_steps."""
    mach, a_um, d_l, nu_w, tt = (float(v) for v in x5)
    te = W.ev_to_kelvin(TE_EV)
    lam = W.debye_length(te, N_INF)
    wpi = W.ion_plasma_frequency(N_INF, W.M_ARGON)
    a = a_um * 1e-6
    d = d_l * lam
    q0 = [0.0] * N_GRAINS if q0 is None else list(q0)
    dust = [(0.0, 0.0, (k - 3.5) * d, a, float(q0[k])) for k in range(N_GRAINS)]
    return W.Workload(Te=te, Ti=te / tt, n_inf=N_INF, m_i=W.M_ARGON, mach=mach, nu_in=nu_w * wpi,
                      E_ext=float("nan"), R=3 * lam, H=7 * d + 5 * lam, dt=dt_wpi / wpi,
                      n_ions=int(n_ions), n_steps=int(steps),
                      n_discard=int(max(steps - avg_steps, 0) if n_discard is None else n_discard),
                      seed=seed,
                      system_id=system_id, charge_mode=W.CHARGE_CONSISTENT, dust=dust,
                      name=f"chain8 {x5}")


def charge_scale(x5) -> float:
    """C per unit of normalised charge: 4 pi eps0 a k_B T_e / e."""
    te = W.ev_to_kelvin(TE_EV)
    return 4 * math.pi * W.EPS0 * float(x5[1]) * 1e-6 * W.KB * te / W.QE


def force_scale(x5) -> float:
    """N per unit of normalised force: a^2 n k_B T_e."""
    te = W.ev_to_kelvin(TE_EV)
    a = float(x5[1]) * 1e-6
    return a * a * N_INF * W.KB * te


def to_targets(x5, q_c, fz_n) -> np.ndarray:
    return np.concatenate([np.asarray(q_c) / charge_scale(x5), np.asarray(fz_n) / force_scale(x5)])


def from_targets(x5, t16):
    t16 = np.asarray(t16, dtype=np.float64)
    return t16[:N_GRAINS] * charge_scale(x5), t16[N_GRAINS:] * force_scale(x5)


def oml_charge(x5) -> float:
    from . import binding as B
    w = chain_workload(x5, 16, 2, 0, 0)
    return B.oml_floating_charge(w, float(x5[1]) * 1e-6)


def run_plain(X: np.ndarray, n_ions: int, steps: int, seed: int, start: str = "oml",
              q0: Optional[np.ndarray] = None, batch_size: int = 512, graph: int = 10,
              log=None, avg_steps: int = AVG_STEPS) -> np.ndarray:
    """Runs the full method for every input row (batched) and returns the
    normalised targets [n, 16]: time-averaged charge and total axial force
    (Eqs. (1)-(4) summed) of each grain over the last avg_steps steps.
    start: "oml" (isolated-grain floating charge), "zero", or "given" (q0 [n, 8] in C)."""
    from . import binding as B
    n = X.shape[0]
    T = np.zeros((n, 16))
    for b0 in range(0, n, batch_size):
        rows = range(b0, min(n, b0 + batch_size))
        ws = []
        for r in rows:
            if start == "oml":
                q = [oml_charge(X[r])] * N_GRAINS
            elif start == "given":
                q = list(q0[r])
            else:
                q = None
            ws.append(chain_workload(X[r], n_ions, steps, seed, r, q, avg_steps=avg_steps))
        t0 = time.time()
        b = B.Batch(ws)
        b.autotune(None)
        if graph and steps % graph == 0:
            b.set_graph(graph)
        done = 0
        chunk = max(graph, 500 // graph * graph) if graph else 500
        while done < steps:
            k = min(chunk, steps - done)
            b.step(k)
            b.sync()
            done += k
            if log:
                log(f"  runs {b0}..{rows[-1]}: step {done}/{steps} ({time.time() - t0:.1f} s)")
        for i, r in enumerate(rows):
            _, qa = b.charges(i)
            F = b.forces(i, 1)
            T[r] = to_targets(X[r], qa, F[:, :, 2].sum(axis=1))
        b.close()
    return T


class Surrogate:
    """Trained network plus its normalisation; raw inputs in, physical outputs out."""

    def __init__(self, mlp, t_mean, t_std):
        self.mlp, self.t_mean, self.t_std = mlp, t_mean, t_std

    @classmethod
    def train(cls, X: np.ndarray, T: np.ndarray, epochs: int = 400, batch: int = 128,
              lr: float = 2e-3, lr_final: float = 2e-5, seed: int = 0):
        from . import binding as B
        mlp = B.Mlp(seed)
        mean = T.mean(axis=0)
        std = T.std(axis=0) + 1e-12
        mlp.set_normalization(BOX_LO, BOX_HI, mean, std)
        hist = mlp.train(X, T, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, seed=seed)
        s = cls(mlp, mean, std)
        s.history = hist
        return s

    def predict_targets(self, X):
        return self.mlp.predict(X)

    def predict(self, X):
        """(Q [n, 8] in C, F_z [n, 8] in N, inside [n]); outside the input box
        the caller must run the full method."""
        Y, inside = self.mlp.predict(X)
        Q = np.zeros((len(X), N_GRAINS))
        F = np.zeros((len(X), N_GRAINS))
        for r in range(len(X)):
            Q[r], F[r] = from_targets(X[r], Y[r])
        return Q, F, inside


def steps_to_converge(trace: np.ndarray, q_ref: np.ndarray, block: int, tol: float) -> Optional[int]:
    """First step count at which the mean charge of a block of `block` steps is
    within `tol` (relative) of q_ref for every grain; trace [steps, grains]."""
    nb = trace.shape[0] // block
    for k in range(nb):
        m = trace[k * block:(k + 1) * block].mean(axis=0)
        if np.all(np.abs(m / q_ref - 1.0) <= tol):
            return (k + 1) * block
    return None


def charge_trace(x5, n_ions: int, steps: int, seed: int, q0, every: int = 10):
    """Charges of a single chain run, read every `every` steps and held in
    between (the block means of the warm-start study average over them)."""
    from . import binding as B
    w = chain_workload(x5, n_ions, steps, seed, 0, q0)
    s = B.System(w)
    tr = np.zeros((steps, N_GRAINS))
    t0 = time.time()
    for k in range(steps):
        s.step(1)
        tr[k] = s.charges()[0] if (k % every == 0 or k + 1 == steps) else np.nan
        if (k + 1) % 2000 == 0:
            print(f"[surrogate]   step {k + 1}/{steps}, {time.time() - t0:.1f} s", flush=True)
    s.sync()
    # fill the unsampled steps by holding the last sample (block means only)
    last = tr[0]
    for k in range(steps):
        if np.isnan(tr[k, 0]):
            tr[k] = last
        else:
            last = tr[k]
    return tr, time.time() - t0


def generate(out: str, tag: str, total: int, start: int, count: int, n_ions: int, steps: int,
             seed: int, run_seed: int, avg_steps: int = AVG_STEPS):
    """Rows [start, start + count) of the sweep of `total` inputs (stream `seed`),
    run with the full method (random stream `run_seed`); saved as DIR/TAG_START.npz."""
    os.makedirs(out, exist_ok=True)
    X = sweep_inputs(total, seed)[start:start + count]
    t0 = time.time()
    print(f"[surrogate] {tag}: rows {start}..{start + count - 1}, N={n_ions}, {steps} steps, "
          f"averages over the last {avg_steps}", flush=True)
    T = run_plain(X, n_ions, steps, seed=run_seed, log=lambda m: print(m, flush=True), avg_steps=avg_steps)
    np.savez(os.path.join(out, f"{tag}_{start:05d}.npz"), X=X, T=T, n_ions=n_ions, steps=steps,
             avg_steps=avg_steps, seconds=time.time() - t0)
    print(f"[surrogate] {tag}: done in {time.time() - t0:.1f} s", flush=True)


def _load(data: str, tag: str, with_meta: bool = False):
    fs = sorted(f for f in os.listdir(data) if f.startswith(tag + "_") and f.endswith(".npz"))
    Xs, Ts, meta = [], [], {}
    for f in fs:
        z = np.load(os.path.join(data, f))
        Xs.append(z["X"])
        Ts.append(z["T"])
        meta = {"n_ions": int(z["n_ions"]), "steps": int(z["steps"]),
                "avg_steps": int(z["avg_steps"]) if "avg_steps" in z.files else AVG_STEPS}
    X, T = np.concatenate(Xs), np.concatenate(Ts)
    return (X, T, meta) if with_meta else (X, T)


def evaluate(data: str, out: str, epochs: int, eval_ions: int, eval_steps: int, seed: int = 11):
    """Trains on DATA/train_*.npz, compares with DATA/testa_*.npz and
    DATA/testb_*.npz (the same held-out inputs, two random streams), and runs
    the warm-start study; writes OUT/surrogate_result.json."""
    os.makedirs(out, exist_ok=True)

    def log(m):
        print(m, flush=True)

    X, T, meta = _load(data, "train", with_meta=True)
    Xt, Ta = _load(data, "testa")
    Xt2, Tb = _load(data, "testb")
    assert np.array_equal(Xt, Xt2)
    res = {"train_rows": int(len(X)), "test_rows": int(len(Xt)), "dt_wpi": DT_WPI,
           "run_n_ions": meta["n_ions"], "run_steps": meta["steps"], "avg_steps": meta["avg_steps"]}
    t1 = time.time()
    sur = Surrogate.train(X, T, epochs=epochs, seed=seed)
    res["train_s"] = time.time() - t1
    res["loss_first_last"] = [float(sur.history[0]), float(sur.history[-1])]
    np.save(os.path.join(out, "params.npy"), sur.mlp.params())
    np.savez(os.path.join(out, "norm.npz"), mean=sur.t_mean, std=sur.t_std)
    t2 = time.time()
    P, inside = sur.predict_targets(Xt)
    res["predict_s_per_point"] = (time.time() - t2) / len(Xt)
    ref = 0.5 * (Ta + Tb)
    q_err = np.abs(P[:, :8] / ref[:, :8] - 1.0)
    q_noise = np.abs(Ta[:, :8] / Tb[:, :8] - 1.0) / math.sqrt(2)
    fscale = np.abs(ref[:, 8:]).mean(axis=1, keepdims=True)
    f_err = np.abs(P[:, 8:] - ref[:, 8:]) / fscale
    f_noise = np.abs(Ta[:, 8:] - Tb[:, 8:]) / fscale / math.sqrt(2)

    def st(a):
        return {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)), "mean": float(a.mean())}
    res["charge_rel_err"] = st(q_err)
    res["charge_noise_of_reference"] = st(q_noise)
    res["force_rel_err_vs_mean_abs"] = st(f_err)
    res["force_noise_of_reference"] = st(f_noise)
    res["inside_box"] = int(inside.sum())
    # warm start vs cold start on one chain at a larger N
    x5 = np.array([1.0, 5.0, 0.4, 0.1, 33.3])
    Qp, Fp, _ = sur.predict(x5[None, :])
    q_oml = oml_charge(x5)
    log("[surrogate] warm-start study: reference run")
    ref_tr, ref_s = charge_trace(x5, eval_ions, eval_steps, seed + 5, Qp[0])
    q_ref = ref_tr[-eval_steps // 2:].mean(axis=0)
    ws = {"x": x5.tolist(), "n_ions": eval_ions, "steps": eval_steps, "q_ref_e": (q_ref / W.QE).tolist(),
          "surrogate_q_e": (Qp[0] / W.QE).tolist(), "oml_q_e": q_oml / W.QE,
          "surrogate_q_err_vs_ref": float(np.max(np.abs(Qp[0] / q_ref - 1))),
          "reference_seconds": ref_s}
    for name, q0 in (("cold", np.zeros(8)), ("oml", np.full(8, q_oml)), ("surrogate", Qp[0])):
        log(f"[surrogate] warm-start study: {name}")
        tr, secs = charge_trace(x5, eval_ions, eval_steps, seed + 6, q0)
        win = 500
        errs = [float(np.max(np.abs(tr[k:k + win].mean(axis=0) / q_ref - 1.0)))
                for k in range(0, eval_steps - win + 1, win)]
        ws[name] = {"initial_max_rel_err": float(np.max(np.abs(q0 / q_ref - 1.0))),
                    "window_steps": win, "window_max_rel_err": errs,
                    "steps_to_5pct": steps_to_converge(tr, q_ref, win, 0.05),
                    "steps_to_3pct": steps_to_converge(tr, q_ref, win, 0.03),
                    "seconds_per_step": secs / eval_steps}
    t3 = time.time()
    for _ in range(100):
        sur.predict(x5[None, :])
    ws["surrogate_seconds_per_eval"] = (time.time() - t3) / 100
    res["warm_start"] = ws
    with open(os.path.join(out, "surrogate_result.json"), "w") as f:
        json.dump(res, f, indent=1)
    log(json.dumps(res))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--out", required=True)
    g.add_argument("--tag", default="train")
    g.add_argument("--total", type=int, default=1024)
    g.add_argument("--start", type=int, default=0)
    g.add_argument("--count", type=int, default=512)
    g.add_argument("--n-ions", type=int, default=1 << 14)
    g.add_argument("--steps", type=int, default=6000)
    g.add_argument("--seed", type=int, default=11)
    g.add_argument("--run-seed", type=int, default=11)
    g.add_argument("--avg-steps", type=int, default=AVG_STEPS)
    e = sub.add_parser("evaluate")
    e.add_argument("--data", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--epochs", type=int, default=600)
    e.add_argument("--eval-ions", type=int, default=1 << 16)
    e.add_argument("--eval-steps", type=int, default=10000)
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(a.out, a.tag, a.total, a.start, a.count, a.n_ions, a.steps, a.seed, a.run_seed,
                 a.avg_steps)
    else:
        evaluate(a.data, a.out, a.epochs, a.eval_ions, a.eval_steps)


if __name__ == "__main__":
    main()
