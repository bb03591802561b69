"""Helpers of the GPU parity tests: moving a GPU state into the oracle and
comparing one shadowed step (GPU state loaded into the oracle, one step on
both).  Tolerances follow the per-step floating-point bar (relative 1e-5 on
forces) and exact agreement of integer decisions.  An absorption or exit
decision may differ only for an ion whose drift segment passes within the
rounding band of a grain surface or the wall: the GPU forms the end point
x + dt v in the state's precision (FP32 by default) and the oracle in FP64,
so the band is a few units in the last place of the end point and of the
step, plus the FP64 cancellation of the GPU's closest-approach test and the
drift of the acceleration difference over dt^2.  At most MAX_MISMATCH such
ions are tolerated per step."""
from __future__ import annotations

import math
import sys

import numpy as np

from oracle import oracle as O

EPS32 = 2.0 ** -23
EPS64 = 2.0 ** -52
MAX_MISMATCH = 3


def rounding_band(w, precision, x1_si, step_si, da_si):
    """Per-ion width (m) within which the GPU's and the oracle's absorption
    and exit decisions may differ: 4 ulp of the end point's and the step's
    largest component in the state's precision, 4 FP64 ulp of the
    closest-approach test's |s|^2 / a (with |s| bounded by the domain), and
    twice dt^2 times the acceleration difference."""
    eps = EPS32 if precision == 0 else EPS64
    lam = w.lam
    span = math.hypot(w.R, 0.5 * w.H) + max(math.hypot(g[0], math.hypot(g[1], g[2])) for g in w.dust) \
        if w.dust else 0.0
    amin = min(g[3] for g in w.dust) if w.dust else lam
    ulps = 4 * eps * (np.abs(x1_si).max(axis=1) + np.abs(step_si).max(axis=1))
    return ulps + 4 * EPS64 * span * span / amin + 2 * w.dt ** 2 * da_si


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_oracle(sysm, orc):
    """Copy the GPU state into the oracle (dimensionless -> SI with the
    oracle's own units).  Returns the dimensionless GPU state."""
    x, v, q, step = sysm.get_state()
    lam, cs = orc.derived["lam"], orc.derived["cs"]
    orc.set_state(x.T.astype(np.float64) * lam, v.T.astype(np.float64) * cs, q, step)
    return x, v, q, step


def accel_errors(a_gpu_si, a_orc):
    """(relative L2 error, 99.9th percentile of per-ion error normalised by
    max(|a_i|, a_rms), max of the same)."""
    d = np.linalg.norm(a_gpu_si - a_orc, axis=1)
    mag = np.linalg.norm(a_orc, axis=1)
    rms = math.sqrt(np.mean(mag ** 2))
    rel = d / np.maximum(mag, rms)
    l2 = np.linalg.norm(a_gpu_si - a_orc) / np.linalg.norm(a_orc)
    return l2, float(np.percentile(rel, 99.9)), float(rel.max())


def oracle_event_codes(ev_orc):
    """Oracle event codes -> the GPU's byte codes (without the collision bit)."""
    out = np.zeros(len(ev_orc), dtype=np.int64)
    out[ev_orc == O.EV_EXITED] = 1
    absd = ev_orc >= 0
    out[absd] = 2 + ev_orc[absd]
    return out


def ambiguous_ions(w, x0_si, x1_si, band):
    """Ions whose drift segment passes within `band` (m) of a grain surface or
    whose end point lies within `band` of the wall."""
    amb = np.zeros(len(x0_si), dtype=bool)
    D = x1_si - x0_si
    DD = np.einsum("ij,ij->i", D, D)
    for (gx, gy, gz, a, _) in w.dust:
        s = x0_si - np.array([gx, gy, gz])
        sD = np.einsum("ij,ij->i", s, D)
        t = np.clip(np.where(DD > 0, -sD / np.where(DD > 0, DD, 1), 0.0), 0.0, 1.0)
        c = s + t[:, None] * D
        dist = np.linalg.norm(c, axis=1)
        amb |= np.abs(dist - a) <= band
        # the end point just outside with the segment's own closest point inside
        amb |= np.abs(np.linalg.norm(x1_si - np.array([gx, gy, gz]), axis=1) - a) <= band
    rr = np.sqrt(x1_si[:, 0] ** 2 + x1_si[:, 1] ** 2)
    amb |= np.abs(rr - w.R) <= band
    amb |= np.abs(np.abs(x1_si[:, 2]) - 0.5 * w.H) <= band
    return amb


def shadow_step(sysm, orc, w, check_state=True, acc_tol=1e-5, force_tol=1e-5):
    """Runs one step on both from the GPU's current state and checks parity.
    Returns a dict of measured errors and event counts."""
    lam, cs, wpi = orc.derived["lam"], orc.derived["cs"], orc.derived["wpi"]
    x0, v0, q0, n0 = to_oracle(sysm, orc)
    sysm.step(1)
    sysm.sync()
    orc.step()
    ls = orc.last_step()
    out = {}
    # accelerations at x^n
    a_gpu = sysm.accelerations().T.astype(np.float64) * lam * wpi * wpi
    l2, p999, pmax = accel_errors(a_gpu, ls["a"])
    out.update(acc_l2=l2, acc_p999=p999, acc_max=pmax)
    assert l2 <= acc_tol, out
    assert p999 <= acc_tol, out
    # events
    ev, nabs, nexit, ncoll = sysm.events()
    gpu_codes = (ev & 0x7F).astype(np.int64)
    gpu_coll = (ev & 0x80) != 0
    assert (gpu_coll == (ls["hit"] != 0)).all(), "collision decisions differ"
    orc_codes = oracle_event_codes(ls["ev"])
    mism = np.nonzero(gpu_codes != orc_codes)[0]
    x0_si = x0.T.astype(np.float64) * lam
    # oracle end points before reinjection are x0 + dt * v_hat; rebuild them
    v_hat = v0.T.astype(np.float64) * cs + w.dt * ls["a"]
    if len(mism):
        x1_si = x0_si + w.dt * v_hat
        da_si = np.linalg.norm(a_gpu - ls["a"], axis=1)
        band = rounding_band(w, sysm.precision, x1_si, w.dt * v_hat, da_si)
        amb = ambiguous_ions(w, x0_si, x1_si, band=band)
        bad = [int(i) for i in mism if not amb[i]]
        assert not bad, f"event sets differ at non-ambiguous ions {bad[:10]} (bands {band[bad[:3]]})"
        assert len(mism) <= MAX_MISMATCH, f"{len(mism)} ambiguous event mismatches in one step"
    out["n_ambiguous_mismatch"] = int(len(mism))
    out["n_abs"] = nabs.tolist()
    out["n_exit"] = nexit
    out["n_coll"] = ncoll
    if not len(mism):
        assert list(nabs) == list(ls["nabs"]) and nexit == ls["nexit"] and ncoll == ls["ncoll"]
    # dust forces of this step (SI)
    F = sysm.forces(0)
    for d in range(len(w.dust)):
        for p in (0, 1, 3):
            ref = ls["F"][d, p]
            err = np.linalg.norm(F[d, p] - ref)
            scale = np.linalg.norm(ref)
            assert err <= force_tol * scale + 1e-300, (d, p, F[d, p], ref)
        if not len(mism):
            ref = ls["F"][d, 2]
            assert np.linalg.norm(F[d, 2] - ref) <= 1e-5 * np.linalg.norm(ref) + 1e-300, (F[d, 2], ref)
    # charges
    q_gpu, _ = sysm.charges()
    _, _, q_orc, _ = orc.get_state()
    if not len(mism):
        assert np.allclose(q_gpu, q_orc, rtol=1e-12, atol=1e-30), (q_gpu, q_orc)
    out["q"] = q_gpu.tolist()
    if check_state:
        x1, v1, _, n1 = sysm.get_state()
        assert n1 == n0 + 1
        xo, vo, _, no = orc.get_state()
        assert no == n0 + 1
        xo_t = xo.T / lam
        vo_t = vo.T / cs
        ok = np.ones(sysm.N, dtype=bool)
        ok[mism] = False
        dt_t = w.dt * wpi
        da = np.linalg.norm(a_gpu - ls["a"], axis=1) / (lam * wpi * wpi)
        eps = EPS32 if sysm.precision == 0 else 2.0 ** -52
        tol_v = 4 * eps * np.maximum(np.abs(vo_t), 0.2) + 1.01 * dt_t * da[None, :] + 1e-12
        tol_x = 4 * eps * np.maximum(np.abs(xo_t), 1.0) + dt_t * tol_v
        dv = np.abs(v1.astype(np.float64) - vo_t)
        dx = np.abs(x1.astype(np.float64) - xo_t)
        bad_v = np.nonzero(((dv > tol_v) & ok[None, :]).any(axis=0))[0]
        bad_x = np.nonzero(((dx > tol_x) & ok[None, :]).any(axis=0))[0]
        assert len(bad_v) == 0, ("velocity", bad_v[:10], dv[:, bad_v[:3]], tol_v[:, bad_v[:3]])
        assert len(bad_x) == 0, ("position", bad_x[:10], dx[:, bad_x[:3]], tol_x[:, bad_x[:3]])
    return out
