"""Oracle pins: leapfrog push, momentum balance, charge-exchange collisions.

  * a single ion in a uniform field follows the exact solution of the
    staggered leapfrog recurrence (x^n = x0 + n dt v0 + a dt^2 n(n+1)/2);
  * with collisions, walls and dust out of play, the internal ion-ion forces
    conserve total momentum to rounding;
  * collision decisions are exactly the draws w0 < floor(P 2^64) of numpy's
    independent Philox, with P = 1 - exp(-nu dt) (Section 2: constant
    collision frequency);
  * the driven, colliding steady state has the mean drift and variance of a
    geometric number of kicks since the last thermalising collision.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.test_oracle_rng import numpy_block


def _far_walls(w):
    return w.with_(R=10.0, H=20.0)


def test_leapfrog_uniform_field_exact():
    w = _far_walls(W.single_grain_small()).with_(n_ions=1, dust=[], nu_in=0.0, E_ext=250.0)
    o = O.Oracle(w)
    x0 = np.array([[1e-4, -2e-4, 3e-4]])
    v0 = np.array([[120.0, -40.0, 900.0]])
    o.set_state(x0, v0, np.zeros(0), 0)
    acc = W.QE * 250.0 / w.m_i
    n = 400
    o.run(n)
    x, v, _, step = o.get_state()
    assert step == n
    expect = x0.copy()
    expect += n * w.dt * v0
    expect[0, 2] += acc * w.dt ** 2 * n * (n + 1) / 2
    assert np.allclose(x, expect, rtol=1e-12, atol=1e-15)
    assert np.allclose(v[0], v0[0] + np.array([0, 0, n * acc * w.dt]), rtol=1e-12)


def test_total_momentum_conserved_by_internal_forces():
    # standard domain (R = 3, H = 6 Debye lengths), ions started in its core
    w = W.single_grain_small().with_(n_ions=300, dust=[], nu_in=0.0, E_ext=0.0)
    o = O.Oracle(w)
    lam = w.lam
    x, v = W.uniform_cylinder_state(w.with_(R=lam, H=2 * lam), 300, seed=4)
    o.set_state(x, v, np.zeros(0), 0)
    p0 = v.sum(axis=0)
    o.run(30)
    _, v1, _, _ = o.get_state()
    ls = o.last_step()
    assert ls["nexit"] == 0
    scale = np.abs(v1).sum()
    assert np.abs(v1.sum(axis=0) - p0).max() <= 1e-13 * scale
    # and the forces are not trivially zero
    assert np.abs(v1 - v).max() > 1e-3 * np.abs(v).max()


def test_collision_decisions_are_philox_threshold_draws():
    w = _far_walls(W.single_grain_small()).with_(n_ions=5000, dust=[], flags=W.FLAG_NO_ION_ION)
    o = O.Oracle(w)
    o.run(3)   # decisions of step 2 (counter step word = 2)
    hit = o.last_step()["hit"]
    P = -math.expm1(-w.nu_in * w.dt)
    T = int(P * 2.0**64)
    expect = np.array([numpy_block([i, 2, 2, 0], [w.seed, 0])[0] < T for i in range(w.n_ions)])
    assert (hit.astype(bool) == expect).all()
    assert 0 < hit.sum() < 30


def test_driven_collisional_steady_state():
    w = _far_walls(W.single_grain_small()).with_(n_ions=20000, dust=[], flags=W.FLAG_NO_ION_ION)
    o = O.Oracle(w)
    cs = math.sqrt(W.KB * w.Te / w.m_i)
    u = w.mach * cs
    sig = math.sqrt(W.KB * w.Ti / w.m_i)
    E = w.m_i * w.nu_in * u / W.QE
    dv = W.QE * E / w.m_i * w.dt
    P = -math.expm1(-w.nu_in * w.dt)
    mean = dv * (1 - P) / P
    var = sig ** 2 + dv ** 2 * (1 - P) / P ** 2
    o.run(4000)
    samples = []
    ncoll = 0
    for k in range(3):
        o.run(1000)
        samples.append(o.get_state()[1][:, 2].copy())
    vz = np.concatenate(samples)
    se = math.sqrt(var / len(vz)) * 2.0     # snapshots 1000 steps apart are mildly correlated
    assert abs(vz.mean() - mean) < 5 * se, (vz.mean() / u, mean / u)
    assert abs(vz.var() / var - 1.0) < 0.06
    # collision count of one step is Binomial(N, P)
    tot = 0
    for k in range(200):
        o.step()
        tot += o.last_step()["ncoll"]
    lam_ = 200 * w.n_ions * P
    assert abs(tot - lam_) < 5 * math.sqrt(lam_)
