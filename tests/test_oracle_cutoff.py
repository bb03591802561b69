"""Pins of the oracle's ion-ion cutoff with a switching function (Section 4,
performance with cutoff; the switch itself is a reading, see the oracle).

* the switched force is minus the gradient of the switched energy,
  differentiated numerically in 40-digit arithmetic, with pairs in all three
  regimes (unswitched, switching, beyond the cutoff);
* the force of a pair is continuous at both ends of the switching interval
  and exactly zero beyond the cutoff;
* a cutoff beyond every pair distance reproduces the plain sum;
* Newton's third law holds for the switched interaction.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W

LAM0 = W.debye_length(W.ev_to_kelvin(1.0), 1e14)


def _system(n, seed=4, dust=True):
    w = W.single_grain_small()
    d = [(0.3 * LAM0, -0.2 * LAM0, 0.1 * LAM0, 5e-6, -9000 * W.QE)] if dust else []
    w = w.with_(n_ions=n, dust=d, nu_in=0.0, E_ext=0.0)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, 3)) * LAM0
    return w, x


def _switched_energy(xs, q, lam, r_sw, r_cut, dust, Q):
    k = 1 / (4 * mp.pi * mp.mpf(W.EPS0))
    U = mp.mpf(0)
    for i in range(len(xs)):
        for j in range(i + 1, len(xs)):
            r = mp.sqrt(sum((xs[i][c] - xs[j][c]) ** 2 for c in range(3)))
            if r >= r_cut:
                continue
            S = mp.mpf(1)
            if r > r_sw:
                t = (r - r_sw) / (r_cut - r_sw)
                S = 1 - 6 * t ** 5 + 15 * t ** 4 - 10 * t ** 3
            U += k * q * q * mp.exp(-r / lam) / r * S
        for d, (dx, dy, dz, _, _) in enumerate(dust):
            r = mp.sqrt((xs[i][0] - dx) ** 2 + (xs[i][1] - dy) ** 2 + (xs[i][2] - dz) ** 2)
            U += k * q * Q[d] / r
    return U


def test_switched_force_is_minus_gradient():
    mp.mp.dps = 40
    n = 9
    w, x = _system(n)
    r_sw, r_cut = 0.6 * LAM0, 1.2 * LAM0
    o = O.Oracle(w)
    o.set_state(x, np.zeros_like(x), np.array([w.dust[0][4]]), 0)
    o.set_cutoff(r_sw, r_cut)
    a = o.accel_subset(np.arange(n))
    # the configuration has pairs in every regime
    dist = np.linalg.norm(x[:, None] - x[None], axis=2)[np.triu_indices(n, 1)]
    assert (dist < r_sw).any() and ((dist > r_sw) & (dist < r_cut)).any() and (dist > r_cut).any()
    lam = mp.mpf(W.debye_length(w.Te, w.n_inf))
    V = mp.pi * mp.mpf(w.R) ** 2 * mp.mpf(w.H)
    wgt = mp.mpf(w.n_inf) * V / n
    q, m = wgt * mp.mpf(W.QE), wgt * mp.mpf(w.m_i)
    Q = [mp.mpf(w.dust[0][4])]
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    for i in range(n):
        for c in range(3):
            def U_of(t, i=i, c=c):
                xx = [row[:] for row in xs]
                xx[i][c] = t
                return _switched_energy(xx, q, lam, mp.mpf(r_sw), mp.mpf(r_cut), w.dust, Q)
            expect = float(-mp.diff(U_of, xs[i][c]) / m)
            assert abs(a[i, c] - expect) <= 1e-11 * np.abs(a[i]).max(), (i, c, a[i, c], expect)


def _pair_accel(r, r_sw, r_cut):
    w = W.single_grain_small().with_(n_ions=2, dust=[], nu_in=0.0, E_ext=0.0)
    o = O.Oracle(w, init=False)
    x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    o.set_state(x, np.zeros_like(x), np.zeros(0), 0)
    o.set_cutoff(r_sw, r_cut)
    return o.accel_subset(np.array([0]))[0, 0]


def test_pair_force_is_continuous_and_vanishes_beyond_the_cutoff():
    r_sw, r_cut = 2.0 * LAM0, 3.0 * LAM0
    eps = 1e-7 * LAM0
    a_in = _pair_accel(r_sw - eps, r_sw, r_cut)
    a_out = _pair_accel(r_sw + eps, r_sw, r_cut)
    assert a_in == pytest.approx(a_out, rel=1e-5)
    a_mid = _pair_accel(0.5 * (r_sw + r_cut), r_sw, r_cut)
    assert abs(_pair_accel(r_cut - eps, r_sw, r_cut)) < 1e-9 * abs(a_mid)
    assert _pair_accel(r_cut, r_sw, r_cut) == 0.0
    assert _pair_accel(1.5 * r_cut, r_sw, r_cut) == 0.0
    # repulsive between like charges wherever it is not zero
    assert a_mid < 0 and a_in < 0


def test_far_cutoff_reproduces_plain_sum():
    w, x = _system(40, seed=7)
    o = O.Oracle(w)
    o.set_state(x, np.zeros_like(x), np.array([w.dust[0][4]]), 0)
    plain = o.accel_subset(np.arange(40))
    o.set_cutoff(50 * LAM0, 60 * LAM0)
    far = o.accel_subset(np.arange(40))
    assert np.allclose(far, plain, rtol=1e-12, atol=1e-14 * np.abs(plain).max())


def test_third_law_with_switching():
    w, x = _system(30, seed=2, dust=False)
    o = O.Oracle(w)
    o.set_state(x, np.zeros_like(x), np.zeros(0), 0)
    o.set_cutoff(0.5 * LAM0, 0.9 * LAM0)
    a = o.accel_subset(np.arange(30))
    assert np.abs(a.sum(axis=0)).max() <= 1e-13 * np.abs(a).sum()
