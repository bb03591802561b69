"""Oracle pins: ion accelerations and the dust forces of Eqs. (1), (2), (4).

Pins used (none re-types the oracle's force expressions):
  * every force is minus the gradient of the potential energy the paper's
    Section 2 names -- screened Coulomb (Yukawa) between superparticles,
    bare Coulomb between a grain and an ion on the ion side, Yukawa on the
    dust side (Eq. 1), Coulomb between grains (Eq. 2), a uniform field --
    differentiated numerically in 40-digit arithmetic;
  * Newton's third law of the ion-ion force;
  * reciprocity of the ion-dust coupling when the screening length goes to
    infinity (the asymmetric model then becomes symmetric Coulomb).
"""
import math

import mpmath as mp
import numpy as np

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W


def _small_system(n=10, nd=2, seed=3, nu_frac=0.1, flags=0, Te=None):
    w = W.single_grain_small()
    if Te is not None:
        w = w.with_(Te=Te)
    lam0 = W.debye_length(W.ev_to_kelvin(1.0), 1e14)
    dust = [(0.3 * lam0, -0.2 * lam0, 0.1 * lam0, 5e-6, -9000 * W.QE),
            (-0.4 * lam0, 0.25 * lam0, -0.5 * lam0, 8e-6, -15000 * W.QE)][:nd]
    w = w.with_(n_ions=n, dust=dust, nu_in=nu_frac * w.wpi, flags=flags)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, 3)) * lam0
    v = rng.normal(size=(n, 3)) * 300.0
    return w, x, v


def _energy(xs, dust, q, Q, lam, E):
    k = 1 / (4 * mp.pi * mp.mpf(W.EPS0))
    U = mp.mpf(0)
    n = len(xs)
    for i in range(n):
        for j in range(i + 1, n):
            r = mp.sqrt(sum((xs[i][c] - xs[j][c]) ** 2 for c in range(3)))
            U += k * q * q * mp.exp(-r / lam) / r
    for i in range(n):
        for d, (dx, dy, dz, _, _) in enumerate(dust):
            r = mp.sqrt((xs[i][0] - dx) ** 2 + (xs[i][1] - dy) ** 2 + (xs[i][2] - dz) ** 2)
            U += k * q * Q[d] / r
        U -= q * E * xs[i][2]
    return U


def test_ion_acceleration_is_minus_gradient_of_energy():
    mp.mp.dps = 40
    w, x, v = _small_system()
    o = O.Oracle(w)
    o.set_state(x, v, np.array([d[4] for d in w.dust]), 0)
    a = o.accel_subset(np.arange(w.n_ions))
    lam = mp.mpf(W.debye_length(w.Te, w.n_inf))
    V = mp.pi * mp.mpf(w.R) ** 2 * mp.mpf(w.H)
    wgt = mp.mpf(w.n_inf) * V / w.n_ions
    q = wgt * mp.mpf(W.QE)
    m = wgt * mp.mpf(w.m_i)
    E = mp.mpf(w.m_i) * mp.mpf(w.nu_in) * w.mach * mp.sqrt(mp.mpf(W.KB) * w.Te / w.m_i) / mp.mpf(W.QE)
    Q = [mp.mpf(d[4]) for d in w.dust]
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    for i in range(w.n_ions):
        for c in range(3):
            def U_of(t, i=i, c=c):
                xx = [row[:] for row in xs]
                xx[i][c] = t
                return _energy(xx, w.dust, q, Q, lam, E)
            g = mp.diff(U_of, xs[i][c])
            expect = float(-g / m)
            assert abs(a[i, c] - expect) <= 1e-11 * np.abs(a[i]).max(), (i, c, a[i, c], expect)


def test_dust_forces_are_minus_gradient_of_energy():
    mp.mp.dps = 40
    w, x, v = _small_system(n=8)
    o = O.Oracle(w)
    Qd = np.array([d[4] for d in w.dust])
    o.set_state(x, v, Qd, 0)
    F = o.dust_forces()
    lam = mp.mpf(W.debye_length(w.Te, w.n_inf))
    V = mp.pi * mp.mpf(w.R) ** 2 * mp.mpf(w.H)
    q = mp.mpf(w.n_inf) * V / w.n_ions * mp.mpf(W.QE)
    k = 1 / (4 * mp.pi * mp.mpf(W.EPS0))
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    pos = [[mp.mpf(dd[0]), mp.mpf(dd[1]), mp.mpf(dd[2])] for dd in w.dust]
    Q = [mp.mpf(float(qq)) for qq in Qd]
    for d in range(len(w.dust)):
        for c in range(3):
            def U_orbit(t, d=d, c=c):
                p = pos[d][:]
                p[c] = t
                U = mp.mpf(0)
                for xi in xs:
                    r = mp.sqrt(sum((xi[cc] - p[cc]) ** 2 for cc in range(3)))
                    U += k * q * Q[d] * mp.exp(-r / lam) / r
                return U

            def U_dd(t, d=d, c=c):
                p = pos[d][:]
                p[c] = t
                U = mp.mpf(0)
                for pp in range(len(pos)):
                    if pp == d:
                        continue
                    r = mp.sqrt(sum((pos[pp][cc] - p[cc]) ** 2 for cc in range(3)))
                    U += k * Q[d] * Q[pp] / r
                return U
            g1 = float(-mp.diff(U_orbit, pos[d][c]))
            g2 = float(-mp.diff(U_dd, pos[d][c]))
            assert abs(F[d, 0, c] - g1) <= 1e-11 * np.abs(F[d, 0]).max()
            assert abs(F[d, 1, c] - g2) <= 1e-11 * np.abs(F[d, 1]).max()
        E = w.m_i * w.nu_in * w.mach * math.sqrt(W.KB * w.Te / w.m_i) / W.QE
        assert np.allclose(F[d, 3], [0.0, 0.0, Qd[d] * E], rtol=1e-13, atol=0)


def test_newton_third_law_ion_ion():
    w, x, v = _small_system(n=300, nd=0, nu_frac=0.0)
    w = w.with_(E_ext=0.0)
    o = O.Oracle(w)
    o.set_state(x, v, np.zeros(0), 0)
    a = o.accel_subset(np.arange(w.n_ions))
    assert np.abs(a.sum(axis=0)).max() <= 1e-13 * np.abs(a).sum()


def test_reciprocity_when_screening_length_is_infinite():
    # Te -> huge makes r_De ~ 1e7 m, so Eq. (1)'s screened force equals the
    # bare Coulomb force the ions feel: total ion-dust momentum exchange is 0.
    w, x, v = _small_system(n=64, nd=2, nu_frac=0.0, flags=W.FLAG_NO_ION_ION, Te=1e24)
    lam0 = W.debye_length(W.ev_to_kelvin(1.0), 1e14)
    w = w.with_(E_ext=0.0, R=3 * lam0, H=6 * lam0)
    o = O.Oracle(w)
    Qd = np.array([d[4] for d in w.dust])
    o.set_state(x, v, Qd, 0)
    a = o.accel_subset(np.arange(w.n_ions))
    F = o.dust_forces()
    m = o.derived["m"]
    total = m * a.sum(axis=0) + F[:, 0, :].sum(axis=0)
    scale = m * np.abs(a).sum()
    assert np.abs(total).max() <= 1e-12 * scale
