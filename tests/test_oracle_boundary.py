"""Oracle pins: the open boundary of Appendix B.

  * face probabilities at Mach 0 are the area ratios (isotropic flow);
  * face inflows agree with direct numerical quadrature of Eqs. (B.2)-(B.4);
  * the flux-weighted inverse CDF reduces to the Rayleigh inverse at zero
    drift and reproduces the quadrature CDF of Eqs. (B.8)-(B.9) (KS test);
  * the whole boundary scheme is stationary: free-streaming test particles
    stay uniform in the cylinder with the shifted Maxwellian N((0,0,u), s^2 I)
    (this fails if the side injection drops its tangential thermal part),
    and the exit rate equals the analytic inflow.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W


def _pdf(v, u, s):
    return math.exp(-0.5 * ((v - u) / s) ** 2) / (s * math.sqrt(2 * math.pi))


def test_face_probabilities_mach0_are_area_ratios():
    w = W.single_grain_small().with_(mach=0.0)
    o = O.Oracle(w, init=False)
    d = o.derived
    J = d["Jb"] + d["Jt"] + d["Js"]
    # R = 3, H = 6: bottom/top disks 9 pi each, side 36 pi
    assert abs(d["Jb"] / J - 1 / 6) < 1e-15
    assert abs(d["Jt"] / J - 1 / 6) < 1e-15
    assert abs(d["Js"] / J - 2 / 3) < 1e-15
    assert abs(o.Tb / 2.0**64 - 1 / 6) < 1e-15
    assert abs(o.Tbt / 2.0**64 - 1 / 3) < 1e-15


@pytest.mark.parametrize("mach", [0.0, 0.5, 1.0, 2.0])
def test_face_inflows_match_quadrature(mach):
    w = W.single_grain_small().with_(mach=mach)
    o = O.Oracle(w, init=False)
    d = o.derived
    u, s = d["u"], d["sig"]
    jb = integrate.quad(lambda v: v * _pdf(v, u, s), 0, u + 40 * s, epsabs=0, epsrel=1e-12)[0]
    jt = integrate.quad(lambda v: -v * _pdf(v, u, s), min(-40 * s, u - 40 * s), 0,
                        epsabs=0, epsrel=1e-12)[0]
    js = integrate.quad(lambda v: v * _pdf(v, 0.0, s), 0, 40 * s, epsabs=0, epsrel=1e-12)[0]
    area = math.pi * w.R ** 2
    assert d["Jb"] == pytest.approx(area * jb, rel=1e-9)
    if jt > 1e-300:
        assert d["Jt"] == pytest.approx(area * jt, rel=1e-6)
    assert d["Js"] == pytest.approx(2 * math.pi * w.R * w.H * js, rel=1e-9)


def test_inverse_cdf_zero_drift_is_rayleigh():
    s = 269.18
    for uu in np.linspace(1e-6, 1 - 1e-6, 101):
        v = O.flux_inverse(uu, 0.0, s)
        assert abs(v - s * math.sqrt(-2 * math.log(uu))) <= 2e-13 * s


@pytest.mark.parametrize("ubar", [1554.0, -1554.0, 400.0, -150.0])
def test_inverse_cdf_matches_quadrature_distribution(ubar):
    s = 269.18
    rng = np.random.default_rng(int(abs(ubar)))
    uu = rng.uniform(0, 1, size=3000)
    vs = np.array([O.flux_inverse(x, ubar, s) for x in uu])
    hi = max(ubar, 0) + 40 * s
    total = integrate.quad(lambda v: v * _pdf(v, ubar, s), 0, hi, epsabs=0, epsrel=1e-12)[0]

    def cdf(vv):
        return np.array([integrate.quad(lambda v: v * _pdf(v, ubar, s), 0, x,
                                        epsabs=0, epsrel=1e-10)[0] / total for x in np.atleast_1d(vv)])
    # KS against the quadrature CDF
    assert stats.kstest(vs, cdf).pvalue > 1e-4
    # and pointwise: G(v(uu)) = 1 - uu
    for x, v in zip(uu[:50], vs[:50]):
        assert abs(cdf(v)[0] - (1 - x)) < 1e-7


def _run_free_streaming(flags, n=20000, steps=2500):
    w = W.single_grain_small().with_(n_ions=n, dust=[], nu_in=0.0, E_ext=0.0,
                                     flags=W.FLAG_NO_ION_ION | flags)
    o = O.Oracle(w)
    nexit = 0
    for k in range(steps):
        o.step()
        nexit += o.last_step()["nexit"]
    x, v, _, _ = o.get_state()
    return w, o, x, v, nexit / steps


def test_boundary_scheme_is_stationary():
    w, o, x, v, exit_rate = _run_free_streaming(0)
    d = o.derived
    u, s = d["u"], d["sig"]
    r2 = (x[:, 0] ** 2 + x[:, 1] ** 2) / w.R ** 2
    zz = x[:, 2] / w.H + 0.5
    assert stats.kstest(r2, "uniform").pvalue > 1e-3
    assert stats.kstest(zz, "uniform").pvalue > 1e-3
    assert stats.kstest(v[:, 0] / s, "norm").pvalue > 1e-3
    assert stats.kstest(v[:, 1] / s, "norm").pvalue > 1e-3
    assert stats.kstest((v[:, 2] - u) / s, "norm").pvalue > 1e-3
    # radial velocity near the side wall is still isotropic-thermal
    near = r2 > 0.9
    vr = (x[near, 0] * v[near, 0] + x[near, 1] * v[near, 1]) / np.sqrt(r2[near] * w.R ** 2)
    vt = (x[near, 0] * v[near, 1] - x[near, 1] * v[near, 0]) / np.sqrt(r2[near] * w.R ** 2)
    assert abs(vt.std() / s - 1) < 0.06
    # exit (= injection) rate equals the analytic inflow n_sp * (Jb + Jt + Js) * dt
    inflow = (w.n_ions / (math.pi * w.R ** 2 * w.H)) * (d["Jb"] + d["Jt"] + d["Js"]) * w.dt
    assert abs(exit_rate / inflow - 1) < 0.02


def test_literal_side_injection_is_not_stationary():
    # Reading of Eqs. (B.10)-(B.11): without the tangential thermal component
    # the side-injected ions carry no tangential velocity, which cools the
    # tangential distribution near the wall.
    w, o, x, v, _ = _run_free_streaming(W.FLAG_LITERAL_SIDE, n=20000, steps=1500)
    s = o.derived["sig"]
    r2 = (x[:, 0] ** 2 + x[:, 1] ** 2) / w.R ** 2
    near = r2 > 0.9
    vt = (x[near, 0] * v[near, 1] - x[near, 1] * v[near, 0]) / np.sqrt(r2[near] * w.R ** 2)
    assert vt.std() / s < 0.9
