"""Pins of the oracle's confinement field (Appendix A) to results the paper and
the mathematics fix independently of the oracle's code:

* the term list of Eq. (A.3) against the printed equation (golden fixture);
* the least-squares fit recovers an exact member of the family;
* E_out = -grad P against central differences of P;
* the grid potential of Eq. (A.1) (a sum over discrete ions) against the
  continuum potential of a homogeneous cylinder, computed from a closed form
  in spherical coordinates around the node, within the Monte-Carlo error of
  the discrete sum (also computed in closed form);
* the fitted field against the closed-form on-axis field of the continuum;
* energy conservation of ions moving in the fitted field alone (sign and
  charge-to-mass factor of the kick).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def _plain(n_ions, seed=3, flags=0, dust=()):
    w = W.single_grain_small()
    return w.with_(n_ions=n_ions, dust=list(dust), seed=seed, flags=flags, nu_in=0.0,
                   E_ext=0.0, mach=0.0, charge_mode=W.CHARGE_GIVEN, n_discard=0)


def test_terms_match_equation_a3():
    rp, zp = O.confinement_terms()
    printed = GOLD["appendix_a_polynomial_terms"]["terms_r_pow_z_pow"]
    assert [[int(a), int(b)] for a, b in zip(rp, zp)] == printed
    # fifteen distinct even monomials of total degree <= 8
    assert len({(a, b) for a, b in printed}) == 15
    assert all(a % 2 == 0 and b % 2 == 0 and a + b <= 8 for a, b in printed)


def test_fit_recovers_a_member_of_the_family():
    printed = GOLD["appendix_a_polynomial_terms"]["terms_r_pow_z_pow"]
    rng = np.random.default_rng(5)
    coef = rng.normal(size=15)
    nx, nz = 24, 20
    k = np.arange(nx + 1)[:, None] / nx
    p = np.arange(nz + 1)[None, :] / nz
    grid = sum(c * k ** a * p ** b for c, (a, b) in zip(coef, printed))
    alpha = O.fit_polynomial(grid, nx, nz)
    assert np.allclose(alpha, coef, rtol=0, atol=1e-9)
    # the fit is an orthogonal projection: it moves a noisy grid by no more than the noise
    noise = 1e-3 * rng.normal(size=grid.shape)
    alpha2 = O.fit_polynomial(grid + noise, nx, nz)
    fit = sum(c * k ** a * p ** b for c, (a, b) in zip(alpha2, printed))
    assert np.linalg.norm(fit - grid - noise) <= np.linalg.norm(noise)


def test_field_is_minus_gradient_of_p():
    w = _plain(64)
    o = O.Oracle(w)
    rng = np.random.default_rng(1)
    alpha = rng.normal(size=15) * 1e-2
    o.set_confinement(alpha)
    lam = o.derived["lam"]
    x = np.stack([rng.uniform(-0.6, 0.6, 20) * w.R, rng.uniform(-0.6, 0.6, 20) * w.R,
                  rng.uniform(-0.45, 0.45, 20) * w.H], axis=1)
    _, E = o.confinement_eval(x)
    h = 1e-4 * lam
    for c in range(3):
        dx = np.zeros(3)
        dx[c] = h
        Pp, _ = o.confinement_eval(x + dx)
        Pm, _ = o.confinement_eval(x - dx)
        fd = -(Pp - Pm) / (2 * h)
        assert np.allclose(E[:, c], fd, rtol=1e-6, atol=1e-8 * np.abs(E).max())
    # the printed polynomial in unscaled r, z: alpha_m(unscaled) r^a z^b
    printed = GOLD["appendix_a_polynomial_terms"]["terms_r_pow_z_pow"]
    P, _ = o.confinement_eval(x)
    r = np.hypot(x[:, 0], x[:, 1])
    z = x[:, 2]
    rs, zs = w.R, 0.5 * w.H
    P2 = sum((c / rs ** a / zs ** b) * r ** a * z ** b for c, (a, b) in zip(alpha, printed))
    assert np.allclose(P, P2, rtol=1e-12, atol=1e-14)


# --- continuum potential of a homogeneous cylinder -------------------------
def _sphere_moments(node, R, H, lam, n_mu=240, n_phi=240):
    """(I1, I2) = (int e^{-s/lam}/s dV, int e^{-2s/lam}/s^2 dV) over the
    cylinder, in spherical coordinates centred on the node: the radial
    integrals are elementary, leaving an integral over directions of the
    distance S(omega) from the node to the boundary."""
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    MU, PHI = np.meshgrid(mu, phi, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    ox, oy, oz = st * np.cos(PHI), st * np.sin(PHI), MU
    px, py, pz = node
    a = ox ** 2 + oy ** 2
    b = px * ox + py * oy
    c = px * px + py * py - R * R
    with np.errstate(divide="ignore", invalid="ignore"):
        s_side = np.where(a > 0, (-b + np.sqrt(np.maximum(b * b - a * c, 0.0))) / a, np.inf)
        s_cap = np.where(oz > 0, (0.5 * H - pz) / oz, np.where(oz < 0, (-0.5 * H - pz) / oz, np.inf))
    S = np.maximum(np.minimum(s_side, s_cap), 0.0) / lam
    dW = wmu[:, None] * (2 * math.pi / n_phi)
    I1 = lam ** 2 * np.sum(dW * (1 - (1 + S) * np.exp(-S)))
    I2 = 0.5 * lam * np.sum(dW * (1 - np.exp(-2 * S)))
    return I1, I2


def test_grid_matches_continuum_within_sampling_error():
    N = 400_000
    w = _plain(N, seed=11)
    o = O.Oracle(w)
    d = o.derived
    lam, V, q = d["lam"], d["V"], d["q"]
    nx, nz = 4, 4
    grid = o.confinement_grid(nx, nz)
    phi0 = W.KB * w.Te / W.QE            # screened potential of the infinite background
    k4 = 1.0 / (4 * math.pi * W.EPS0)
    zs = []
    for kk in range(nx + 1):
        for pp in range(nz + 1):
            node = (w.R * kk / nx, 0.0, 0.5 * w.H * pp / nz)
            I1, I2 = _sphere_moments(node, w.R, w.H, lam)
            cont = phi0 - k4 * w.n_inf * W.QE * I1
            se = k4 * q * math.sqrt(N * max(I2 / V - (I1 / V) ** 2, 0.0))
            zs.append((grid[kk, pp] - cont) / se)
            # the sampling error is small against the potential drop it measures
            assert se < 0.02 * k4 * w.n_inf * W.QE * I1
    zs = np.array(zs)
    assert np.abs(zs).max() < 5.0, zs
    # and the deviations look like noise, not a bias
    assert abs(zs.mean()) < 5.0 / math.sqrt(len(zs)) + 1.0


def _axis_field_continuum(z0, w, lam):
    """E_z of Phi0 - Phi_cyl on the axis: the ring integral over the radius is
    elementary, 2 pi lam (e^{-|D|/lam} - e^{-sqrt(R^2+D^2)/lam}), and its
    integral over the height differentiates to the two end values."""
    f = lambda D: math.exp(-abs(D) / lam) - math.exp(-math.hypot(w.R, D) / lam)
    a, b = -0.5 * w.H - z0, 0.5 * w.H - z0
    return w.n_inf * W.QE / (4 * math.pi * W.EPS0) * 2 * math.pi * lam * (f(a) - f(b))


def test_fitted_field_is_restoring_and_matches_continuum():
    N = 400_000
    w = _plain(N, seed=12, flags=W.FLAG_CONFINEMENT)
    o = O.Oracle(w)
    lam = o.derived["lam"]
    assert o.conf_alpha is not None and o.conf_grid.shape == (O.CONF_NX + 1, O.CONF_NZ + 1)
    # fit quality: residual small against the variation of the grid
    rp, zp = O.confinement_terms()
    pts = np.array([[w.R * k / O.CONF_NX, 0.0, 0.5 * w.H * p / O.CONF_NZ]
                    for k in range(O.CONF_NX + 1) for p in range(O.CONF_NZ + 1)])
    P, _ = o.confinement_eval(pts)
    res = P - o.conf_grid.ravel()
    span = o.conf_grid.max() - o.conf_grid.min()
    assert np.sqrt(np.mean(res ** 2)) < 0.02 * span
    # on the axis: E_z(0) = 0, E_z < 0 above the midplane, close to the continuum
    zz = np.array([0.0, 0.25, 0.5, 0.75]) * 0.5 * w.H
    _, E = o.confinement_eval(np.stack([0 * zz, 0 * zz, zz], axis=1))
    assert E[0, 2] == 0.0 and np.all(E[1:, 2] < 0)
    assert np.allclose(E[:, :2], 0.0)
    for i in (2, 3):
        ref = _axis_field_continuum(zz[i], w, lam)
        assert ref < 0
        assert abs(E[i, 2] - ref) <= 0.15 * abs(ref), (zz[i] / lam, E[i, 2], ref)
    # radial: pointing inward in the midplane
    xr = np.array([0.3, 0.6, 0.9]) * w.R
    _, Er = o.confinement_eval(np.stack([xr, 0 * xr, 0 * xr], axis=1))
    assert np.all(Er[:, 0] < 0) and np.all(np.diff(Er[:, 0]) < 0)


def test_ions_conserve_energy_in_the_field():
    """Test particles (no ion-ion force, no grain, no collisions, no drive)
    moving in E_out alone keep (1/2) m v^2 + e P(x) to leapfrog accuracy."""
    w = _plain(20_000, seed=4, flags=W.FLAG_CONFINEMENT | W.FLAG_NO_ION_ION)
    o = O.Oracle(w)
    mi = w.m_i
    x0, v_prev, _, _ = o.get_state()
    hist = []
    steps = 200
    keep = np.ones(o.N, dtype=bool)
    for n in range(steps):
        o.step()
        ls = o.last_step()
        keep &= ls["ev"] == O.EV_NONE
        x, v, _, _ = o.get_state()
        hist.append((x, v))
    # energy at integer steps: positions x^n with v^n = (v^{n-1/2} + v^{n+1/2}) / 2
    def energy(n):
        xn = hist[n - 1][0]
        vn = 0.5 * (hist[n - 1][1] + hist[n][1])
        P, _ = o.confinement_eval(xn)
        return 0.5 * mi * np.sum(vn ** 2, axis=1) + W.QE * P, W.QE * P
    e1, p1 = energy(1)
    e2, p2 = energy(steps - 1)
    dpe = np.abs(p2 - p1)[keep]
    de = np.abs(e2 - e1)[keep]
    sel = dpe > np.percentile(dpe, 90)
    assert keep.sum() > 0.9 * o.N and sel.sum() > 100
    # the potential energy changed a lot for these ions; the total did not
    assert np.median(de[sel] / dpe[sel]) < 1e-3
    assert np.percentile(de[sel] / dpe[sel], 99) < 5e-3


def test_dust_force_carries_q_e_out():
    dust = [(0.0, 0.0, 1.0 * W.single_grain_small().lam, 5e-6, -5e-15)]
    w = _plain(3000, seed=9, flags=W.FLAG_CONFINEMENT, dust=dust)
    o = O.Oracle(w)
    F_on = o.dust_forces()
    alpha = o.conf_alpha
    o.set_confinement(alpha, on=False)
    F_off = o.dust_forces()
    o.set_confinement(alpha, on=True)
    _, E = o.confinement_eval(np.array(dust[0][:3]))
    Q = o.get_state()[2][0]
    assert np.allclose(F_on[0, 0] - F_off[0, 0], Q * E[0], rtol=1e-12, atol=1e-30)
    assert E[0, 2] < 0 and abs(E[0, 0]) < 1e-12 * abs(E[0, 2]) + 1e-300
    assert np.array_equal(F_on[0, 1:], F_off[0, 1:])
