"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module only *describes inputs*: the paper's parameter sets written out in
SI units and seeded generators of particle states.  It holds none of the
method's arithmetic (no forces, pushes, collisions, charging or reinjection),
so that the HIP library and the CPU oracle can both be fed from it without
sharing any computation.

Inputs follow the paper's problem statement (Section 3: plasma, simulation and
dust parameter objects in SI units).  Geometry given "in Debye lengths" and
times "in 1/omega_pi" are converted with the textbook definitions of the
electron Debye length and the ion plasma frequency.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

# CODATA 2018
QE = 1.602176634e-19
KB = 1.380649e-23
EPS0 = 8.8541878128e-12
M_ARGON = 6.6335209e-26          # kg, the ion mass of the paper's Table 2

CHARGE_GIVEN, CHARGE_OML, CHARGE_CONSISTENT = 0, 1, 2
FLAG_LITERAL_SIDE = 1            # side injection: radial + v_z only
FLAG_NO_ION_ION = 2              # test-particle mode (ion-ion force off)
FLAG_CONFINEMENT = 4             # confinement field of the outer plasma (Appendix A)
FLAG_FIELD_DRIVEN = 8            # field-driven collisional flow: injection from its stationary distribution


def ev_to_kelvin(t_ev: float) -> float:
    return t_ev * QE / KB


def debye_length(te_k: float, n: float) -> float:
    """Electron Debye length sqrt(eps0 kB Te / (n e^2))."""
    return math.sqrt(EPS0 * KB * te_k / (n * QE * QE))


def ion_plasma_frequency(n: float, mi: float) -> float:
    """Ion plasma frequency sqrt(n e^2 / (eps0 mi))."""
    return math.sqrt(n * QE * QE / (EPS0 * mi))


@dataclass
class Workload:
    """One dust system, all quantities SI (K, m^-3, kg, m, s, C)."""
    Te: float
    Ti: float
    n_inf: float
    m_i: float
    mach: float
    nu_in: float
    E_ext: float                 # NaN: derived from the drift (m_i nu u / e)
    R: float
    H: float
    dt: float
    n_ions: int
    n_steps: int
    n_discard: int
    seed: int
    system_id: int = 0
    charge_mode: int = CHARGE_CONSISTENT
    flags: int = 0
    dust: List[Tuple[float, float, float, float, float]] = field(default_factory=list)
    name: str = ""

    @property
    def lam(self) -> float:
        return debye_length(self.Te, self.n_inf)

    @property
    def wpi(self) -> float:
        return ion_plasma_frequency(self.n_inf, self.m_i)

    def plasma7(self) -> List[float]:
        return [self.Te, self.Ti, self.n_inf, self.m_i, self.mach, self.nu_in, self.E_ext]

    def geom3(self) -> List[float]:
        return [self.R, self.H, self.dt]

    def dust_array(self) -> np.ndarray:
        return np.asarray(self.dust, dtype=np.float64).reshape(-1, 5)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The plasma of the benchmark configurations: Te = 1 eV, Ti = 0.03 eV,
# n = 1e14 m^-3, argon ions (mass from the paper's Table 2).
_TE = ev_to_kelvin(1.0)
_TI = ev_to_kelvin(0.03)
_N = 1e14
_LAM = debye_length(_TE, _N)
_WPI = ion_plasma_frequency(_N, M_ARGON)


def single_grain_small(seed: int = 1) -> Workload:
    """One 5 um grain at the origin, Q0 = 0, self-consistent charging, Mach 1,
    nu = 0.1 omega_pi, R = 3 lambda, H = 6 lambda, N = 2000, dt = 0.01/omega_pi,
    200 steps."""
    return Workload(Te=_TE, Ti=_TI, n_inf=_N, m_i=M_ARGON, mach=1.0, nu_in=0.1 * _WPI,
                    E_ext=float("nan"), R=3 * _LAM, H=6 * _LAM, dt=0.01 / _WPI,
                    n_ions=2000, n_steps=200, n_discard=0, seed=seed,
                    charge_mode=CHARGE_CONSISTENT,
                    dust=[(0.0, 0.0, 0.0, 5e-6, 0.0)], name="single-grain N=2000")


def single_grain_production(mach: float = 1.0, seed: int = 11) -> Workload:
    """Same plasma and geometry, N = 2^18, 10,000 steps, first 5,000 discarded."""
    return single_grain_small(seed).with_(mach=mach, n_ions=1 << 18, n_steps=10000,
                                          n_discard=5000,
                                          name=f"single-grain N=2^18 M={mach}")


def two_grain_wake(seed: int = 2) -> Workload:
    """Two 5 um grains on the axis 0.5 lambda apart (z = -/+ 0.25 lambda), Mach 1,
    N = 2^20, R = 3 lambda, H = 8 lambda, 20,000 steps."""
    return single_grain_small(seed).with_(
        n_ions=1 << 20, H=8 * _LAM, n_steps=20000, n_discard=10000,
        dust=[(0.0, 0.0, -0.25 * _LAM, 5e-6, 0.0), (0.0, 0.0, 0.25 * _LAM, 5e-6, 0.0)],
        name="two-grain wake N=2^20")


def chain8(n_ions: int = 1 << 21, seed: int = 4) -> Workload:
    """Vertical chain of 8 grains at 0.4 lambda spacing, centred on the axis."""
    dust = [(0.0, 0.0, (k - 3.5) * 0.4 * _LAM, 5e-6, 0.0) for k in range(8)]
    return single_grain_small(seed).with_(n_ions=n_ions, H=8 * _LAM, dust=dust,
                                          n_steps=5000, n_discard=2500,
                                          name=f"chain-8 N={n_ions}")


def long_domain(n_ions: int = 1 << 20, seed: int = 5) -> Workload:
    """The constant-concentration series of the cutoff study: one 5 um grain
    at the origin, R = 3 lambda, and a height that grows with N so that the
    superparticle density stays that of 2^16 ions in 6 lambda
    (H = 6 lambda N / 2^16); otherwise the single-grain plasma (Mach 1,
    nu = 0.1 omega_pi).  Used with an ion-ion cutoff of 4 lambda switched
    from 3 lambda (CUTOFF_SWITCH, CUTOFF_RADIUS)."""
    return single_grain_small(seed).with_(n_ions=n_ions, H=6 * _LAM * n_ions / (1 << 16),
                                          n_steps=1000, n_discard=500,
                                          name=f"long domain N={n_ions}")


CUTOFF_SWITCH = 3 * _LAM
CUTOFF_RADIUS = 4 * _LAM


def paper_table2(n_ions: int = 1 << 16) -> Workload:
    """The paper's first test case (Table 2): Te = 29011 K, Ti = 290.11 K,
    n = 1e14, argon, M = 1, R = 3, H = 6 (Debye lengths), dt = 3.5148e-10 s,
    grain r = 58.8 um at (0, 0, -1) lambda, preset charge 392,500 e."""
    te, ti, n = 29011.0, 290.11, 1e14
    lam = debye_length(te, n)
    return Workload(Te=te, Ti=ti, n_inf=n, m_i=M_ARGON, mach=1.0, nu_in=0.0, E_ext=0.0,
                    R=3 * lam, H=6 * lam, dt=3.5148e-10, n_ions=n_ions, n_steps=3000,
                    n_discard=0, seed=7, charge_mode=CHARGE_GIVEN,
                    dust=[(0.0, 0.0, -lam, 58.8e-6, -392500 * QE)], name="paper table 2")


def sweep_systems(n_systems: int = 64, seed: int = 3, log2n_lo: float = 14.0,
                  log2n_hi: float = 17.0) -> List[Workload]:
    """Batched sweep: log2 N ~ U(lo, hi) rounded to a multiple of 256,
    Mach ~ U(0.3, 2), radius ~ U(2, 10) um, nu ~ U(0.02, 0.3) omega_pi."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    out = []
    for s in range(n_systems):
        n = int(round(2.0 ** rng.uniform(log2n_lo, log2n_hi) / 256.0)) * 256
        mach = rng.uniform(0.3, 2.0)
        rad = rng.uniform(2e-6, 10e-6)
        nu = rng.uniform(0.02, 0.3) * _WPI
        w = single_grain_small(seed).with_(n_ions=max(n, 256), mach=mach, nu_in=nu,
                                           n_steps=5000, system_id=s,
                                           dust=[(0.0, 0.0, 0.0, rad, 0.0)],
                                           name=f"sweep[{s}]")
        out.append(w)
    return out


# ---------------------------------------------------------------------------
# Seeded particle-state generators (positions/velocities in SI).

def absorption_shell_state(w: Workload, n: int, grain: int = 0, shell_steps: float = 3.0,
                           seed: int = 99):
    """Ions placed uniformly in a shell just outside a grain (up to
    `shell_steps` thermal-plus-drift step lengths away) with velocities aimed
    inward with a random spread, so that many are absorbed in one step.
    Returns (x[n,3], v[n,3]) in SI."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    gx, gy, gz, a, _ = w.dust[grain]
    c = np.array([gx, gy, gz])
    speed = (w.mach + 1.0) * math.sqrt(KB * w.Te / w.m_i)
    dr = shell_steps * speed * w.dt
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = a * (1.0 + 1e-3) + dr * rng.uniform(0.0, 1.0, size=(n, 1))
    x = c + d * r
    aim = -d + 0.6 * rng.normal(size=(n, 3))
    aim /= np.linalg.norm(aim, axis=1, keepdims=True)
    v = aim * speed * rng.uniform(0.3, 1.5, size=(n, 1))
    return x, v


def wall_shell_state(w: Workload, n: int, seed: int = 98):
    """Ions within one step length of the cylinder wall or end caps, with
    random velocities, so that many exit in one step.  SI."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    speed = (w.mach + 1.0) * math.sqrt(KB * w.Te / w.m_i)
    band = 2.0 * speed * w.dt
    x = np.empty((n, 3))
    kind = rng.integers(0, 3, size=n)
    th = rng.uniform(0, 2 * math.pi, size=n)
    # side band
    r_side = w.R - band * rng.uniform(0, 1, size=n)
    z_side = w.H * (rng.uniform(0, 1, size=n) - 0.5)
    # cap band
    r_cap = w.R * np.sqrt(rng.uniform(0, 0.98, size=n))
    z_cap = (0.5 * w.H - band * rng.uniform(0, 1, size=n)) * np.where(kind == 1, 1.0, -1.0)
    side = kind == 0
    rr = np.where(side, r_side, r_cap)
    x[:, 0] = rr * np.cos(th)
    x[:, 1] = rr * np.sin(th)
    x[:, 2] = np.where(side, z_side, z_cap)
    v = rng.normal(size=(n, 3)) * speed
    return x, v


def uniform_cylinder_state(w: Workload, n: int, seed: int = 97):
    """Uniform positions in the cylinder, thermal velocities around (0,0,u)
    (drawn with numpy, independent of the methods' own Philox init).  SI."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    r = w.R * np.sqrt(rng.uniform(0, 1, size=n))
    th = rng.uniform(0, 2 * math.pi, size=n)
    z = w.H * (rng.uniform(0, 1, size=n) - 0.5)
    x = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)
    sig = math.sqrt(KB * w.Ti / w.m_i)
    u = w.mach * math.sqrt(KB * w.Te / w.m_i)
    v = rng.normal(size=(n, 3)) * sig
    v[:, 2] += u
    return x, v
