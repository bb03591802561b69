"""ctypes front end of the FP64 CPU oracle (``odust_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library never imports,
links or calls it, and it imports nothing from the product package except the
input descriptions in ``workloads``.

All quantities are SI (m, m/s, m/s^2, C, N).  The arithmetic lives in the C
file; this module only builds it, marshals arrays and exposes a few
closed-form helpers that the C file exports (Philox, uniforms, face fluxes,
flux-weighted inverse CDF, OML currents).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "odust_oracle.c")
LIB = os.path.join(HERE, "libodust_oracle.so")

EV_NONE = -1
EV_EXITED = -2
FLAG_CONFINEMENT = 4
FLAG_FIELD_DRIVEN = 8
# grid of the confinement potential (Appendix A): intervals along r and along z
CONF_NX = 32
CONF_NZ = 32


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def sanitizer_command(out: str) -> list:
    """gcc line of an AddressSanitizer + UBSan build of the oracle (same
    floating-point flags as build()); load it with ODUST_ORACLE_LIB=out and
    LD_PRELOAD naming libasan.so and libubsan.so."""
    return ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
            "-fPIC", "-shared", "-std=c11", "-o", out, SRC, "-lm"]


_lib = None


def lib():
    """The oracle library: the build next to this file, or, when the
    environment names one in ODUST_ORACLE_LIB, another build of the same
    source (for instance one with AddressSanitizer and UBSan, see
    ``sanitizer_command``)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("ODUST_ORACLE_LIB")
        if not alt:
            build()
        L = C.CDLL(alt or LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        u64p = C.POINTER(C.c_uint64)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        L.orc_create.restype = P
        L.orc_create.argtypes = [dp, dp, C.c_int64, C.c_int64, C.c_uint64, C.c_uint64,
                                 C.c_int, C.c_int, dp, C.c_int]
        L.orc_destroy.argtypes = [P]
        L.orc_derived.argtypes = [P, dp, u64p]
        L.orc_init.argtypes = [P]
        L.orc_init.restype = C.c_int
        L.orc_step.argtypes = [P]
        L.orc_step.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_get_state.argtypes = [P, dp, dp, dp, i64p]
        L.orc_set_state.argtypes = [P, dp, dp, dp, C.c_int64]
        L.orc_last_step.argtypes = [P, dp, i32p, i32p, dp, dp, i64p, i64p]
        L.orc_averages.argtypes = [P, dp, dp]
        L.orc_averages.restype = C.c_int64
        L.orc_accel_subset.argtypes = [P, i64p, C.c_int64, dp]
        L.orc_dust_forces_now.argtypes = [P, dp]
        L.orc_philox.argtypes = [u64p, u64p, u64p]
        L.orc_uniform.argtypes = [C.c_uint64]
        L.orc_uniform.restype = C.c_double
        for name in ("orc_face_flux",):
            getattr(L, name).argtypes = [C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        for name in ("orc_flux_tail", "orc_flux_inverse"):
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.orc_electron_current.argtypes = [C.c_double] * 4
        L.orc_electron_current.restype = C.c_double
        L.orc_ion_current_oml.argtypes = [C.c_double] * 6
        L.orc_ion_current_oml.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        for name in ("orc_fd_density", "orc_fd_tail", "orc_fd_head"):
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double]
            getattr(L, name).restype = C.c_double
        L.orc_fd_inverse.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_fd_inverse.restype = C.c_double
        L.orc_set_cutoff.argtypes = [P, C.c_double, C.c_double]
        L.orc_confinement_grid.argtypes = [P, C.c_int, C.c_int, dp]
        L.orc_set_confinement.argtypes = [P, dp, C.c_double, C.c_double, C.c_int]
        L.orc_confinement_terms.argtypes = [i32p, i32p]
        L.orc_confinement_eval.argtypes = [P, C.c_int64, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    u64 = C.POINTER(C.c_uint64)
    lib().orc_philox(c.ctypes.data_as(u64), k.ctypes.data_as(u64), out.ctypes.data_as(u64))
    return out


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w))


def face_flux(ubar: float, sig: float) -> float:
    return lib().orc_face_flux(ubar, sig)


def flux_tail(v: float, ubar: float, sig: float) -> float:
    return lib().orc_flux_tail(v, ubar, sig)


def flux_inverse(uu: float, ubar: float, sig: float) -> float:
    return lib().orc_flux_inverse(uu, ubar, sig)


def electron_current(Q: float, a: float, n: float, Te: float) -> float:
    return lib().orc_electron_current(Q, a, n, Te)


def ion_current_oml(Q: float, a: float, n: float, Ti: float, mi: float, u: float) -> float:
    return lib().orc_ion_current_oml(Q, a, n, Ti, mi, u)


def fd_density(v: float, ufd: float, sig: float) -> float:
    """Stationary v_z density of the field-driven collisional flow."""
    return lib().orc_fd_density(v, ufd, sig)


def fd_tail(x: float, ufd: float, sig: float) -> float:
    """int_x^inf v phi(v) dv of the field-driven distribution."""
    return lib().orc_fd_tail(x, ufd, sig)


def fd_head(w: float, ufd: float, sig: float) -> float:
    """-int_-inf^-w v phi(v) dv of the field-driven distribution."""
    return lib().orc_fd_head(w, ufd, sig)


def fd_inverse(uu: float, ufd: float, sig: float, top: bool) -> float:
    """Flux-weighted inward speed at the bottom (top=False) or top face."""
    return lib().orc_fd_inverse(uu, ufd, sig, 1 if top else 0)


def confinement_terms():
    """(powers of r, powers of z) of the fifteen terms of Eq. (A.3), in the
    order of their coefficients alpha_0 .. alpha_14."""
    a = np.zeros(15, dtype=np.int32)
    b = np.zeros(15, dtype=np.int32)
    i32 = C.POINTER(C.c_int32)
    lib().orc_confinement_terms(a.ctypes.data_as(i32), b.ctypes.data_as(i32))
    return a, b


def fit_polynomial(grid: np.ndarray, nx: int, nz: int) -> np.ndarray:
    """Least-squares fit of Eq. (A.3) to the grid of Eq. (A.2), every node
    weighted alike.  The terms are written in the scaled variables
    (r/R)^2 = (k/nx)^2 and (z/(H/2))^2 = (p/nz)^2, which spans the same
    polynomials as the printed form and keeps the system well conditioned;
    coefficient m multiplies (r/R)^(r_pow_m) (z/(H/2))^(z_pow_m)."""
    rp, zp = confinement_terms()
    k, p = np.meshgrid(np.arange(nx + 1) / nx, np.arange(nz + 1) / nz, indexing="ij")
    A = np.stack([k.ravel() ** a * p.ravel() ** b for a, b in zip(rp, zp)], axis=1)
    alpha, *_ = np.linalg.lstsq(A, np.asarray(grid, dtype=np.float64).ravel(), rcond=None)
    return alpha


def num_threads() -> int:
    return lib().orc_num_threads()


class Oracle:
    """One dust system on the CPU, FP64, SI units."""

    DERIVED = ("lam", "wpi", "cs", "sig", "u", "V", "w", "q", "m", "E", "Pc", "Jb", "Jt", "Js", "ufd")

    def __init__(self, w, n_ions: Optional[int] = None, init: bool = True):
        L = lib()
        self.w = w
        self.N = int(n_ions if n_ions is not None else w.n_ions)
        self.nd = len(w.dust)
        plasma = np.asarray(w.plasma7(), dtype=np.float64)
        geom = np.asarray(w.geom3(), dtype=np.float64)
        dust = np.ascontiguousarray(w.dust_array().reshape(-1)) if self.nd else np.zeros(1)
        self._h = L.orc_create(_dp(plasma), _dp(geom), self.N, int(w.n_discard),
                               int(w.seed), int(w.system_id), int(w.charge_mode),
                               int(w.flags), _dp(dust), self.nd)
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        d = np.zeros(15)
        t = np.zeros(3, dtype=np.uint64)
        L.orc_derived(self._h, _dp(d), t.ctypes.data_as(C.POINTER(C.c_uint64)))
        self.derived = dict(zip(self.DERIVED, d.tolist()))
        self.Tc, self.Tb, self.Tbt = (int(x) for x in t)
        self.conf_alpha = None
        self.conf_grid = None
        if init:
            st = L.orc_init(self._h)
            if st != 0:
                raise RuntimeError(f"oracle init failed ({st})")
            if int(w.flags) & FLAG_CONFINEMENT:
                self.fit_confinement()

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    # --- stepping -------------------------------------------------------
    def step(self) -> int:
        return lib().orc_step(self._h)

    def run(self, n: int) -> int:
        return lib().orc_run(self._h, int(n))

    # --- state ----------------------------------------------------------
    def get_state(self):
        x = np.zeros((self.N, 3))
        v = np.zeros((self.N, 3))
        Q = np.zeros(max(self.nd, 1))
        st = C.c_int64(0)
        lib().orc_get_state(self._h, _dp(x), _dp(v), _dp(Q), C.byref(st))
        return x, v, Q[: self.nd].copy(), st.value

    def set_state(self, x, v, Q, step: int):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.N, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.N, 3)
        Qa = np.ascontiguousarray(Q if self.nd else np.zeros(1), dtype=np.float64)
        lib().orc_set_state(self._h, _dp(x), _dp(v), _dp(Qa), int(step))

    def last_step(self):
        """Outputs of the last step: dict with a [N,3], ev [N], hit [N],
        Qrec [nd], F [nd,4,3], nabs [nd], nexit, ncoll."""
        a = np.zeros((self.N, 3))
        ev = np.zeros(self.N, dtype=np.int32)
        hit = np.zeros(self.N, dtype=np.int32)
        nd1 = max(self.nd, 1)
        Qrec = np.zeros(nd1)
        F = np.zeros((nd1, 4, 3))
        nabs = np.zeros(nd1, dtype=np.int64)
        ec = np.zeros(2, dtype=np.int64)
        i32 = C.POINTER(C.c_int32)
        i64 = C.POINTER(C.c_int64)
        lib().orc_last_step(self._h, _dp(a), ev.ctypes.data_as(i32), hit.ctypes.data_as(i32),
                            _dp(Qrec), _dp(F), nabs.ctypes.data_as(i64), ec.ctypes.data_as(i64))
        nd = self.nd
        return dict(a=a, ev=ev, hit=hit, Qrec=Qrec[:nd], F=F[:nd], nabs=nabs[:nd],
                    nexit=int(ec[0]), ncoll=int(ec[1]))

    def last_counts(self):
        """(absorbed counts [nd], collection force of Eq. (3) [nd,3]) of the
        last step, without copying the per-ion arrays."""
        nd1 = max(self.nd, 1)
        F = np.zeros((nd1, 4, 3))
        nabs = np.zeros(nd1, dtype=np.int64)
        lib().orc_last_step(self._h, None, None, None, None, _dp(F),
                            nabs.ctypes.data_as(C.POINTER(C.c_int64)), None)
        return nabs[: self.nd], F[: self.nd, 2].copy()

    def averages(self):
        nd1 = max(self.nd, 1)
        Q = np.zeros(nd1)
        F = np.zeros((nd1, 4, 3))
        n = lib().orc_averages(self._h, _dp(Q), _dp(F))
        return Q[: self.nd], F[: self.nd], int(n)

    def accel_subset(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        a = np.zeros((len(idx), 3))
        lib().orc_accel_subset(self._h, idx.ctypes.data_as(C.POINTER(C.c_int64)), len(idx), _dp(a))
        return a

    # --- ion-ion cutoff with a switching function ----------------------
    def set_cutoff(self, r_switch: float, r_cut: float):
        """Switch the ion-ion energy off between r_switch and r_cut (m);
        r_cut <= 0 restores the plain all-pairs sum."""
        lib().orc_set_cutoff(self._h, float(r_switch), float(r_cut))

    # --- confinement field (Appendix A) ---------------------------------
    def confinement_grid(self, nx: int = CONF_NX, nz: int = CONF_NZ) -> np.ndarray:
        """Phi_ext of Eq. (A.1) at the nodes of Eq. (A.2) from the current ion
        positions, volts, shape [nx+1, nz+1] (index k along r, p along z)."""
        out = np.zeros((nx + 1) * (nz + 1))
        lib().orc_confinement_grid(self._h, nx, nz, _dp(out))
        return out.reshape(nx + 1, nz + 1)

    def fit_confinement(self, nx: int = CONF_NX, nz: int = CONF_NZ) -> np.ndarray:
        """Computes the grid from the current positions, fits Eq. (A.3) by
        least squares and installs the field.  Returns the coefficients."""
        grid = self.confinement_grid(nx, nz)
        rs, zs = self.w.R, 0.5 * self.w.H
        alpha = fit_polynomial(grid, nx, nz)
        lib().orc_set_confinement(self._h, _dp(alpha), rs, zs, 1)
        self.conf_grid, self.conf_alpha = grid, alpha
        return alpha

    def set_confinement(self, alpha, on: bool = True):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        lib().orc_set_confinement(self._h, _dp(a), self.w.R, 0.5 * self.w.H, int(on))

    def confinement_eval(self, x):
        """(P [n] volts, E_out [n,3] V/m) of the installed polynomial at x [n,3] (m)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        P = np.zeros(len(x))
        E = np.zeros((len(x), 3))
        lib().orc_confinement_eval(self._h, len(x), _dp(x), _dp(P), _dp(E))
        return P, E

    def dust_forces(self) -> np.ndarray:
        F = np.zeros((max(self.nd, 1), 4, 3))
        lib().orc_dust_forces_now(self._h, _dp(F))
        return F[: self.nd]
