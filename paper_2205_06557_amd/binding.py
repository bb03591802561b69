"""ctypes binding of libodust.so (the C-ABI of include/odust.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch, when present, supplies the HIP stream and (optionally) the
device memory through the library's allocator hook.  If the library has not
been built this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libodust.so")

OD_OK, OD_EINVAL, OD_EDEVICE, OD_ENUMERIC, OD_ESTATE, OD_ENOMEM = 0, -1, -2, -3, -4, -5
PREC_FP32, PREC_FP64 = 0, 1
PAIR_AUTO, PAIR_ONE_SIDED, PAIR_SYMMETRIC = 0, 1, 2
EV_NONE, EV_EXIT, EV_ABS_BASE, EV_COLL_BIT = 0, 1, 2, 0x80
KERNEL_CLASSES = ("pair", "tail", "reinject", "finalize")   # finalize runs inside the tail


class OdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"odust error {status}: {msg}")
        self.status = status


class Plasma(C.Structure):
    _fields_ = [("T_e", C.c_double), ("T_i", C.c_double), ("n_inf", C.c_double),
                ("m_i", C.c_double), ("mach", C.c_double), ("nu_in", C.c_double),
                ("E_ext", C.c_double)]


class Sim(C.Structure):
    _fields_ = [("R", C.c_double), ("H", C.c_double), ("dt", C.c_double),
                ("n_ions", C.c_int64), ("n_discard", C.c_int64), ("seed", C.c_uint64),
                ("system_id", C.c_uint64), ("charge_mode", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class Dust(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double),
                ("radius", C.c_double), ("q0", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", FREE_FN), ("ctx", C.c_void_p)]


_lib = None


def lib():
    """Loads libodust.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2205_06557_amd.build` (no CPU fallback exists)")
        # PyTorch ships its own HIP runtime.  Loading it first makes the
        # library bind to that same runtime (one HIP/HSA runtime per process),
        # so PyTorch's streams and memory are valid handles for the library;
        # loading the library first would bring in a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i64, u64 = C.c_void_p, C.c_int64, C.c_uint64
        L.od_init_system.argtypes = [C.POINTER(Plasma), C.POINTER(Sim), C.POINTER(Dust), C.c_int32,
                                     vp, C.POINTER(Allocator), C.POINTER(vp)]
        L.od_step.argtypes = [vp, i64]
        L.od_sync.argtypes = [vp]
        L.od_get_dust_charges.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.od_get_dust_forces.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
        L.od_destroy.argtypes = [vp]
        L.od_destroy.restype = None
        L.od_last_error.restype = C.c_char_p
        L.od_get_units.argtypes = [vp, C.POINTER(C.c_double)]
        L.od_get_sizes.argtypes = [vp, C.POINTER(C.c_int64)]
        L.od_get_state.argtypes = [vp, vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.od_set_state.argtypes = [vp, vp, vp, C.POINTER(C.c_double), i64]
        L.od_get_accelerations.argtypes = [vp, vp]
        L.od_get_step_events.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.od_rng_block.argtypes = [u64, u64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.od_set_timing.argtypes = [vp, C.c_int32]
        L.od_get_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.od_get_confinement.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.od_set_cutoff.argtypes = [vp, C.c_double, C.c_double]
        L.od_set_pair_split.argtypes = [vp, C.c_int32]
        L.od_get_pair_split.argtypes = [vp, C.POINTER(C.c_int32)]
        L.od_set_pair_kernel.argtypes = [vp, C.c_int32]
        L.od_get_pair_kernel.argtypes = [vp, C.POINTER(C.c_int32)]
        L.od_get_cutoff_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.od_set_graph.argtypes = [vp, C.c_int32]
        L.od_get_absorbed.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), i64, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
        L.od_set_history.argtypes = [vp, i64]
        L.od_get_history.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        for name in ("od_init_system", "od_step", "od_sync", "od_get_dust_charges",
                     "od_get_dust_forces", "od_get_units", "od_get_sizes", "od_get_state",
                     "od_set_state", "od_get_accelerations", "od_get_step_events",
                     "od_rng_block", "od_set_timing", "od_get_kernel_times",
                     "od_get_confinement", "od_set_cutoff", "od_get_cutoff_info",
                     "od_set_pair_split", "od_get_pair_split", "od_set_pair_kernel",
                     "od_get_pair_kernel", "od_set_graph", "od_get_absorbed", "od_set_history",
                     "od_get_history"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != OD_OK:
        raise OdError(st, lib().od_last_error().decode(errors="replace"))


def _ptr(a: Optional[np.ndarray], ctype=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class TorchAllocator:
    """Device memory from PyTorch's caching allocator, handed to the library
    through its allocator hook."""

    def __init__(self):
        import torch
        self._torch = torch
        self._live = {}

        def _alloc(ctx, nbytes):
            t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
            p = (t.data_ptr() + 255) // 256 * 256
            self._live[p] = t
            return p

        def _free(ctx, ptr):
            self._live.pop(ptr, None)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = Allocator(self._a, self._f, None)


def rng_block(seed: int, system: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _check(lib().od_rng_block(seed, system, _ptr(c, C.c_uint64), _ptr(out, C.c_uint64)))
    return out


def _confinement(call):
    nr, nz = C.c_int32(0), C.c_int32(0)
    _check(call(None, None, C.byref(nr), C.byref(nz)))
    coef = np.zeros(15)
    grid = np.zeros((nr.value + 1) * (nz.value + 1))
    _check(call(_ptr(coef), _ptr(grid), C.byref(nr), C.byref(nz)))
    return coef, grid.reshape(nr.value + 1, nz.value + 1)


class System:
    """One dust system on the GPU.  `w` is a workloads.Workload (SI)."""

    def __init__(self, w, precision: int = PREC_FP32, stream=None, torch_memory: bool = False,
                 n_ions: Optional[int] = None):
        L = lib()
        self.w = w
        pl = Plasma(w.Te, w.Ti, w.n_inf, w.m_i, w.mach, w.nu_in, w.E_ext)
        N = int(n_ions if n_ions is not None else w.n_ions)
        sim = Sim(w.R, w.H, w.dt, N, int(w.n_discard), int(w.seed), int(w.system_id),
                  int(w.charge_mode), int(precision), int(w.flags), 0)
        nd = len(w.dust)
        dust = (Dust * max(nd, 1))(*[Dust(*d) for d in w.dust])
        if stream is None:
            stream = _torch_stream()
        self._alloc = TorchAllocator() if torch_memory else None
        h = C.c_void_p()
        _check(L.od_init_system(C.byref(pl), C.byref(sim), dust, nd, stream,
                                C.byref(self._alloc.struct) if self._alloc else None, C.byref(h)))
        self._h = h
        sz = np.zeros(4, dtype=np.int64)
        _check(L.od_get_sizes(h, _ptr(sz, C.c_int64)))
        self.N, self.nd, self.precision, self.Npad = (int(x) for x in sz)
        self.dtype = np.float32 if self.precision == PREC_FP32 else np.float64
        u = np.zeros(4)
        _check(L.od_get_units(h, _ptr(u)))
        self.units = dict(length=u[0], time=u[1], velocity=u[2], accel=u[3])

    def close(self):
        if getattr(self, "_h", None):
            lib().od_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- stepping ---------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().od_step(self._h, int(n)))

    def sync(self):
        _check(lib().od_sync(self._h))

    # --- observables --------------------------------------------------------
    def charges(self):
        q = np.zeros(max(self.nd, 1))
        qa = np.zeros(max(self.nd, 1))
        _check(lib().od_get_dust_charges(self._h, _ptr(q), _ptr(qa)))
        return q[: self.nd], qa[: self.nd]

    def forces(self, which: int = 0) -> np.ndarray:
        f = np.zeros((max(self.nd, 1), 4, 3))
        _check(lib().od_get_dust_forces(self._h, which, _ptr(f)))
        return f[: self.nd]

    # --- state --------------------------------------------------------------
    def get_state(self):
        x = np.zeros((3, self.N), dtype=self.dtype)
        v = np.zeros((3, self.N), dtype=self.dtype)
        q = np.zeros(max(self.nd, 1))
        st = C.c_int64(0)
        _check(lib().od_get_state(self._h, x.ctypes.data, v.ctypes.data, _ptr(q), C.byref(st)))
        return x, v, q[: self.nd], st.value

    def set_state(self, x=None, v=None, q=None, step: int = 0):
        xs = None if x is None else np.ascontiguousarray(x, dtype=self.dtype).reshape(3, self.N)
        vs = None if v is None else np.ascontiguousarray(v, dtype=self.dtype).reshape(3, self.N)
        qs = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        _check(lib().od_set_state(self._h, None if xs is None else xs.ctypes.data,
                                  None if vs is None else vs.ctypes.data, _ptr(qs), int(step)))

    def accelerations(self) -> np.ndarray:
        a = np.zeros((3, self.N), dtype=self.dtype)
        _check(lib().od_get_accelerations(self._h, a.ctypes.data))
        return a

    def confinement(self):
        """(coefficients [15] in volts, grid [nr+1, nz+1] in volts) of the
        confinement field fitted at creation."""
        return _confinement(lambda *a: lib().od_get_confinement(self._h, *a))

    def set_pair_split(self, nsplit: int):
        """Source splits of the one-sided pair sum (1..4)."""
        _check(lib().od_set_pair_split(self._h, int(nsplit)))

    def pair_split(self) -> int:
        n = C.c_int32(0)
        _check(lib().od_get_pair_split(self._h, C.byref(n)))
        return n.value

    def set_pair_kernel(self, kind: int):
        """PAIR_AUTO, PAIR_ONE_SIDED or PAIR_SYMMETRIC."""
        _check(lib().od_set_pair_kernel(self._h, int(kind)))

    def pair_kernel(self) -> int:
        k = C.c_int32(0)
        _check(lib().od_get_pair_kernel(self._h, C.byref(k)))
        return k.value

    def set_cutoff(self, r_switch: float, r_cut: float):
        """Ion-ion cutoff with a switching function (distances in m); r_cut <= 0 removes it."""
        _check(lib().od_set_cutoff(self._h, float(r_switch), float(r_cut)))

    def cutoff_info(self):
        """(number of slabs, ion pairs evaluated in the last step)."""
        ns, npairs = C.c_int32(0), C.c_int64(0)
        _check(lib().od_get_cutoff_info(self._h, C.byref(ns), C.byref(npairs)))
        return ns.value, npairs.value

    def events(self):
        ev = np.zeros(self.N, dtype=np.uint8)
        nabs = np.zeros(max(self.nd, 1), dtype=np.int64)
        ne = C.c_int64(0)
        nc = C.c_int64(0)
        _check(lib().od_get_step_events(self._h, _ptr(ev, C.c_uint8), _ptr(nabs, C.c_int64),
                                        C.byref(ne), C.byref(nc)))
        return ev, nabs[: self.nd], ne.value, nc.value

    # --- timing -------------------------------------------------------------
    def absorbed(self, cap: Optional[int] = None):
        """(ion indices, grains) of the ions absorbed in the last step, and the
        number that exited."""
        cap = self.N if cap is None else int(cap)
        idx = np.zeros(max(cap, 1), dtype=np.int64)
        by = np.zeros(max(cap, 1), dtype=np.int32)
        na, ne = C.c_int64(0), C.c_int64(0)
        _check(lib().od_get_absorbed(self._h, _ptr(idx, C.c_int64), _ptr(by, C.c_int32), cap, C.byref(na),
                                     C.byref(ne)))
        k = min(na.value, cap)
        return idx[:k], by[:k], na.value, ne.value

    def set_history(self, capacity: int):
        _check(lib().od_set_history(self._h, int(capacity)))

    def history(self):
        """Per-step records [steps, n_dust, 14]: Q^n (C), 12 force components (N), absorbed count."""
        n = C.c_int64(0)
        _check(lib().od_get_history(self._h, None, C.byref(n)))
        rec = np.zeros((max(n.value, 1), self.nd, 14))
        _check(lib().od_get_history(self._h, _ptr(rec), C.byref(n)))
        return rec[: n.value]

    def set_timing(self, enable: bool):
        _check(lib().od_set_timing(self._h, 1 if enable else 0))

    def set_graph(self, steps_per_graph: int):
        """Replay steps_per_graph steps as one HIP graph (0: off); needs a
        system created on a stream other than the null stream."""
        _check(lib().od_set_graph(self._h, int(steps_per_graph)))

    def kernel_times(self):
        ms = np.zeros(len(KERNEL_CLASSES))
        n = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        _check(lib().od_get_kernel_times(self._h, _ptr(ms), _ptr(n, C.c_int64)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}


_batch_sigs = False


def _batch_lib():
    global _batch_sigs
    L = lib()
    if not _batch_sigs:
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        dp, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.od_init_batch.argtypes = [C.POINTER(Plasma), C.POINTER(Sim), C.POINTER(Dust),
                                    C.POINTER(C.c_int32), i32, vp, C.POINTER(Allocator), C.POINTER(vp)]
        L.od_destroy_batch.argtypes = [vp]
        L.od_destroy_batch.restype = None
        L.od_batch_set_config.argtypes = [vp, i32, i32, i64]
        L.od_batch_get_config.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), i64p,
                                          C.POINTER(C.c_int32)]
        L.od_batch_autotune.argtypes = [vp, C.c_char_p, dp]
        L.od_batch_set_graph.argtypes = [vp, i32]
        L.od_step_batch.argtypes = [vp, i64]
        L.od_batch_sync.argtypes = [vp]
        L.od_batch_get_sizes.argtypes = [vp, i32, i64p]
        L.od_batch_get_dust_charges.argtypes = [vp, i32, dp, dp]
        L.od_batch_get_dust_forces.argtypes = [vp, i32, i32, dp]
        L.od_batch_get_state.argtypes = [vp, i32, vp, vp, dp, i64p]
        L.od_batch_set_state.argtypes = [vp, i32, vp, vp, dp, i64]
        L.od_batch_get_accelerations.argtypes = [vp, i32, vp]
        L.od_batch_get_step_events.argtypes = [vp, i32, C.POINTER(C.c_uint8), i64p, i64p, i64p]
        L.od_batch_set_timing.argtypes = [vp, i32]
        L.od_batch_get_kernel_times.argtypes = [vp, dp, i64p]
        L.od_batch_get_confinement.argtypes = [vp, i32, dp, dp, C.POINTER(C.c_int32),
                                               C.POINTER(C.c_int32)]
        L.od_batch_set_pair_kernel.argtypes = [vp, i32]
        L.od_batch_get_pair_kernel.argtypes = [vp, C.POINTER(C.c_int32)]
        L.od_batch_set_sym_config.argtypes = [vp, i32, i32, i64]
        L.od_batch_get_sym_config.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), i64p,
                                              C.POINTER(C.c_int32)]
        for name in ("od_init_batch", "od_batch_set_config", "od_batch_get_config", "od_batch_autotune",
                     "od_batch_set_graph", "od_step_batch", "od_batch_sync", "od_batch_get_sizes",
                     "od_batch_get_dust_charges", "od_batch_get_dust_forces", "od_batch_get_state",
                     "od_batch_set_state", "od_batch_get_accelerations", "od_batch_get_step_events",
                     "od_batch_set_timing", "od_batch_get_kernel_times", "od_batch_get_confinement",
                     "od_batch_set_pair_kernel", "od_batch_get_pair_kernel", "od_batch_set_sym_config",
                     "od_batch_get_sym_config"):
            getattr(L, name).restype = C.c_int
        _batch_sigs = True
    return L


BATCH_TIME_CLASSES = ("pair", "tail", "reinject", "finalize", "graph")   # finalize runs inside the tail


class Batch:
    """Independent dust systems (a list of workloads.Workload) advanced
    together.  stream=None lets the library create its own stream."""

    def __init__(self, workloads, stream=None, torch_memory: bool = False):
        L = _batch_lib()
        ws = list(workloads)
        self.ws = ws
        n = len(ws)
        pls = (Plasma * n)(*[Plasma(w.Te, w.Ti, w.n_inf, w.m_i, w.mach, w.nu_in, w.E_ext) for w in ws])
        sims = (Sim * n)(*[Sim(w.R, w.H, w.dt, int(w.n_ions), int(w.n_discard), int(w.seed),
                               int(w.system_id), int(w.charge_mode), PREC_FP32, int(w.flags), 0)
                           for w in ws])
        dl = [Dust(*d) for w in ws for d in w.dust]
        dust = (Dust * max(len(dl), 1))(*dl)
        nd = (C.c_int32 * n)(*[len(w.dust) for w in ws])
        self._alloc = TorchAllocator() if torch_memory else None
        h = C.c_void_p()
        _check(L.od_init_batch(pls, sims, dust, nd, n, stream,
                               C.byref(self._alloc.struct) if self._alloc else None, C.byref(h)))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().od_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_config(self, persistent: bool = True, jsplit: int = 1, split_max_n: int = 0):
        _check(_batch_lib().od_batch_set_config(self._h, 1 if persistent else 0, int(jsplit),
                                                int(split_max_n)))

    def config(self):
        p, j, n = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        t = C.c_int64(0)
        _check(_batch_lib().od_batch_get_config(self._h, C.byref(p), C.byref(j), C.byref(t), C.byref(n)))
        return dict(persistent=p.value, jsplit=j.value, split_max_n=t.value, n_items=n.value)

    def autotune(self, cache_path: Optional[str] = None) -> float:
        ms = C.c_double(0)
        _check(_batch_lib().od_batch_autotune(self._h, cache_path.encode() if cache_path else None,
                                              C.byref(ms)))
        return ms.value

    def set_graph(self, steps: int):
        _check(_batch_lib().od_batch_set_graph(self._h, int(steps)))

    def step(self, n: int = 1):
        _check(_batch_lib().od_step_batch(self._h, int(n)))

    def sync(self):
        _check(_batch_lib().od_batch_sync(self._h))

    def sizes(self, s: int):
        o = np.zeros(4, dtype=np.int64)
        _check(_batch_lib().od_batch_get_sizes(self._h, s, _ptr(o, C.c_int64)))
        return dict(N=int(o[0]), n_dust=int(o[1]), nsplit=int(o[2]), Npad=int(o[3]))

    def charges(self, s: int):
        nd = max(len(self.ws[s].dust), 1)
        q, qa = np.zeros(nd), np.zeros(nd)
        _check(_batch_lib().od_batch_get_dust_charges(self._h, s, _ptr(q), _ptr(qa)))
        return q[: len(self.ws[s].dust)], qa[: len(self.ws[s].dust)]

    def forces(self, s: int, which: int = 0):
        nd = len(self.ws[s].dust)
        f = np.zeros((max(nd, 1), 4, 3))
        _check(_batch_lib().od_batch_get_dust_forces(self._h, s, which, _ptr(f)))
        return f[:nd]

    def get_state(self, s: int):
        N = int(self.ws[s].n_ions)
        x = np.zeros((3, N), dtype=np.float32)
        v = np.zeros((3, N), dtype=np.float32)
        q = np.zeros(max(len(self.ws[s].dust), 1))
        st = C.c_int64(0)
        _check(_batch_lib().od_batch_get_state(self._h, s, x.ctypes.data, v.ctypes.data, _ptr(q),
                                               C.byref(st)))
        return x, v, q[: len(self.ws[s].dust)], st.value

    def set_state(self, s: int, x=None, v=None, q=None, step: int = 0):
        N = int(self.ws[s].n_ions)
        xs = None if x is None else np.ascontiguousarray(x, dtype=np.float32).reshape(3, N)
        vs = None if v is None else np.ascontiguousarray(v, dtype=np.float32).reshape(3, N)
        qs = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        _check(_batch_lib().od_batch_set_state(self._h, s, None if xs is None else xs.ctypes.data,
                                               None if vs is None else vs.ctypes.data, _ptr(qs),
                                               int(step)))

    def accelerations(self, s: int):
        a = np.zeros((3, int(self.ws[s].n_ions)), dtype=np.float32)
        _check(_batch_lib().od_batch_get_accelerations(self._h, s, a.ctypes.data))
        return a

    def confinement(self, s: int):
        return _confinement(lambda *a: _batch_lib().od_batch_get_confinement(self._h, s, *a))

    def set_pair_kernel(self, kind: int):
        _check(_batch_lib().od_batch_set_pair_kernel(self._h, int(kind)))

    def pair_kernel(self) -> int:
        k = C.c_int32(0)
        _check(_batch_lib().od_batch_get_pair_kernel(self._h, C.byref(k)))
        return k.value

    def set_sym_config(self, persistent: bool = False, one_row: bool = False, items_target: int = 0):
        _check(_batch_lib().od_batch_set_sym_config(self._h, 1 if persistent else 0, 1 if one_row else 0,
                                                    int(items_target)))

    def sym_config(self):
        p, r, n = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        t = C.c_int64(0)
        _check(_batch_lib().od_batch_get_sym_config(self._h, C.byref(p), C.byref(r), C.byref(t), C.byref(n)))
        return dict(persistent=p.value, one_row=r.value, items_target=t.value, n_items=n.value)

    def events(self, s: int):
        N = int(self.ws[s].n_ions)
        ev = np.zeros(N, dtype=np.uint8)
        nabs = np.zeros(max(len(self.ws[s].dust), 1), dtype=np.int64)
        ne, nc = C.c_int64(0), C.c_int64(0)
        _check(_batch_lib().od_batch_get_step_events(self._h, s, _ptr(ev, C.c_uint8),
                                                     _ptr(nabs, C.c_int64), C.byref(ne), C.byref(nc)))
        return ev, nabs[: len(self.ws[s].dust)], ne.value, nc.value

    def absorbed(self, cap: Optional[int] = None):
        """(ion indices, grains) of the ions absorbed in the last step, and the
        number that exited."""
        cap = self.N if cap is None else int(cap)
        idx = np.zeros(max(cap, 1), dtype=np.int64)
        by = np.zeros(max(cap, 1), dtype=np.int32)
        na, ne = C.c_int64(0), C.c_int64(0)
        _check(lib().od_get_absorbed(self._h, _ptr(idx, C.c_int64), _ptr(by, C.c_int32), cap, C.byref(na),
                                     C.byref(ne)))
        k = min(na.value, cap)
        return idx[:k], by[:k], na.value, ne.value

    def set_history(self, capacity: int):
        _check(lib().od_set_history(self._h, int(capacity)))

    def history(self):
        """Per-step records [steps, n_dust, 14]: Q^n (C), 12 force components (N), absorbed count."""
        n = C.c_int64(0)
        _check(lib().od_get_history(self._h, None, C.byref(n)))
        rec = np.zeros((max(n.value, 1), self.nd, 14))
        _check(lib().od_get_history(self._h, _ptr(rec), C.byref(n)))
        return rec[: n.value]

    def set_timing(self, enable: bool):
        _check(_batch_lib().od_batch_set_timing(self._h, 1 if enable else 0))

    def kernel_times(self):
        ms = np.zeros(5)
        n = np.zeros(5, dtype=np.int64)
        _check(_batch_lib().od_batch_get_kernel_times(self._h, _ptr(ms), _ptr(n, C.c_int64)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(BATCH_TIME_CLASSES)}


class BatchMember:
    """Adapter exposing one system of a Batch with the System interface used
    by the shadowed-step parity helper."""

    def __init__(self, batch: Batch, s: int):
        self.b, self.s = batch, s
        self.N = int(batch.ws[s].n_ions)
        self.precision = PREC_FP32

    def get_state(self):
        return self.b.get_state(self.s)

    def set_state(self, x=None, v=None, q=None, step: int = 0):
        self.b.set_state(self.s, x, v, q, step)

    def step(self, n: int = 1):
        self.b.step(n)

    def sync(self):
        self.b.sync()

    def accelerations(self):
        return self.b.accelerations(self.s)

    def confinement(self):
        return self.b.confinement(self.s)

    def events(self):
        return self.b.events(self.s)

    def forces(self, which: int = 0):
        return self.b.forces(self.s, which)

    def charges(self):
        return self.b.charges(self.s)


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("lr_final", C.c_double), ("seed", C.c_uint64)]


_mlp_sigs = False
MLP_PARAMS = 35856


def _mlp_lib():
    global _mlp_sigs
    L = lib()
    if not _mlp_sigs:
        vp, i64 = C.c_void_p, C.c_int64
        fp, dp = C.POINTER(C.c_float), C.POINTER(C.c_double)
        L.od_mlp_create.argtypes = [C.c_uint64, vp, C.POINTER(vp)]
        L.od_mlp_destroy.argtypes = [vp]
        L.od_mlp_destroy.restype = None
        L.od_mlp_get_params.argtypes = [vp, fp]
        L.od_mlp_set_params.argtypes = [vp, fp]
        L.od_mlp_set_normalization.argtypes = [vp, fp, fp, fp, fp]
        L.od_mlp_predict.argtypes = [vp, fp, i64, fp, C.POINTER(C.c_int32)]
        L.od_mlp_predict_noalloc.argtypes = [vp, vp, i64, vp, vp]
        L.od_surrogate_train.argtypes = [fp, fp, i64, fp, fp, C.POINTER(TrainCfg), C.c_uint64, vp, C.POINTER(vp)]
        L.od_surrogate_predict.argtypes = [vp, fp, i64, fp, C.POINTER(C.c_int32)]
        L.od_mlp_loss_grad.argtypes = [vp, fp, fp, i64, fp, dp]
        L.od_mlp_train.argtypes = [vp, fp, fp, i64, C.POINTER(TrainCfg), dp]
        L.od_oml_floating_charge.argtypes = [C.POINTER(Plasma), C.c_double, dp]
        for name in ("od_mlp_create", "od_mlp_get_params", "od_mlp_set_params", "od_mlp_set_normalization",
                     "od_mlp_predict", "od_mlp_predict_noalloc", "od_mlp_loss_grad", "od_mlp_train",
                     "od_oml_floating_charge", "od_surrogate_train", "od_surrogate_predict"):
            getattr(L, name).restype = C.c_int
        _mlp_sigs = True
    return L


def oml_floating_charge(w, radius: float) -> float:
    """Floating charge (C) of an isolated grain of `radius` in workload w's plasma."""
    pl = Plasma(w.Te, w.Ti, w.n_inf, w.m_i, w.mach, w.nu_in, w.E_ext)
    q = C.c_double(0)
    _check(_mlp_lib().od_oml_floating_charge(C.byref(pl), float(radius), C.byref(q)))
    return q.value


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Mlp:
    """The 5 -> 128 -> 128 -> 128 -> 16 surrogate network on the GPU."""

    def __init__(self, seed: int = 0, stream=None):
        h = C.c_void_p()
        if stream is None:
            stream = _torch_stream()
        _check(_mlp_lib().od_mlp_create(int(seed), stream, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _mlp_lib().od_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_mlp_lib().od_mlp_get_params(self._h, _ptr(p, C.c_float)))
        return p

    def set_params(self, p):
        p = _f32(p)
        assert p.size == MLP_PARAMS
        _check(_mlp_lib().od_mlp_set_params(self._h, _ptr(p, C.c_float)))

    def set_normalization(self, in_lo, in_hi, out_mean, out_std):
        a, b, c, d = _f32(in_lo), _f32(in_hi), _f32(out_mean), _f32(out_std)
        _check(_mlp_lib().od_mlp_set_normalization(self._h, _ptr(a, C.c_float), _ptr(b, C.c_float),
                                                    _ptr(c, C.c_float), _ptr(d, C.c_float)))

    def predict(self, X):
        X = _f32(X).reshape(-1, 5)
        n = X.shape[0]
        Y = np.zeros((n, 16), dtype=np.float32)
        inside = np.zeros(n, dtype=np.int32)
        _check(_mlp_lib().od_mlp_predict(self._h, _ptr(X, C.c_float), n, _ptr(Y, C.c_float),
                                         _ptr(inside, C.c_int32)))
        return Y, inside.astype(bool)

    def predict_noalloc(self, X_dev: int, n: int, Y_dev: int, inside_dev: Optional[int] = None):
        """od_mlp_predict_noalloc on device addresses (for instance
        ``tensor.data_ptr()`` of float32 [n,5], float32 [n,16] and int32 [n]
        tensors); asynchronous on the network's stream."""
        _check(_mlp_lib().od_mlp_predict_noalloc(self._h, C.c_void_p(X_dev), int(n), C.c_void_p(Y_dev),
                                                 None if inside_dev is None else C.c_void_p(inside_dev)))

    def loss_grad(self, Xn, Tn):
        Xn = _f32(Xn).reshape(-1, 5)
        Tn = _f32(Tn).reshape(-1, 16)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        L = C.c_double(0)
        _check(_mlp_lib().od_mlp_loss_grad(self._h, _ptr(Xn, C.c_float), _ptr(Tn, C.c_float),
                                           Xn.shape[0], _ptr(g, C.c_float), C.byref(L)))
        return L.value, g

    def train(self, X, T, epochs: int, batch: int, lr: float = 2e-3, lr_final: float = 5e-5,
              seed: int = 0):
        X = _f32(X).reshape(-1, 5)
        T = _f32(T).reshape(-1, 16)
        cfg = TrainCfg(int(epochs), int(batch), float(lr), float(lr_final), int(seed))
        hist = np.zeros(int(epochs))
        _check(_mlp_lib().od_mlp_train(self._h, _ptr(X, C.c_float), _ptr(T, C.c_float), X.shape[0],
                                       C.byref(cfg), _ptr(hist)))
        return hist

