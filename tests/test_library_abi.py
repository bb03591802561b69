"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid parameters before touching a device."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2205_06557_amd import binding as B
from paper_2205_06557_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "odust.h")).read()
    return sorted(set(re.findall(r"\b(od_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert "od_init_system" in names and "od_step" in names
    for n in names:
        assert hasattr(L, n), n


def _init(w, **over):
    pl = B.Plasma(w.Te, w.Ti, w.n_inf, w.m_i, w.mach, w.nu_in, w.E_ext)
    sim = B.Sim(w.R, w.H, w.dt, w.n_ions, w.n_discard, w.seed, 0, w.charge_mode, 0, w.flags, 0)
    for k, v in over.items():
        setattr(sim, k, v)
    nd = len(w.dust)
    dust = (B.Dust * max(nd, 1))(*[B.Dust(*d) for d in w.dust])
    h = C.c_void_p()
    return B.lib().od_init_system(C.byref(pl), C.byref(sim), dust, nd, None, None, C.byref(h))


@pytest.mark.parametrize("over", [dict(n_ions=1), dict(n_ions=(1 << 29) + 1), dict(dt=0.0), dict(R=-1.0), dict(charge_mode=5),
                                  dict(precision=3), dict(flags=64), dict(reserved=1)])
def test_invalid_parameters_rejected(over):
    assert _init(W.single_grain_small(), **over) == B.OD_EINVAL
    assert B.lib().od_last_error()


def test_invalid_dust_rejected():
    w = W.single_grain_small()
    lam = w.lam
    assert _init(w.with_(dust=[(2.99 * lam, 0, 0, 20e-6, 0.0)])) == B.OD_EINVAL      # crosses wall
    assert _init(w.with_(dust=[(0, 0, 0, 5e-6, 0.0), (0, 0, 8e-6, 5e-6, 0.0)])) == B.OD_EINVAL
    assert _init(w.with_(dust=[(0, 0, 0, 5e-6, 0.0)] * 40)) == B.OD_EINVAL


def test_null_arguments_rejected():
    L = B.lib()
    assert L.od_step(None, 1) == B.OD_EINVAL
    assert L.od_sync(None) == B.OD_EINVAL
    assert L.od_get_dust_forces(None, 0, None) == B.OD_EINVAL
    L.od_destroy(None)


def test_missing_device_is_reported():
    """Without a visible GPU, creating a system fails with OD_EDEVICE and a
    plain message (valid parameters, so the device check is what fails)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    assert _init(W.single_grain_small()) == B.OD_EDEVICE
    assert b"no HIP device" in B.lib().od_last_error()
