"""Oracle pin: the full model at Mach 0 is isotropic.

With no flow, no drive and no collisions (ion-ion and ion-dust forces on, a
grain of fixed charge at the centre), the time-averaged force on the grain
(Eq. (1) plus Eq. (3)) vanishes within its block-averaged standard error, and
the ion density around the grain is symmetric in +-z.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W


@pytest.mark.slow
def test_mach0_zero_net_force_and_isotropy():
    w = W.single_grain_small().with_(mach=0.0, nu_in=0.0, E_ext=0.0, n_ions=800,
                                     charge_mode=W.CHARGE_GIVEN,
                                     dust=[(0.0, 0.0, 0.0, 20e-6, -20000 * W.QE)])
    o = O.Oracle(w)
    o.run(200)
    blocks = []
    zs = []
    nb, bl = 12, 100
    for b in range(nb):
        acc = np.zeros(3)
        for k in range(bl):
            o.step()
            F = o.last_step()["F"][0]
            acc += F[0] + F[2]
        blocks.append(acc / bl)
        zs.append(o.get_state()[0][:, 2].copy())
    blocks = np.array(blocks)
    mean = blocks.mean(axis=0)
    se = blocks.std(axis=0, ddof=1) / math.sqrt(nb)
    assert (np.abs(mean) <= 4 * se + 1e-30).all(), (mean, se)
    z = np.concatenate(zs)
    lam = w.lam
    up = np.sum((z > 0) & (z < lam))
    dn = np.sum((z < 0) & (z > -lam))
    assert abs(up - dn) < 5 * math.sqrt(up + dn)
