"""GPU parity of the ion-ion cutoff with a switching function against the
FP64 oracle (which sums every pair with the switched force), plus the
properties of the slab sort: a cutoff beyond every distance gives the
all-pairs result, the sorted path is bitwise reproducible, and removing the
cutoff restores the all-pairs kernel exactly."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import accel_errors, say, shadow_step, to_oracle

pytestmark = pytest.mark.gpu

LAM = W.single_grain_small().lam


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("n_ions,H,r_sw,r_cut", [
    (2000, 6.0, 1.0, 1.5),          # 64 slabs
    (8229, 24.0, 1.2, 2.0),         # 192 slabs, ragged N
    (3000, 6.0, 0.0, 7.0),          # 13 slabs, all within reach, switching from r = 0
    (3000, 6.0, 0.0, 100.0),        # one slab
])
def test_shadowed_steps_with_cutoff(B, n_ions, H, r_sw, r_cut):
    w = W.single_grain_small().with_(n_ions=n_ions, H=H * LAM)
    say("cutoff", n_ions, "H", H, "r_sw", r_sw, "r_cut", r_cut)
    with B.System(w) as s:
        s.set_cutoff(r_sw * LAM, r_cut * LAM)
        o = O.Oracle(w)
        o.set_cutoff(r_sw * LAM, r_cut * LAM)
        for k in range(2):
            say("  step", k, shadow_step(s, o, w))
        s.step(20)
        say("  after 20 free steps", shadow_step(s, o, w))
        ns, npairs = s.cutoff_info()
        say("  slabs", ns, "pairs evaluated", npairs, "of", n_ions * n_ions)
        # about 16 H / r_cut slabs, 8 H / r_cut where that passes the 1024-slab
        # limit (one fewer if the ratio rounds below an integer)
        per = 16 if int(16 * H // r_cut) <= 1024 else 8
        k = min(1024, int(per * H // r_cut))
        assert ns in (max(1, k), max(1, k - 1)) and 0 < npairs


def test_cutoff_with_confinement_and_field_driven(B):
    """Every option of the paper at once: the ion-ion cutoff, the confinement
    field of Appendix A and the field-driven injection distribution, shadowed
    against the oracle with the same options."""
    w = W.single_grain_small().with_(n_ions=5000, H=12 * LAM,
                                     flags=W.FLAG_CONFINEMENT | W.FLAG_FIELD_DRIVEN)
    say("cutoff + confinement + field-driven")
    with B.System(w) as s:
        s.set_cutoff(2.0 * LAM, 3.0 * LAM)
        o = O.Oracle(w)
        o.set_cutoff(2.0 * LAM, 3.0 * LAM)
        for k in range(3):
            say("  step", k, shadow_step(s, o, w))
        s.step(20)
        say("  after 20 free steps", shadow_step(s, o, w))


def test_far_cutoff_equals_all_pairs(B):
    w = W.single_grain_small().with_(n_ions=4000)
    with B.System(w) as a, B.System(w) as c:
        a.set_pair_split(1)
        c.set_cutoff(40 * LAM, 50 * LAM)
        a.step(1)
        c.step(1)
        aa, ac = a.accelerations().astype(np.float64), c.accelerations().astype(np.float64)
        l2, p999, pmax = accel_errors(ac.T, aa.T)
        say("far cutoff vs all pairs", l2, p999, pmax)
        assert l2 < 2e-6 and p999 < 5e-6


@pytest.mark.parametrize("n_ions", [1 << 20, (1 << 21) + 600])
def test_sampled_outputs_long_domain(B, n_ions):
    """Sampled accelerations and grain forces against the oracle in the long
    domain, at 2^20 ions and at 2^21 + 600 (192 slabs, 8195 sorted tiles, a
    ragged last tile; the last 600 ions are in the sample)."""
    w = W.long_domain(n_ions)
    say("long domain", w.n_ions, "H/lambda", w.H / LAM)
    with B.System(w) as s:
        s.set_cutoff(W.CUTOFF_SWITCH, W.CUTOFF_RADIUS)
        s.step(2)
        o = O.Oracle(w, init=False)
        o.set_cutoff(W.CUTOFF_SWITCH, W.CUTOFF_RADIUS)
        to_oracle(s, o)
        s.step(1)
        s.sync()
        a = s.accelerations().T.astype(np.float64)
        lam, wpi = o.derived["lam"], o.derived["wpi"]
        idx = np.unique(np.concatenate([np.random.default_rng(3).choice(w.n_ions, size=384, replace=False),
                                        np.arange(w.n_ions - 600, w.n_ions, 8)]))
        ref = o.accel_subset(idx)
        l2, p999, pmax = accel_errors(a[idx] * lam * wpi * wpi, ref)
        say("  sampled accel errors", l2, p999, pmax)
        assert l2 <= 1e-5 and p999 <= 1e-5
        F, Fo = s.forces(0), o.dust_forces()
        for p in (0, 3):
            assert np.linalg.norm(F[0, p] - Fo[0, p]) <= 1e-5 * np.linalg.norm(Fo[0, p])
        ns, npairs = s.cutoff_info()
        say("  slabs", ns, "evaluated pairs per ion", npairs / w.n_ions)


def test_bitwise_reproducible_and_removable(B):
    w = W.single_grain_small().with_(n_ions=6000, H=18 * LAM)
    res = []
    for _ in range(2):
        with B.System(w) as s:
            s.set_cutoff(1.5 * LAM, 2.5 * LAM)
            s.step(15)
            x, v, q, _ = s.get_state()
            res.append((x, v, q, s.forces(0)))
    for a, b in zip(*res):
        assert np.array_equal(a, b)
    # removing the cutoff brings back the all-pairs kernel and its split
    with B.System(w) as plain, B.System(w) as s:
        split = plain.pair_split()
        s.set_cutoff(1.5 * LAM, 2.5 * LAM)
        s.set_cutoff(0.0, 0.0)
        assert s.pair_split() == split
        plain.step(5)
        s.step(5)
        for a, b in zip(plain.get_state()[:3], s.get_state()[:3]):
            assert np.array_equal(a, b)


def test_cutoff_errors(B):
    w = W.single_grain_small()
    with B.System(w, precision=B.PREC_FP64) as s:
        with pytest.raises(B.OdError):
            s.set_cutoff(LAM, 2 * LAM)
    with B.System(w) as s:
        with pytest.raises(B.OdError):
            s.set_cutoff(2 * LAM, 2 * LAM)
        with pytest.raises(B.OdError):
            s.cutoff_info()
        s.set_cutoff(LAM, 2 * LAM)
        with pytest.raises(B.OdError):
            s.set_pair_split(2)
