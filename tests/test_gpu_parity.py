"""GPU parity: the HIP path against the FP64 oracle, through the C-ABI.

Protocol: the GPU state is loaded into the oracle and both advance one step
(a "shadowed" step); accelerations, dust forces, collision decisions,
absorbed/exited sets, charges and the post-step state are compared (see
tests/gpu_util.py for the tolerances).  Cases cover the small single-grain
workload, multi-grain layouts, ragged and minimal ion counts, many
absorptions, many exits and reinjections, the FP64 mode and sampled outputs
at 2^20 ions.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import say, shadow_step, to_oracle, accel_errors
from tests.test_oracle_rng import numpy_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


def test_device_rng_matches_numpy(B):
    rng = np.random.default_rng(1)
    for _ in range(64):
        ctr = [int(x) for x in rng.integers(0, 2**62, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**62, size=2, dtype=np.int64)]
        assert list(B.rng_block(key[0], key[1], ctr)) == list(numpy_block(ctr, key))


def test_init_state_matches_oracle(B):
    w = W.single_grain_small()
    say("init parity", w.name)
    with B.System(w) as s:
        x, v, q, step = s.get_state()
        o = O.Oracle(w)
        xo, vo, qo, so = o.get_state()
        lam, cs = o.derived["lam"], o.derived["cs"]
        assert step == 0 and so == 0
        assert np.allclose(x.T, xo / lam, rtol=2 * 2.0**-23, atol=1e-12)
        assert np.allclose(v.T, vo / cs, rtol=2 * 2.0**-23, atol=1e-12)
        assert np.array_equal(q, qo)
        assert s.units["length"] == pytest.approx(lam, rel=1e-14)
        assert s.units["velocity"] == pytest.approx(cs, rel=1e-14)


@pytest.mark.parametrize("n_ions", [2000, 2, 257, 1037])
def test_shadowed_steps_single_grain(B, n_ions):
    w = W.single_grain_small().with_(n_ions=n_ions)
    say("shadowed steps", w.name, "N", n_ions)
    with B.System(w) as s:
        o = O.Oracle(w)
        for k in range(3):
            r = shadow_step(s, o, w)
            say("  step", k, r)
        s.step(40)
        r = shadow_step(s, o, w)
        say("  after 40 free steps", r)


def test_shadowed_steps_two_grains_and_chain(B):
    w2 = W.two_grain_wake().with_(n_ions=4096)
    w8 = W.chain8(n_ions=3000)
    for w in (w2, w8):
        say("shadowed steps", w.name)
        with B.System(w) as s:
            o = O.Oracle(w)
            for k in range(2):
                r = shadow_step(s, o, w)
                say("  ", r)


def test_many_absorptions(B):
    lam = W.single_grain_small().lam
    w = W.single_grain_small().with_(n_ions=1 << 14, dust=[(0.0, 0.0, 0.0, 50e-6, -2e4 * W.QE)])
    say("absorption shell", w.name)
    with B.System(w) as s:
        o = O.Oracle(w)
        x, v = W.absorption_shell_state(w, w.n_ions)
        s.set_state(x.T / lam, v.T / o.derived["cs"], np.array([-2e4 * W.QE]), 5)
        r = shadow_step(s, o, w)
        say("  ", r)
        assert r["n_abs"][0] > 200
        # the absorbed-ion list against the oracle's events
        idx, by, na, ne = s.absorbed()
        ev = o.last_step()["ev"]
        ref = np.nonzero(ev >= 0)[0]
        assert na == r["n_abs"][0] and ne == r["n_exit"]
        if r["n_ambiguous_mismatch"] == 0:
            assert np.array_equal(idx, ref) and np.array_equal(by, ev[ref])
        idx2, _, na2, _ = s.absorbed(cap=10)
        assert na2 == na and np.array_equal(idx2, idx[:10])
        r = shadow_step(s, o, w)
        say("  ", r)


# up to 16384 ions the tail kernel reinjects lost ions itself, above that a
# separate kernel walks the list of lost ions
@pytest.mark.parametrize("n_ions", [1 << 13, 20000])
def test_many_exits_and_reinjections(B, n_ions):
    w = W.single_grain_small().with_(n_ions=n_ions, mach=0.5)
    say("wall shell", w.name, "N", n_ions)
    with B.System(w) as s:
        o = O.Oracle(w)
        x, v = W.wall_shell_state(w, w.n_ions)
        s.set_state(x.T / o.derived["lam"], v.T / o.derived["cs"], None, 11)
        r = shadow_step(s, o, w)
        say("  ", r)
        assert r["n_exit"] > n_ions // 8


def test_test_particle_mode_and_literal_side(B):
    w = W.single_grain_small().with_(n_ions=3000, flags=W.FLAG_NO_ION_ION | W.FLAG_LITERAL_SIDE,
                                     charge_mode=W.CHARGE_OML)
    with B.System(w) as s:
        o = O.Oracle(w)
        s.step(30)
        r = shadow_step(s, o, w)
        say("test-particle", r)


def test_fp64_mode(B):
    w = W.single_grain_small()
    with B.System(w, precision=B.PREC_FP64) as s:
        o = O.Oracle(w)
        s.step(5)
        r = shadow_step(s, o, w, acc_tol=1e-11, force_tol=1e-9)
        say("fp64", r)


def test_sampled_outputs_at_full_size(B):
    w = W.two_grain_wake()
    N = w.n_ions
    say("full size", w.name, N)
    with B.System(w) as s:
        s.step(2)
        o = O.Oracle(w, init=False)
        x0, v0, q0, n0 = to_oracle(s, o)
        s.step(1)
        s.sync()
        a = s.accelerations().T.astype(np.float64)
        lam, wpi = o.derived["lam"], o.derived["wpi"]
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(N, size=512, replace=False))
        a_ref = o.accel_subset(idx)
        l2, p999, pmax = accel_errors(a[idx] * lam * wpi * wpi, a_ref)
        say("  sampled accel errors", l2, p999, pmax)
        assert l2 <= 1e-5 and p999 <= 1e-5
        F = s.forces(0)
        Fo = o.dust_forces()
        for d in range(2):
            for p in (0, 1, 3):
                assert np.linalg.norm(F[d, p] - Fo[d, p]) <= 1e-5 * np.linalg.norm(Fo[d, p])


def test_errors_from_host_checks(B):
    w = W.single_grain_small()
    with B.System(w) as s:
        x, v, q, st = s.get_state()
        bad = x.copy()
        bad[0, 5] = np.nan
        with pytest.raises(B.OdError) as e:
            s.set_state(bad, None, None, st)
        assert e.value.status == B.OD_ENUMERIC
        inside = x.copy()
        inside[:, 7] = 0.0          # the grain sits at the origin
        with pytest.raises(B.OdError) as e:
            s.set_state(inside, None, None, st)
        assert e.value.status == B.OD_ESTATE
        s.step(2)
        s.sync()


def test_bitwise_reproducible(B):
    w = W.single_grain_small().with_(n_ions=3000)
    res = []
    for _ in range(2):
        with B.System(w) as s:
            s.step(25)
            x, v, q, _ = s.get_state()
            res.append((x.copy(), v.copy(), q.copy(), s.forces(0).copy()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
