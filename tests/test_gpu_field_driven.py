"""GPU parity of the field-driven collisional flow (initial and injected v_z
from the flow's stationary distribution) against the FP64 oracle, plus the
stationarity property at a size the oracle does not reach."""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import say, shadow_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


def _fd(w):
    return w.with_(flags=int(w.flags) | W.FLAG_FIELD_DRIVEN)


def test_init_matches_oracle(B):
    w = _fd(W.single_grain_small().with_(n_ions=5000))
    with B.System(w) as s:
        x, v, q, _ = s.get_state()
    o = O.Oracle(w)
    xo, vo, _, _ = o.get_state()
    lam, cs = o.derived["lam"], o.derived["cs"]
    assert np.allclose(x.T, xo / lam, rtol=2 * 2.0 ** -23, atol=1e-12)
    assert np.allclose(v.T, vo / cs, rtol=2 * 2.0 ** -23, atol=1e-12)


@pytest.mark.parametrize("mach", [1.0, 0.4])
def test_shadowed_steps_with_reinjections(B, mach):
    w = _fd(W.single_grain_small().with_(n_ions=1 << 13, mach=mach))
    say("field-driven wall shell, Mach", mach)
    with B.System(w) as s:
        o = O.Oracle(w)
        x, v = W.wall_shell_state(w, w.n_ions)
        s.set_state(x.T / o.derived["lam"], v.T / o.derived["cs"], None, 11)
        r = shadow_step(s, o, w)
        say("  ", r)
        assert r["n_exit"] > 1000
        for _ in range(2):
            say("  ", shadow_step(s, o, w))


def test_shadowed_steps_two_grains(B):
    w = _fd(W.two_grain_wake().with_(n_ions=3000))
    with B.System(w) as s:
        o = O.Oracle(w)
        s.step(20)
        for _ in range(2):
            say("  two grains", shadow_step(s, o, w))


def test_stationary_flow_at_size(B):
    base = W.single_grain_small()
    w = _fd(base.with_(n_ions=1 << 16, dust=[], flags=W.FLAG_NO_ION_ION, nu_in=0.5 * base.wpi,
                       charge_mode=W.CHARGE_GIVEN, n_discard=0, seed=21))
    with B.System(w) as s:
        s.step(1500)
        x, v, _, _ = s.get_state()
        H = w.H / s.units["length"]
    cnt, _ = np.histogram(x[2] / H + 0.5, bins=8, range=(0, 1))
    e = x.shape[1] / 8
    chi2 = float(((cnt - e) ** 2 / e).sum())
    o = O.Oracle(w, init=False)
    ufd, sig = o.derived["ufd"] / o.derived["cs"], o.derived["sig"] / o.derived["cs"]
    p = stats.kstest(v[2].astype(np.float64), stats.exponnorm(K=ufd / sig, scale=sig).cdf).pvalue
    say("stationary flow: chi2", chi2, "KS p", p, "counts", cnt.tolist())
    assert chi2 < 30.0 and p > 1e-3


def test_batch_member_equals_single(B):
    base = W.single_grain_small()
    ws = [_fd(base.with_(n_ions=1800, system_id=0)), base.with_(n_ions=1200, system_id=1),
          _fd(base.with_(n_ions=2500, system_id=2, mach=0.7))]
    steps = 25
    with B.Batch(ws) as b:
        b.set_config(persistent=True, jsplit=1, split_max_n=0)
        b.step(steps)
        b.sync()
        got = [(*b.get_state(s)[:3], b.forces(s, 0)) for s in range(len(ws))]
    for s, w in enumerate(ws):
        with B.System(w) as single:
            single.set_pair_split(1)
            single.step(steps)
            x, v, q, _ = single.get_state()
            ref = (x, v, q, single.forces(0))
        for a, r in zip(got[s], ref):
            assert np.array_equal(np.asarray(a), np.asarray(r)), (s, w.name)


def test_needs_collisions(B):
    w = _fd(W.single_grain_small().with_(nu_in=0.0))
    with pytest.raises(B.OdError) as e:
        B.System(w)
    assert e.value.status == B.OD_EINVAL
