"""GPU parity of the symmetric all-pairs kernel (each unordered pair once,
reactions applied to the sources) against the FP64 oracle, plus its
agreement with the one-sided kernel, determinism and selection rules."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import accel_errors, say, shadow_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


# up to 4096 ions (16 tiles) the items are single 64-ion source sub-tiles,
# at 12000 (47 tiles) whole tile pairs
@pytest.mark.parametrize("n_ions", [2000, 257, 1037, 4096, 12000])
def test_shadowed_steps_symmetric(B, n_ions):
    w = W.single_grain_small().with_(n_ions=n_ions)
    say("symmetric kernel, N", n_ions)
    with B.System(w) as s:
        s.set_pair_kernel(B.PAIR_SYMMETRIC)
        assert s.pair_kernel() == B.PAIR_SYMMETRIC and s.pair_split() == 1
        o = O.Oracle(w)
        for k in range(2):
            say("  step", k, shadow_step(s, o, w))
        s.step(30)
        say("  after 30 free steps", shadow_step(s, o, w))


@pytest.mark.parametrize("n_ions", [2, 3, 255, 256, 512])
def test_smallest_and_exact_tile_systems(B, n_ions):
    """Degenerate and boundary sizes of the symmetric sum: two and three ions
    (one tile, mostly padding), one ion short of a tile, exactly one and two
    tiles (no padding): shadowed steps against the oracle."""
    w = W.single_grain_small().with_(n_ions=n_ions)
    say("smallest / exact tiles, N", n_ions)
    with B.System(w) as s:
        assert s.pair_kernel() == B.PAIR_SYMMETRIC
        o = O.Oracle(w)
        for k in range(3):
            say("  step", k, shadow_step(s, o, w))
        s.step(20)
        say("  after 20 free steps", shadow_step(s, o, w))


def test_no_grains_symmetric(B):
    """A plasma cylinder without grains (n_dust = 0): only the ion-ion sum,
    the drive and the boundary act; shadowed steps against the oracle."""
    w = W.single_grain_small().with_(n_ions=3000, dust=[])
    with B.System(w) as s:
        assert s.nd == 0 and s.pair_kernel() == B.PAIR_SYMMETRIC
        o = O.Oracle(w)
        for k in range(2):
            say("no grains, step", k, shadow_step(s, o, w))
        s.step(20)
        say("no grains, after 20 free steps", shadow_step(s, o, w))


def test_two_grains_symmetric(B):
    w = W.two_grain_wake().with_(n_ions=5000)
    with B.System(w) as s:
        s.set_pair_kernel(B.PAIR_SYMMETRIC)
        o = O.Oracle(w)
        s.step(10)
        say("two grains, symmetric", shadow_step(s, o, w))


def test_symmetric_matches_one_sided(B):
    w = W.single_grain_small().with_(n_ions=(1 << 17) + 77)
    with B.System(w) as sym, B.System(w) as one:
        assert sym.pair_kernel() == B.PAIR_SYMMETRIC          # the default
        one.set_pair_kernel(B.PAIR_ONE_SIDED)
        sym.step(1)
        one.step(1)
        a_s = sym.accelerations().astype(np.float64).T
        a_o = one.accelerations().astype(np.float64).T
        l2, p999, pmax = accel_errors(a_s, a_o)
        say("symmetric vs one-sided at 2^17+77:", l2, p999, pmax)
        assert l2 < 1e-6 and p999 < 3e-6
        Fs, Fo = sym.forces(0), one.forces(0)
        assert np.allclose(Fs[0, 0], Fo[0, 0], rtol=1e-9, atol=0)   # Eq. (1) sums do not use the pair sums


def test_symmetric_bitwise_reproducible(B):
    w = W.single_grain_small().with_(n_ions=(1 << 16) + 37)
    res = []
    for _ in range(2):
        with B.System(w) as s:
            assert s.pair_kernel() == B.PAIR_SYMMETRIC
            s.step(8)
            x, v, q, _ = s.get_state()
            res.append((x, v, q, s.accelerations()))
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_selection_rules(B):
    small = W.single_grain_small()
    with B.System(small) as s:
        assert s.pair_kernel() == B.PAIR_SYMMETRIC          # the default for FP32 with ion-ion forces
        with pytest.raises(B.OdError):
            s.set_pair_split(2)
        s.set_pair_split(1)
        s.set_pair_kernel(B.PAIR_ONE_SIDED)
        assert s.pair_kernel() == B.PAIR_ONE_SIDED
        s.set_pair_split(2)
        assert s.pair_split() == 2
        s.set_pair_kernel(B.PAIR_AUTO)
        assert s.pair_kernel() == B.PAIR_SYMMETRIC and s.pair_split() == 1
    with B.System(small, precision=B.PREC_FP64) as s:
        with pytest.raises(B.OdError):
            s.set_pair_kernel(B.PAIR_SYMMETRIC)
    # test-particle mode: the symmetric setting (the default) runs no pair
    # kernel, the one-sided one a grain-terms-only kernel
    tp = small.with_(flags=W.FLAG_NO_ION_ION)
    with B.System(tp) as s:
        assert s.pair_kernel() == B.PAIR_SYMMETRIC
        s.set_pair_kernel(B.PAIR_ONE_SIDED)
        assert s.pair_kernel() == B.PAIR_ONE_SIDED
        s.set_pair_kernel(B.PAIR_SYMMETRIC)
        assert s.pair_kernel() == B.PAIR_SYMMETRIC


def _batch_systems():
    base = W.single_grain_small()
    return [base.with_(n_ions=1500, system_id=0),
            base.with_(n_ions=4099, system_id=1, mach=0.6, nu_in=0.2 * base.wpi),
            base.with_(n_ions=700, system_id=2, flags=W.FLAG_NO_ION_ION),
            W.two_grain_wake().with_(n_ions=2600, system_id=3, seed=3),
            base.with_(n_ions=(1 << 16) + 600, system_id=4, seed=5)]    # grouped target rows


def test_batch_symmetric_equals_single(B):
    ws = _batch_systems()
    steps = 9
    with B.Batch(ws) as b:
        b.set_pair_kernel(B.PAIR_SYMMETRIC)
        assert b.pair_kernel() == B.PAIR_SYMMETRIC
        b.step(steps)
        b.sync()
        got = [(*b.get_state(s)[:3], b.forces(s, 0), b.accelerations(s)) for s in range(len(ws))]
    for s, w in enumerate(ws):
        with B.System(w) as one:
            if not (int(w.flags) & W.FLAG_NO_ION_ION):
                one.set_pair_kernel(B.PAIR_SYMMETRIC)
            one.step(steps)
            x, v, q, _ = one.get_state()
            ref = (x, v, q, one.forces(0), one.accelerations())
        for a, r in zip(got[s], ref):
            assert np.array_equal(np.asarray(a), np.asarray(r)), (s, w.name)


def test_batch_symmetric_graph_and_oracle(B):
    ws = _batch_systems()
    with B.Batch(ws) as eager, B.Batch(ws) as graph:
        for b in (eager, graph):
            b.set_pair_kernel(B.PAIR_SYMMETRIC)
        graph.set_graph(4)
        eager.step(8)
        graph.step(8)
        eager.sync()
        graph.sync()
        for s in range(len(ws)):
            for a, r in zip(eager.get_state(s)[:3], graph.get_state(s)[:3]):
                assert np.array_equal(a, r)
        m = B.BatchMember(eager, 1)
        o = O.Oracle(ws[1])
        say("batch member, symmetric", shadow_step(m, o, ws[1]))


def test_batch_symmetric_queue_and_one_row(B):
    """The symmetric batch decompositions: items pulled from the atomic queue
    by a resident grid give the same integer totals as one block per item
    (bit for bit); one target row per item changes only the FP32 partial sums
    (close to the default split, and a member against the oracle)."""
    ws = _batch_systems()
    steps = 7
    res = {}
    for cfg in ((False, False), (True, False), (True, True)):
        with B.Batch(ws) as b:
            b.set_sym_config(*cfg)
            c = b.sym_config()
            assert (c["persistent"], c["one_row"]) == cfg and c["items_target"] == 65536
            b.step(steps)
            b.sync()
            res[cfg] = [(*b.get_state(s)[:3], b.accelerations(s)) for s in range(len(ws))]
            if cfg == (True, True):
                m = B.BatchMember(b, 4)
                say("one-row batch member, 2^16 + 600 ions", shadow_step(m, O.Oracle(ws[4]), ws[4]))
    for s in range(len(ws)):
        for a, r in zip(res[(True, False)][s], res[(False, False)][s]):
            assert np.array_equal(a, r), s
    # one row per item, or fewer and longer items (a target of 512 items
    # per system changes the 2^16 + 600-ion member's split: 22 source tiles
    # per grouped item, too few such items, so one row of 66 tiles each):
    # the first step's accelerations differ from the default split's by
    # FP32 rounding of the item sums only
    with B.Batch(ws) as g, B.Batch(ws) as o, B.Batch(ws) as t:
        o.set_sym_config(False, True)
        t.set_sym_config(False, False, 512)
        assert t.sym_config()["n_items"] < g.sym_config()["n_items"]
        for b in (g, o, t):
            b.step(1)
        for s in range(len(ws)):
            for b in (o, t):
                l2, p999, _ = accel_errors(b.accelerations(s).astype(np.float64).T,
                                           g.accelerations(s).astype(np.float64).T)
                assert l2 < 1e-6 and p999 < 3e-6, (s, l2, p999)


@pytest.mark.parametrize("n_ions", [(1 << 16) + 600, (1 << 16) + 412, (1 << 16) + 900])
def test_grouped_rows_sampled_parity(B, n_ions):
    """Systems large enough for items of three target rows (259 tiles: one
    row left over; 258 tiles: none; 260 tiles: two), each with a ragged last
    tile: sampled accelerations against the oracle, the last 600 ions
    included."""
    w = W.single_grain_small().with_(n_ions=n_ions)
    say("grouped rows, N", n_ions)
    with B.System(w) as s:
        assert s.pair_kernel() == B.PAIR_SYMMETRIC
        s.step(1)
        o = O.Oracle(w, init=False)
        from tests.gpu_util import to_oracle
        to_oracle(s, o)
        s.step(1)
        s.sync()
        a = s.accelerations().T.astype(np.float64)
        lam, wpi = o.derived["lam"], o.derived["wpi"]
        rng = np.random.default_rng(n_ions)
        idx = np.unique(np.concatenate([rng.choice(n_ions - 600, size=200, replace=False),
                                        np.arange(n_ions - 600, n_ions, 5)]))
        l2, p999, pmax = accel_errors(a[idx] * lam * wpi * wpi, o.accel_subset(idx))
        say("  sampled accel errors", l2, p999, pmax)
        assert l2 <= 1e-5 and p999 <= 1e-5


def test_sampled_outputs_chain_2p21(B):
    """The largest all-pairs configuration: the 8-grain chain at 2^21 ions,
    sampled accelerations and every grain's Eq. (1) and Eq. (2) forces."""
    w = W.chain8()
    assert w.n_ions == 1 << 21
    say("chain of 8 grains", w.n_ions)
    with B.System(w) as s:
        assert s.pair_kernel() == B.PAIR_SYMMETRIC
        s.step(1)
        o = O.Oracle(w, init=False)
        from tests.gpu_util import to_oracle
        to_oracle(s, o)
        s.step(1)
        s.sync()
        a = s.accelerations().T.astype(np.float64)
        lam, wpi = o.derived["lam"], o.derived["wpi"]
        idx = np.sort(np.random.default_rng(21).choice(w.n_ions, size=256, replace=False))
        l2, p999, pmax = accel_errors(a[idx] * lam * wpi * wpi, o.accel_subset(idx))
        say("  sampled accel errors", l2, p999, pmax)
        assert l2 <= 1e-5 and p999 <= 1e-5
        F, Fo = s.forces(0), o.dust_forces()
        for d in range(8):
            for p in (0, 1, 3):
                assert np.linalg.norm(F[d, p] - Fo[d, p]) <= 1e-5 * np.linalg.norm(Fo[d, p]) + 1e-300, (d, p)


def test_fixed_point_overflow_is_reported(B):
    """Two ions 1e-12 r_De apart make a pair sum far beyond the accumulators'
    range: the step must end with OD_ENUMERIC (the kernel clamps and flags),
    not with silently wrapped sums."""
    w = W.single_grain_small().with_(n_ions=600, dust=[])
    with B.System(w) as s:
        x, v, q, st = s.get_state()
        x = x.copy()
        x[:, 0] = (0.0, 0.0, 0.5)
        x[:, 1] = (1e-12, 0.0, 0.5)
        s.set_state(x, None, None, st)
        s.step(1)
        with pytest.raises(B.OdError) as e:
            s.sync()
        assert e.value.status == B.OD_ENUMERIC
