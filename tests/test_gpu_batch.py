"""GPU tests of the batched path: many systems of uneven N in one launch per
phase.  A system in a batch must reproduce, bit for bit, the same system run
alone when its pair sum is not split; split sums, persistent vs one-block-per-
item scheduling and graph replay are checked against that, and batched
systems are checked against the FP64 oracle with the shadowed-step protocol.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import say, shadow_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


def _systems():
    base = W.single_grain_small()
    out = []
    specs = [(300, 0.6, 4e-6, 0.05), (1037, 1.0, 5e-6, 0.1), (2048, 1.7, 9e-6, 0.25),
             (777, 0.35, 2.5e-6, 0.02), (4096, 1.2, 6e-6, 0.3), (2600, 2.0, 7e-6, 0.12)]
    for s, (n, mach, a, nu) in enumerate(specs):
        out.append(base.with_(n_ions=n, mach=mach, nu_in=nu * base.wpi, system_id=s, seed=3,
                              dust=[(0.0, 0.0, 0.0, a, 0.0)], name=f"sys{s}"))
    # one two-grain system in the mix
    out.append(W.two_grain_wake().with_(n_ions=3000, system_id=len(out), seed=3))
    return out


def _run_single(B, w, steps, nsplit=1):
    with B.System(w) as s:
        s.set_pair_kernel(B.PAIR_ONE_SIDED)
        s.set_pair_split(nsplit)
        s.step(steps)
        x, v, q, st = s.get_state()
        return x, v, q, s.forces(0), st


def _run_batch(B, ws, steps, **cfg):
    """The one-sided kernel with the given decomposition."""
    with B.Batch(ws) as b:
        b.set_pair_kernel(B.PAIR_ONE_SIDED)
        graph = cfg.pop("graph", 0)
        if cfg:
            b.set_config(**cfg)
        if graph:
            b.set_graph(graph)
        b.step(steps)
        b.sync()
        return [(*b.get_state(s)[:3], b.forces(s, 0), b.get_state(s)[3]) for s in range(len(ws))]


def test_batch_equals_single_bitwise(B):
    ws = _systems()
    steps = 12
    say("batch vs single:", [w.n_ions for w in ws])
    got = _run_batch(B, ws, steps, persistent=True, jsplit=1, split_max_n=0)
    for s, w in enumerate(ws):
        ref = _run_single(B, w, steps)
        for a, r in zip(got[s], ref):
            assert np.array_equal(np.asarray(a), np.asarray(r)), (s, w.name)


def test_scheduling_and_graph_replay_bitwise(B):
    ws = _systems()
    steps = 11
    ref = _run_batch(B, ws, steps, persistent=True, jsplit=1, split_max_n=0)
    for cfg in (dict(persistent=False, jsplit=1, split_max_n=0),
                dict(persistent=True, jsplit=1, split_max_n=0, graph=4)):
        got = _run_batch(B, ws, steps, **cfg)
        for s in range(len(ws)):
            for a, r in zip(got[s], ref[s]):
                assert np.array_equal(np.asarray(a), np.asarray(r)), (cfg, s)


def test_split_sums_close_to_unsplit(B):
    ws = _systems()
    with B.Batch(ws) as b1, B.Batch(ws) as b4:
        for b in (b1, b4):
            b.set_pair_kernel(B.PAIR_ONE_SIDED)
        b1.set_config(True, 1, 0)
        b4.set_config(True, 4, 1 << 20)
        for s in range(len(ws)):
            assert b4.sizes(s)["nsplit"] > 1
        b1.step(1)
        b4.step(1)
        for s in range(len(ws)):
            a1 = b1.accelerations(s).astype(np.float64)
            a4 = b4.accelerations(s).astype(np.float64)
            err = np.linalg.norm(a1 - a4) / np.linalg.norm(a1)
            assert err < 1e-6, (s, err)


def test_batched_systems_match_oracle(B):
    ws = _systems()
    with B.Batch(ws) as b:
        b.set_pair_kernel(B.PAIR_ONE_SIDED)
        b.set_config(True, 2, 1 << 20)
        b.step(3)
        for s in (0, 2, 6):
            o = O.Oracle(ws[s])
            r = shadow_step(B.BatchMember(b, s), o, ws[s])
            say("  batch member", s, r)


def test_autotune_keeps_state_and_caches(B, tmp_path):
    ws = _systems()
    cache = str(tmp_path / "tune.jsonl")
    with B.Batch(ws) as b:
        b.step(2)
        before = [b.get_state(s) for s in range(len(ws))]
        ms = b.autotune(cache)
        cfg = b.config()
        kind = b.pair_kernel()
        say("autotune", ms, cfg, "pair kernel", kind)
        assert ms > 0 and os.path.exists(cache)
        after = [b.get_state(s) for s in range(len(ws))]
        for x, y in zip(before, after):
            for a, c in zip(x, y):
                assert np.array_equal(np.asarray(a), np.asarray(c))
        b.step(2)
        b.sync()
    with B.Batch(ws) as b2:
        ms2 = b2.autotune(cache)
        assert ms2 == pytest.approx(ms, rel=1e-6)
        assert b2.config()["jsplit"] == cfg["jsplit"]
        assert b2.pair_kernel() == kind
        assert len(open(cache).read().strip().splitlines()) == 1
