"""GPU tests of the surrogate network kernels (matrix-core products, FP32)
against the FP64 CPU reference, training behaviour, and a miniature run of
the surrogate pipeline (solver-generated data -> training -> prediction with
fallback flags -> warm start)."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2205_06557_amd import surrogate as S
from paper_2205_06557_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2205_06557_amd import binding
    binding.lib()
    return binding


def _identity_norm(net):
    net.set_normalization(-np.ones(5), np.ones(5), np.zeros(16), np.ones(16))


def test_forward_matches_fp64_reference(B):
    rng = np.random.default_rng(1)
    net = B.Mlp(3)
    _identity_norm(net)
    p = (rng.normal(size=M.N_PARAMS) * 0.2).astype(np.float32)
    net.set_params(p)
    X = rng.uniform(-1, 1, size=(1000, 5)).astype(np.float32)
    Y, inside = net.predict(X)
    Yr, _ = M.forward(p.astype(np.float64), X.astype(np.float64))
    err = np.linalg.norm(Y - Yr) / np.linalg.norm(Yr)
    say("forward rel err", err)
    assert err < 2e-6
    assert inside.all()
    Y2, inside2 = net.predict(np.array([[1.5, 0, 0, 0, 0]], dtype=np.float32))
    assert not inside2[0]


def test_gradients_match_fp64_reference(B):
    rng = np.random.default_rng(2)
    net = B.Mlp(4)
    p = (rng.normal(size=M.N_PARAMS) * 0.15).astype(np.float32)
    net.set_params(p)
    X = rng.uniform(-1, 1, size=(256, 5)).astype(np.float32)
    T = rng.normal(size=(256, 16)).astype(np.float32)
    L, g = net.loss_grad(X, T)
    Lr, gr = M.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert L == pytest.approx(Lr, rel=1e-5)
    k = 0
    for (i, o) in M.SIZES:
        for n in (i * o, o):
            a, r = g[k:k + n], gr[k:k + n]
            err = np.linalg.norm(a - r) / np.linalg.norm(r)
            say("grad tensor", k, n, err)
            assert err < 1e-4
            k += n


def test_training_fits_smooth_function_and_is_reproducible(B):
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, size=(2048, 5))
    A = rng.normal(size=(5, 16))
    T = np.sin(X @ A) + 0.3 * X[:, :1] ** 2
    hist = []
    params = []
    for _ in range(2):
        net = B.Mlp(7)
        _identity_norm(net)
        h = net.train(X, T, epochs=60, batch=128, lr=3e-3, lr_final=1e-4, seed=9)
        hist.append(h)
        params.append(net.params())
    say("loss first/last", hist[0][0], hist[0][-1])
    assert hist[0][-1] < hist[0][0] / 30
    assert np.array_equal(params[0], params[1])
    assert np.array_equal(hist[0], hist[1])


def test_miniature_surrogate_pipeline(B):
    X = S.sweep_inputs(12, 5)
    T = S.run_plain(X, n_ions=512, steps=60, seed=5, batch_size=12, graph=10)
    assert np.isfinite(T).all()
    assert (T[:, :8] < 0).all()                       # grains charge negatively
    sur = S.Surrogate.train(X, T, epochs=40, batch=12, seed=1)
    Q, F, inside = sur.predict(X)
    assert inside.all() and np.isfinite(Q).all() and np.isfinite(F).all()
    _, _, ins = sur.predict(np.array([[2.5, 5.0, 0.5, 0.1, 30.0]]))
    assert not ins[0]                                 # outside the box: fall back
    # warm start of a chain from the predicted charges
    w = S.chain_workload(X[0], 1024, 20, 1, 0, Q[0])
    with B.System(w) as s:
        q0, _ = s.charges()
        assert np.allclose(q0, Q[0])
        s.step(20)
        s.sync()


def test_adam_steps_match_fp64_reference(B):
    # two od_mlp_train steps (the whole set as one batch, constant learning
    # rate) against the FP64 Adam of Kingma & Ba fed with the GPU's own
    # gradients (tight), and the first step with the FP64 reference gradients
    # (loose: FP32 gradients).  The GPU's training gathers the rows in a
    # shuffled order, so its gradient differs from od_mlp_loss_grad's by the
    # summation order (~1e-7 relative), which moves an update noticeably only
    # where |g| is near Adam's eps = 1e-8 (none is here: min |g| ~ 2e-7).
    rng = np.random.default_rng(8)
    net = B.Mlp(6)
    _identity_norm(net)
    p0 = (rng.normal(size=M.N_PARAMS) * 0.15).astype(np.float32)
    net.set_params(p0)
    # inputs on a 1/64 grid: the [-1, 1] normalisation maps them exactly
    X = (rng.integers(-64, 65, size=(256, 5)) / 64.0).astype(np.float32)
    T = rng.normal(size=(256, 16)).astype(np.float32)
    lr = 1e-3
    _, g0 = net.loss_grad(X, T)
    net.train(X, T, epochs=1, batch=256, lr=lr, lr_final=lr, seed=1)
    p1 = net.params()
    _, g1 = net.loss_grad(X, T)
    net.train(X, T, epochs=1, batch=256, lr=lr, lr_final=lr, seed=2)   # moments carried over
    p2 = net.params()
    m, v = np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    r1 = M.adam_step(p0, g0, m, v, 1, lr)
    r2 = M.adam_step(p1, g1, m, v, 2, lr)
    ulp = 2e-7 * np.abs(p0).max()
    for k, (got, ref) in enumerate(((p1, r1), (p2, r2)), start=1):
        d = np.abs(got - ref)
        say("adam step", k, "max", d.max() / lr, "p99.9", np.percentile(d, 99.9) / lr, "(units of lr)")
        assert d.max() < 2e-3 * lr + ulp
        assert np.percentile(d, 99.9) < 1e-3 * lr + ulp
    # the second step depends on the first step's moments: a fresh optimiser
    # from p1 would move differently
    fresh = M.adam_step(p1, g1, np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), 1, lr)
    assert np.percentile(np.abs(fresh - r2), 50) > 5e-3 * lr
    # against FP64 gradients: relative size of the update difference
    _, gr = M.loss_grad(p0.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    rr = M.adam_step(p0, gr, np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), 1, lr)
    d_gpu, d_ref = p1.astype(np.float64) - p0, rr - p0
    rel = np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref)
    say("adam step 1 vs FP64 gradients, relative L2 of the update difference", rel)
    assert rel < 1e-2


def test_surrogate_train_and_predict_calls(B):
    # the two-call surrogate interface: standardised by the data, trained,
    # and predicting as od_mlp_predict does
    import ctypes as C
    L = B._mlp_lib()
    rng = np.random.default_rng(12)
    X = rng.uniform(-1, 1, size=(512, 5)).astype(np.float32)
    Y = (np.sin(X @ rng.normal(size=(5, 16))) * 3.0 + 5.0).astype(np.float32)
    lo, hi = -np.ones(5, dtype=np.float32), np.ones(5, dtype=np.float32)
    cfg = B.TrainCfg(60, 64, 3e-3, 1e-4, 1)
    h = C.c_void_p()
    fp = C.POINTER(C.c_float)
    B._check(L.od_surrogate_train(X.ctypes.data_as(fp), Y.ctypes.data_as(fp), 512, lo.ctypes.data_as(fp),
                                  hi.ctypes.data_as(fp), C.byref(cfg), 3, None, C.byref(h)))
    try:
        Yp = np.zeros((512, 16), dtype=np.float32)
        ins = np.zeros(512, dtype=np.int32)
        B._check(L.od_surrogate_predict(h, X.ctypes.data_as(fp), 512, Yp.ctypes.data_as(fp),
                                        ins.ctypes.data_as(C.POINTER(C.c_int32))))
        Yq = np.zeros((512, 16), dtype=np.float32)
        B._check(L.od_mlp_predict(h, X.ctypes.data_as(fp), 512, Yq.ctypes.data_as(fp), None))
        assert np.array_equal(Yp, Yq) and ins.all()
        err = np.sqrt(np.mean((Yp - Y) ** 2)) / Y.std()
        say("surrogate train/predict relative rms error", err)
        assert err < 0.5          # the mean alone gives 1
    finally:
        L.od_mlp_destroy(h)
