"""GPU test of od_mlp_predict_noalloc, the surrogate inference entry point
for callers that cannot allocate: through the C-ABI on device buffers, its
outputs and inside flags must equal od_mlp_predict's bit for bit, on two
calls in a row (the second with fewer rows, so that stale rows of the
shared buffer would show), and it must reject more rows than its buffer
holds."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_noalloc_predict_equals_predict():
    import torch
    from paper_2205_06557_amd import binding as B
    rng = np.random.default_rng(21)
    net = B.Mlp(5)
    lo = np.array([0.3, 2e-6, 0.25, 0.02, 10.0])
    hi = np.array([2.0, 10e-6, 1.0, 0.3, 100.0])
    net.set_normalization(lo, hi, rng.normal(size=16), 0.5 + rng.uniform(size=16))
    net.set_params((rng.normal(size=B.MLP_PARAMS) * 0.2).astype(np.float32))
    dev = torch.device("cuda:0")
    for n in (1000, 300):
        X = (lo + (hi - lo) * rng.uniform(-0.1, 1.1, size=(n, 5))).astype(np.float32)
        say("noalloc predict rows", n)
        Y_ref, in_ref = net.predict(X)
        Xd = torch.from_numpy(X).to(dev)
        Yd = torch.full((n, 16), float("nan"), dtype=torch.float32, device=dev)
        Id = torch.full((n,), -7, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        net.predict_noalloc(Xd.data_ptr(), n, Yd.data_ptr(), Id.data_ptr())
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        ins = Id.cpu().numpy()
        assert np.array_equal(Y, Y_ref), np.abs(Y - Y_ref).max()
        assert np.array_equal(ins.astype(bool), in_ref) and set(np.unique(ins)) <= {0, 1}
        assert (~in_ref).any() and in_ref.any()
    # without inside flags
    Yd2 = torch.zeros((300, 16), dtype=torch.float32, device=dev)
    net.predict_noalloc(Xd.data_ptr(), 300, Yd2.data_ptr(), None)
    torch.cuda.synchronize()
    assert np.array_equal(Yd2.cpu().numpy(), Y_ref)
    with pytest.raises(B.OdError):
        net.predict_noalloc(Xd.data_ptr(), 1025, Yd2.data_ptr(), None)
