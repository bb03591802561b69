"""Oracle pin: the FP64 backpropagation of the surrogate network equals
central finite differences of its loss."""
import numpy as np

from oracle import mlp_oracle as M


def test_param_count():
    assert M.N_PARAMS == 35856


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(size=M.N_PARAMS) * 0.15
    X = rng.uniform(-1, 1, size=(7, 5))
    T = rng.normal(size=(7, 16))
    L, g = M.loss_grad(p, X, T)
    assert abs(L - M.loss(p, X, T)) < 1e-14
    h = 1e-6
    idx = np.concatenate([rng.choice(M.N_PARAMS, 300, replace=False),
                          np.arange(0, 5), np.arange(640, 645), np.arange(35840, 35856)])
    # central differences carry ~eps*L/h ~ 1e-10 of rounding: absolute floor 2e-9
    big = 0
    for k in idx:
        e = np.zeros(M.N_PARAMS)
        e[k] = h
        fd = (M.loss(p + e, X, T) - M.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * abs(g[k]) + 2e-9, (k, fd, g[k])
        big += abs(g[k]) > 1e-6
    assert big > len(idx) // 2


def test_forward_is_the_network():
    # a network with one nonzero path reduces to a scalar composition
    p = np.zeros(M.N_PARAMS)
    layers = M.unpack(p)
    layers[0][0][2, 3] = 0.7
    layers[0][1][3] = 0.1
    layers[1][0][3, 5] = -1.3
    layers[2][0][5, 9] = 0.4
    layers[3][0][9, 11] = 2.0
    layers[3][1][11] = -0.25
    x = np.array([[0.0, 0.0, 0.6, 0.0, 0.0]])
    Y, _ = M.forward(p, x)
    expect = 2.0 * np.tanh(0.4 * np.tanh(-1.3 * np.tanh(0.7 * 0.6 + 0.1))) - 0.25
    assert abs(Y[0, 11] - expect) < 1e-15
    assert np.abs(np.delete(Y[0], 11)).max() == 0.0


def test_adam_constant_gradient_moves_by_the_learning_rate():
    # Kingma & Ba: with bias correction, a constant gradient g gives
    # m_hat = g and v_hat = g^2 at every step, so each step moves the
    # parameter by lr * g / (|g| + eps), whatever the step number.
    lr, eps = 0.01, 1e-8
    for g0 in (2.0, -0.5, 3e-4):
        p = np.array([1.0])
        m, v = np.zeros(1), np.zeros(1)
        for t in range(1, 6):
            q = M.adam_step(p, [g0], m, v, t, lr)
            assert abs((p - q)[0] - lr * g0 / (abs(g0) + eps)) < 1e-15
            p = q


def test_adam_sign_reversal_by_hand():
    # gradients g then -g: after step 2, m = -(1 - b1)^2 g, v = (1 - b2)(1 + b2) g^2,
    # so m_hat = -(1 - b1) g / (1 + b1), v_hat = g^2 and the second step moves
    # the parameter by +lr (1 - b1)/(1 + b1) sign(g) (eps = 0).
    lr, b1, b2 = 0.1, 0.9, 0.999
    g = 1.7
    p = np.array([0.0])
    m, v = np.zeros(1), np.zeros(1)
    p1 = M.adam_step(p, [g], m, v, 1, lr, b1, b2, eps=0.0)
    assert abs(p1[0] + lr) < 1e-15
    p2 = M.adam_step(p1, [-g], m, v, 2, lr, b1, b2, eps=0.0)
    assert abs((p2 - p1)[0] - lr * (1 - b1) / (1 + b1)) < 1e-15
    assert abs(m[0] + (1 - b1) ** 2 * g) < 1e-15
    assert abs(v[0] - (1 - b2) * (1 + b2) * g * g) < 1e-15
