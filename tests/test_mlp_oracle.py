"""Pins of the FP64 picker-network reference (oracle.mlp_ref), CPU only."""
import numpy as np

from oracle import mlp_ref

DIMS = (5, 7, 3)


def _case(seed, batch=6, dims=DIMS):
    rng = np.random.default_rng(seed)
    p = mlp_ref.init_params(rng, *dims)
    p[dims[0] * dims[1]:dims[0] * dims[1] + dims[1]] = rng.uniform(-0.3, 0.3, dims[1])  # nonzero b0
    X = rng.standard_normal((batch, dims[0]))
    T = rng.standard_normal((batch, dims[2]))
    M = (rng.uniform(size=(batch, dims[2])) < 0.7).astype(np.float64)
    M[0, 0] = 1.0
    return p, X, T, M


def test_parameter_count():
    # 5*7 + 7 + 7*7 + 7 + 7*3 + 3
    assert mlp_ref.num_params(*DIMS) == 122
    assert mlp_ref.num_params(32, 64, 15) == 7247


def test_gradient_matches_central_differences():
    for seed in range(3):
        p, X, T, M = _case(seed)
        _, g = mlp_ref.loss_and_grad(p, X, T, M, *DIMS)
        h = 1e-6
        fd = np.empty_like(p)
        for i in range(p.size):
            e = np.zeros_like(p)
            e[i] = h
            fd[i] = (mlp_ref.loss_and_grad(p + e, X, T, M, *DIMS)[0] -
                     mlp_ref.loss_and_grad(p - e, X, T, M, *DIMS)[0]) / (2 * h)
        assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_forward_reduces_to_a_linear_map():
    # W0 = [I 0], W1 = I, b = 0: for x >= 0 both ReLUs pass everything, so y = x[:3] W2' + b2
    n_in, hidden, n_out = 3, 4, 2
    W0 = np.zeros((n_in, hidden))
    W0[:, :n_in] = np.eye(n_in)
    W1 = np.eye(hidden)
    W2 = np.array([[1.0, 2.0], [3.0, -1.0], [0.5, 0.25], [9.0, 9.0]])
    b2 = np.array([0.5, -2.0])
    p = np.concatenate([W0.ravel(), np.zeros(hidden), W1.ravel(), np.zeros(hidden), W2.ravel(), b2])
    X = np.array([[1.0, 2.0, 4.0], [0.0, 0.0, 0.0]])
    y, _ = mlp_ref.forward(p, X, n_in, hidden, n_out)
    # first row: (1*1 + 2*3 + 4*0.5 + 0.5, 1*2 - 2*1 + 4*0.25 - 2)
    np.testing.assert_array_equal(y, [[9.5, -1.0], [0.5, -2.0]])
    # negative inputs are cut by the first ReLU
    y2, _ = mlp_ref.forward(p, -X, n_in, hidden, n_out)
    np.testing.assert_array_equal(y2, [[0.5, -2.0], [0.5, -2.0]])


def test_masked_loss_counts_only_masked_entries():
    Y = np.array([[1.0, 5.0], [2.0, -3.0]])
    T = np.array([[0.0, 100.0], [4.0, 7.0]])
    M = np.array([[1.0, 0.0], [1.0, 0.0]])
    assert mlp_ref.masked_mse(Y, T, M) == (1.0 + 4.0) / 2
    assert mlp_ref.masked_mse(Y, T, np.zeros_like(M)) == 0.0
    # masked-out targets do not move the gradient
    p, X, T2, M2 = _case(7)
    T3 = T2.copy()
    T3[M2 == 0] += 1e3
    g2 = mlp_ref.loss_and_grad(p, X, T2, M2, *DIMS)[1]
    g3 = mlp_ref.loss_and_grad(p, X, T3, M2, *DIMS)[1]
    np.testing.assert_array_equal(g2, g3)


def test_adam_first_step_and_constant_gradient():
    p0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.25, -4.0, 1e-3, 0.0])
    lr = 0.01
    # with bias correction, step one moves each weight by lr * g / (|g| + eps)
    p1, m, v = mlp_ref.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr)
    np.testing.assert_allclose(p1, p0 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the corrected moments at g and g^2 at every step
    p = p1
    for t in range(2, 11):
        p, m, v = mlp_ref.adam_step(p, g, m, v, t, lr)
    np.testing.assert_allclose(p, p0 - 10 * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_adam_hand_checked_second_step():
    # g1 = 1, g2 = -1, lr = 1: m2 = 0.9*0.1 - 0.1 = -0.01, v2 = 0.999*0.001 + 0.001 = 0.001999
    # m_hat = -0.01/0.19, v_hat = 0.001999/0.001999 = 1 -> update = +0.0526315...
    p1, m, v = mlp_ref.adam_step(np.array([0.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, 1.0, eps=0.0)
    assert p1[0] == -1.0
    p2, m, v = mlp_ref.adam_step(p1, np.array([-1.0]), m, v, 2, 1.0, eps=0.0)
    np.testing.assert_allclose(m, [-0.01], rtol=1e-14)
    np.testing.assert_allclose(v, [0.001999], rtol=1e-14)
    np.testing.assert_allclose(p2, [-1.0 + 0.01 / 0.19], rtol=1e-13)


def test_training_fits_a_separable_target():
    # plain gradient descent with the reference gradient fits a linear target
    rng = np.random.default_rng(3)
    dims = (4, 16, 2)
    p = mlp_ref.init_params(rng, *dims)
    X = rng.standard_normal((64, 4))
    T = X @ np.array([[1.0, -1.0], [0.5, 0.0], [0.0, 2.0], [-1.0, 1.0]])
    M = np.ones_like(T)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    first = mlp_ref.loss_and_grad(p, X, T, M, *dims)[0]
    for t in range(1, 801):
        loss, g = mlp_ref.loss_and_grad(p, X, T, M, *dims)
        p, m, v = mlp_ref.adam_step(p, g, m, v, t, 1e-2)
    assert loss < 0.02 * first
