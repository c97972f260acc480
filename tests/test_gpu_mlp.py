"""The picker network's HIP kernels (forward, masked-MSE gradient, Adam)
against the FP64 reference of oracle.mlp_ref."""
import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1307_2100_amd as tc  # noqa: E402

DIMS = (32, 64, 15)


def _case(seed, batch, dims=DIMS):
    rng = np.random.default_rng(seed)
    p = mlp_ref.init_params(rng, *dims)
    p += 0.05 * rng.standard_normal(p.size)   # nonzero biases too
    X = rng.standard_normal((batch, dims[0]))
    T = rng.standard_normal((batch, dims[2]))
    M = (rng.uniform(size=(batch, dims[2])) < 0.8).astype(np.float64)
    return p, X, T, M


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _net(p, dims, max_batch):
    net = tc.MLP(*dims, max_batch)
    assert net.num_params == mlp_ref.num_params(*dims)
    net.set_params(p.astype(np.float32))
    return net


@pytest.mark.parametrize("batch", [1, 37, 300])
def test_forward_matches_reference(batch):
    p, X, _, _ = _case(1, batch)
    net = _net(p, DIMS, 300)
    p32 = p.astype(np.float32).astype(np.float64)   # the reference sees the same rounded weights
    X32 = X.astype(np.float32).astype(np.float64)
    ref, _ = mlp_ref.forward(p32, X32, *DIMS)
    got = net.forward(_dev(X)).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))
    net.close()


@pytest.mark.parametrize("seed,batch", [(2, 5), (3, 256), (4, 300)])
def test_gradient_matches_reference(seed, batch):
    p, X, T, M = _case(seed, batch)
    net = _net(p, DIMS, 300)
    p32 = p.astype(np.float32).astype(np.float64)
    X32, T32 = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    loss_ref, g_ref = mlp_ref.loss_and_grad(p32, X32, T32, M, *DIMS)
    loss, g = net.loss_grad(_dev(X), _dev(T), _dev(M))
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - loss_ref) <= 1e-5 * loss_ref
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))
    net.close()


def test_adam_step_matches_reference():
    p, X, T, M = _case(5, 128)
    net = _net(p, DIMS, 128)
    p32 = p.astype(np.float32).astype(np.float64)
    X32, T32 = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    pr, m, v = p32, np.zeros_like(p32), np.zeros_like(p32)
    lr = 1e-3
    for step in (1, 2, 3):
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        net.train_step(_dev(X), _dev(T), _dev(M), lr, loss=loss)
        _, g = mlp_ref.loss_and_grad(pr, X32, T32, M, *DIMS)
        pr, m, v = mlp_ref.adam_step(pr, g, m, v, step, lr)
    got = np.array(net.get_params(), dtype=np.float64)
    # the update of a weight with a gradient near zero is g / (|g| + eps): sensitive, leave those out
    _, g_last = mlp_ref.loss_and_grad(pr, X32, T32, M, *DIMS)
    steady = np.abs(g_last) > 1e-3 * np.max(np.abs(g_last))
    assert np.max(np.abs(got - pr)[steady]) <= 2e-2 * lr
    net.close()


def test_training_reduces_loss_and_sizes_are_checked():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((512, 32))
    W = rng.standard_normal((32, 15)) / 6
    T = np.tanh(X @ W)
    M = np.ones_like(T)
    net = tc.MLP(32, 64, 15, 256)
    net.set_params(mlp_ref.init_params(rng, *DIMS).astype(np.float32))
    Xd, Td, Md = _dev(X), _dev(T), _dev(M)
    first, _ = net.loss_grad(Xd[:256], Td[:256], Md[:256])
    first = float(first.item())
    for it in range(400):
        b = (it % 2) * 256
        net.train_step(Xd[b:b + 256], Td[b:b + 256], Md[b:b + 256], 3e-3)
    last, _ = net.loss_grad(Xd[:256], Td[:256], Md[:256])
    assert float(last.item()) < 0.1 * first
    with pytest.raises(tc.TCError):
        net.loss_grad(Xd, Td, Md)           # 512 rows > max_batch 256
    # a smaller batch right after a larger one
    y1 = net.forward(Xd[:3]).cpu().numpy()
    y2 = net.forward(Xd[:256]).cpu().numpy()[:3]
    np.testing.assert_array_equal(y1, y2)
    net.close()
