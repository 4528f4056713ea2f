"""GPU parity of the BF16-MFMA network kernels against the oracle with
bfloat16 rounding emulated at the same storage points.

Tolerance.  bf16 x bf16 products are exact in FP32, so a single contraction
differs from the FP64 oracle only by FP32 accumulation rounding.  Across
layers that rounding can flip the bf16 rounding of an activation or gradient
(probability ~1e-4 per element), which moves a few rows by ~2^-8 relative.
Hence: relative Frobenius error <= 1e-3 for outputs and gradients, and most
rows agreeing to 1e-5.
"""
import numpy as np
import pytest

import paper_1307_6489_amd as rta
from oracle import mlp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rta.lib()
    return torch.device("cuda:0")


def t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def rel_fro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def make(dev, seed, B, scale=1.0):
    rng = np.random.default_rng(seed)
    theta = (mlp.init_params(seed) * scale).astype(np.float32)
    x = rng.normal(size=(B, 10)).astype(np.float32)
    lab = (rng.random(B) < 0.4).astype(np.float32)
    y = rng.normal(size=B).astype(np.float32)
    net = rta.Mlp(max_batch=max(B, 64))
    net.set_params(theta, np.zeros(10), np.ones(10))
    return net, theta.astype(np.float64), x, lab, y


@pytest.mark.parametrize("B", [1, 37, 1000, 4096])
def test_forward_parity(dev, B):
    say("forward parity B=%d seed 5" % B)
    net, theta, x, lab, y = make(dev, 5, B)
    out = net.forward(t(x, dev)).cpu().numpy()
    ref, _ = mlp.forward(theta, x.astype(np.float64))
    assert rel_fro(out, ref) <= 1e-3
    close = np.all(np.abs(out - ref) <= 1e-5 * (np.abs(ref) + 1.0), axis=1)
    assert close.mean() >= 0.8


def test_standardisation_inside_kernel(dev):
    rng = np.random.default_rng(9)
    theta = mlp.init_params(9).astype(np.float32)
    mean = rng.normal(size=10).astype(np.float32) * 5
    std = rng.uniform(0.5, 3, size=10).astype(np.float32)
    x = (rng.normal(size=(300, 10)) * std + mean).astype(np.float32)
    net = rta.Mlp(max_batch=64)
    net.set_params(theta, mean, std)
    out = net.forward(t(x, dev)).cpu().numpy()
    xs = ((x - mean) / std).astype(np.float32)   # the kernels standardise in FP32
    ref, _ = mlp.forward(theta.astype(np.float64), xs.astype(np.float64))
    assert rel_fro(out, ref) <= 1e-3


@pytest.mark.parametrize("B", [64, 1000, 4096])
def test_gradient_parity(dev, B):
    say("gradient parity B=%d seed 6" % B)
    net, theta, x, lab, y = make(dev, 6, B)
    loss, grad = net.loss_grad(t(x, dev), t(lab, dev), t(y, dev))
    L_ref, g_ref = mlp.loss_grad(theta, x.astype(np.float64), lab, y)
    assert float(loss.cpu()[0]) == pytest.approx(L_ref, rel=1e-4)
    g = grad.cpu().numpy().astype(np.float64)
    assert rel_fro(g, g_ref) <= 1e-3
    off = 0
    for name, shp in mlp.SHAPES:
        n = int(np.prod(shp))
        assert rel_fro(g[off:off + n], g_ref[off:off + n]) <= 5e-3, name
        off += n


def test_adam_step_parity(dev):
    """One train step = the GPU's own gradient fed to the oracle's Adam."""
    import torch
    net, theta, x, lab, y = make(dev, 7, 512)
    xd, ld, yd = t(x, dev), t(lab, dev), t(y, dev)
    opt = mlp.Adam(mlp.N_PARAMS)
    th = theta.copy()
    for step in range(3):
        _, grad = net.loss_grad(xd, ld, yd)
        g = grad.cpu().numpy().astype(np.float64)
        net.train_step(xd, ld, yd)
        th = opt.step(th, g)
        got = net.get_params().astype(np.float64)
        assert np.max(np.abs(got - th)) <= 1e-6 + 1e-5 * np.max(np.abs(th)), step
        th = got


def test_params_roundtrip(dev):
    theta = mlp.init_params(11).astype(np.float32)
    net = rta.Mlp(max_batch=64)
    net.set_params(theta, np.zeros(10), np.ones(10))
    assert np.array_equal(net.get_params(), theta)


def test_training_learns_a_separable_problem(dev):
    """Labels from a fixed hyperplane, energy linear in two features: the loss
    falls by more than 5x within 400 Adam steps."""
    import torch
    rng = np.random.default_rng(12)
    B = 2048
    net = rta.Mlp(max_batch=B, lr=3e-3)
    net.set_params(mlp.init_params(12).astype(np.float32), np.zeros(10), np.ones(10))
    loss = torch.zeros(1, device=dev)
    first = None
    for step in range(400):
        x = rng.normal(size=(B, 10)).astype(np.float32)
        lab = (x[:, 0] + 0.5 * x[:, 3] > 0).astype(np.float32)
        y = (0.7 * x[:, 1] - 0.3 * x[:, 2]).astype(np.float32)
        net.train_step(t(x, dev), t(lab, dev), t(y, dev), loss_out=loss)
        if step == 0:
            first = float(loss.cpu()[0])
    last = float(loss.cpu()[0])
    say("training loss %.4f -> %.4f" % (first, last))
    assert last < first / 5


@pytest.mark.parametrize("B", [1, 100, 4096])
def test_train_step_gathering_rows(dev, B):
    """A step on rows of data arrays gathered in the kernel equals, bit for
    bit, the step on the arrays gathered beforehand: parameters and loss
    after three steps, with repeated rows and rows outside [0, n) clamped to
    the first / last row."""
    import torch
    say("train step gathering rows B=%d seed 9" % B)
    n = 5000
    a, theta, x, lab, y = make(dev, 9, n)
    b = rta.Mlp(max_batch=n)
    b.set_params(theta.astype(np.float32), np.zeros(10), np.ones(10))
    X, L, Y = t(x, dev), t(lab, dev), t(y, dev)
    rng = np.random.default_rng(B)
    la, lb = torch.zeros(1, device=dev), torch.zeros(1, device=dev)
    for step in range(3):
        rows = rng.integers(-3, n + 3, size=B).astype(np.int64)
        rows[: B // 4] = rows[B // 2: B // 2 + B // 4]
        r = np.clip(rows, 0, n - 1)
        a.train_step(X[r].contiguous(), L[r].contiguous(), Y[r].contiguous(), loss_out=la)
        b.train_step(X, L, Y, loss_out=lb, rows=torch.from_numpy(rows).to(dev))
        assert np.array_equal(a.get_params(), b.get_params()), step
        assert torch.equal(la, lb), step


def test_train_step_rows_rejects_bad_args(dev):
    import torch
    net, theta, x, lab, y = make(dev, 9, 64)
    X, L, Y = t(x, dev), t(lab, dev), t(y, dev)
    with pytest.raises(TypeError):
        net.train_step(X, L, Y, rows=torch.zeros(8, dtype=torch.int32, device=dev))
    with pytest.raises(rta.RTAError):
        net.train_step(X, L, Y, rows=torch.zeros(0, dtype=torch.int64, device=dev))
    with pytest.raises(rta.RTAError):
        net.train_step(X, L, Y, rows=torch.zeros(65, dtype=torch.int64, device=dev))
