"""Surrogate network kernels (BF16 matrix cores, FP32 accumulation and
master weights) against the FP64 CPU reference with the same BF16 rounding
points.  Tolerance: relative norm error <= 1e-2 (bfloat16 unit roundoff is
2^-8; accumulation order differs)."""
import math

import numpy as np
import pytest

from oracle import mlp as OL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = (15, 256, 256, 256, 1)


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_06938_amd import dalia
    dalia.lib()
    return dalia


def _setup(D, n=300, seed=0):
    rng = np.random.default_rng(seed)
    params = [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
              for i, o in zip(SIZES[:-1], SIZES[1:])]
    net = D.MLP(SIZES, max_batch=512)
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])
    net.params.copy_(torch.from_numpy(flat.astype(np.float32)))
    # the reference uses the same FP32-representable weights
    params = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
              for W, b in params]
    X = rng.standard_normal((n, SIZES[0])).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return net, params, X, y


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30)


def test_forward_backward_input_gradient(D):
    net, params, X, y = _setup(D)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    yhat = net.forward(Xd)
    dy, loss = net.mse_grad(yd)
    net.backward(dy)
    torch.cuda.synchronize()
    ref_y, cache = OL.forward(params, X.astype(np.float64), bf16=True)
    assert _rel(yhat.cpu().numpy(), ref_y) <= 1e-2
    r = ref_y - y
    assert abs(loss.item() - np.mean(r * r)) <= 1e-2 * np.mean(r * r)
    grads, _ = OL.backward(params, cache, 2.0 * r / len(y), bf16=True)
    flat_ref = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    assert _rel(net.grads.cpu().numpy(), flat_ref) <= 1e-2
    # per layer as well (a misplaced block would hide in the global norm)
    off = 0
    for (gW, gb) in grads:
        nW = gW.size
        assert _rel(net.grads[off:off + nW].cpu().numpy(), gW.ravel()) <= 2e-2
        off += nW + gb.size
    # input gradient: dy = 1
    net.forward(Xd)
    dX = net.backward(torch.ones(len(y), device="cuda", dtype=torch.float32), want_dx=True)
    torch.cuda.synchronize()
    _, dX_ref = OL.input_gradient(params, X.astype(np.float64), bf16=True)
    assert _rel(dX.cpu().numpy(), dX_ref) <= 1e-2


def test_adam_step_matches_reference(D):
    net, params, X, y = _setup(D, seed=1)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    net.forward(Xd)
    dy, _ = net.mse_grad(yd)
    net.backward(dy)
    g = net.grads.cpu().numpy().astype(np.float64)
    w0 = net.params.cpu().numpy().astype(np.float64)
    net.adam(lr=1e-3)
    torch.cuda.synchronize()
    p = [(w0.copy(), np.zeros(1))]
    OL.adam(p, [(g, np.zeros(1))], {}, lr=1e-3)
    np.testing.assert_allclose(net.params.cpu().numpy(), p[0][0], rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(D):
    net, params, X, _ = _setup(D, seed=2, n=256)
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2 - X[:, 2] * X[:, 3]
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y.astype(np.float32)).cuda()
    losses = []
    for it in range(300):
        net.forward(Xd)
        dy, loss = net.mse_grad(yd)
        net.backward(dy)
        net.adam(lr=2e-3)
        if it % 50 == 0:
            losses.append(loss.item())
    torch.cuda.synchronize()
    net.forward(Xd)
    _, loss = net.mse_grad(yd)
    assert loss.item() < 0.2 * losses[0]
