"""Pins of the FP64 CNN oracle: torch's float64 CPU convolution as a library
special case, finite differences of every parameter tensor, the parameter count,
and Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import cnn


def test_shapes_and_parameter_count():
    p = cnn.init_params(0)
    assert cnn.n_params(p) == 64918
    x = np.zeros((2, 2, 60, 94))
    out, cache = cnn.forward(p, x)
    assert out.shape == (2, 6)
    assert [a.shape[2:] for a in cache["acts"][1:]] == [(30, 47), (15, 24), (8, 12), (4, 6)]


def test_conv_matches_torch_float64():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 5, 13, 17))
    w = rng.normal(size=(7, 5, 3, 3))
    b = rng.normal(size=7)
    y = cnn.conv_forward(x, w, b)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    yt = torch.nn.functional.conv2d(xt, wt, bt, stride=2, padding=1)
    np.testing.assert_allclose(y, yt.detach().numpy(), atol=1e-12)
    dy = rng.normal(size=y.shape)
    yt.backward(torch.tensor(dy))
    dx, dw, db = cnn.conv_backward(x, w, dy)
    np.testing.assert_allclose(dx, xt.grad.numpy(), atol=1e-11)
    np.testing.assert_allclose(dw, wt.grad.numpy(), atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-11)


def test_network_matches_torch_autograd():
    p = cnn.init_params(3)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 2, 60, 94))
    tgt = rng.normal(size=(4, 6))
    out, cache = cnn.forward(p, x)
    loss, dout = cnn.mse(out, tgt)
    g = cnn.backward(p, cache, dout)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    h = torch.tensor(x)
    for i in range(4):
        h = torch.relu(torch.nn.functional.conv2d(h, tp[f"w{i+1}"], tp[f"b{i+1}"], stride=2, padding=1))
    h = h.mean(dim=(2, 3))
    h = torch.relu(h @ tp["fw1"].T + tp["fb1"])
    o = h @ tp["fw2"].T + tp["fb2"]
    tl = torch.nn.functional.mse_loss(o, torch.tensor(tgt))
    tl.backward()
    assert abs(loss - tl.item()) < 1e-12
    for k in cnn.PARAM_NAMES:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-12)


def test_gradients_finite_differences():
    p = cnn.init_params(5)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(2, 2, 60, 94))
    tgt = rng.normal(size=(2, 6))

    def loss_of(q):
        return cnn.mse(cnn.forward(q, x)[0], tgt)[0]

    out, cache = cnn.forward(p, x)
    g = cnn.backward(p, cache, cnn.mse(out, tgt)[1])
    h = 1e-6
    for k in cnn.PARAM_NAMES:
        flat = p[k].reshape(-1)
        for j in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + h
            lp = loss_of(p)
            flat[j] = old - h
            lm = loss_of(p)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(fd)), (k, j, fd, g[k].reshape(-1)[j])


def test_adam_matches_torch():
    p = cnn.init_params(7)
    rng = np.random.default_rng(7)
    grads = [{k: rng.normal(size=v.shape) for k, v in p.items()} for _ in range(3)]
    tp = {k: torch.tensor(v.copy(), requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    for t, g in enumerate(grads, 1):
        cnn.adam_step(p, g, m, v, t)
        opt.zero_grad()
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-10, atol=1e-12)
