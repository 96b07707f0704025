"""Learned initialiser on the GPU (BF16 MFMA forward and backward with FP32
accumulation, Adam) against the FP64 oracle.

Two references: the FP64 oracle itself (per layer and per gradient tensor:
cosine > 0.999 / relative error < 2e-2 for activations; for gradients the
bound BF16 activation storage allows, cosine > 0.998 / relative error < 6e-2,
measured on this data as 4.6e-2 for the first layer by the FP64 emulation
below), and the oracle's own layers evaluated in FP64 with every stored
activation and every gradient passed between convolution layers rounded to
BF16 as the GPU stores them, which must agree to FP32 accumulation rounding
(cosine > 0.99999, relative error < 2e-3)."""
import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cos(a, b):
    a, b = a.reshape(-1), b.reshape(-1)
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


def _data(B, seed=0):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 256, (B, 60, 94)).astype(np.float64)
    # smooth-ish images so activations are not all noise
    k = np.ones(5) / 5
    for ax in (1, 2):
        base = np.apply_along_axis(lambda v: np.convolve(v, k, mode="same"), ax, base)
    cur = np.roll(base, 1, axis=2) + rng.normal(0, 2, base.shape)
    pairs = np.clip(np.stack([base, cur], axis=1), 0, 255).astype(np.uint8)
    tgt = rng.normal(0, 0.5, (B, 6))
    return pairs, tgt


def _bf16(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def setup(gpu_lib):
    dpt = gpu_lib
    p = ocnn.init_params(11)
    for i in range(1, 5):  # nonzero biases exercise the bias paths
        p[f"b{i}"] = np.random.default_rng(i).normal(0, 0.05, p[f"b{i}"].shape)
    net = dpt.Cnn(max_batch=64)
    net.set_params(p)
    return dpt, net, p


def test_forward_matches_oracle(setup):
    dpt, net, p = setup
    pairs, _ = _data(16)
    out = net.forward(pairs)
    # oracle on the same (BF16-rounded) conv weights, FP64 arithmetic
    q = {k: (_bf16(v) if k.startswith("w") else v) for k, v in p.items()}
    o, cache = ocnn.forward(q, ocnn.normalise(pairs))
    for l in range(1, 5):
        g = net.activation(l, 16)                       # NHWC
        r = cache["acts"][l].transpose(0, 2, 3, 1)      # NCHW -> NHWC
        print(f"layer {l}: cos {_cos(g, r):.6f} rel {_rel(g, r):.2e}")
        assert _cos(g, r) > 0.999 and _rel(g, r) < 2e-2
    print(f"out: cos {_cos(out, o):.6f} rel {_rel(out, o):.2e}")
    assert _cos(out, o) > 0.999 and _rel(out, o) < 2e-2


def _bf16_storage_grads(q, x, tgt):
    """Oracle layers in FP64, with activations and the gradients flowing
    between convolution layers rounded to BF16 where the GPU stores them."""
    acts, h = [x], x
    for i in range(4):
        h = _bf16(np.maximum(ocnn.conv_forward(h, q[f"w{i + 1}"], q[f"b{i + 1}"]), 0.0))
        acts.append(h)
    g = h.mean(axis=(2, 3))
    h1 = np.maximum(g @ q["fw1"].T + q["fb1"], 0.0)
    out = h1 @ q["fw2"].T + q["fb2"]
    loss, dout = ocnn.mse(out, tgt)
    grads = {"fw2": dout.T @ h1, "fb2": dout.sum(axis=0)}
    dz1 = (dout @ q["fw2"]) * (h1 > 0)
    grads["fw1"], grads["fb1"] = dz1.T @ g, dz1.sum(axis=0)
    dh = np.broadcast_to((dz1 @ q["fw1"])[:, :, None, None] / (h.shape[2] * h.shape[3]), h.shape)
    for i in range(3, -1, -1):
        dz = _bf16(dh * (acts[i + 1] > 0))
        dh, grads[f"w{i + 1}"], grads[f"b{i + 1}"] = ocnn.conv_backward(acts[i], q[f"w{i + 1}"], dz)
    return loss, grads


@pytest.mark.parametrize("B", [32, 5])
def test_gradients_match_oracle(setup, B):
    dpt, net, p = setup
    pairs, tgt = _data(B, seed=1)
    loss = net.train_step(pairs, tgt, lr=0.0)
    g = dpt.cnn_unflatten(net.get_grads())
    q = {k: (_bf16(v) if k.startswith("w") else v) for k, v in p.items()}
    x = ocnn.normalise(pairs)
    o, cache = ocnn.forward(q, x)
    lo, dout = ocnn.mse(o, tgt)
    og = ocnn.backward(q, cache, dout)
    le, eg = _bf16_storage_grads(q, x, tgt)
    assert abs(loss - lo) / lo < 2e-2 and abs(loss - le) / le < 1e-4
    for k in ocnn.PARAM_NAMES:
        print(f"{k}: vs oracle cos {_cos(g[k], og[k]):.6f} rel {_rel(g[k], og[k]):.2e}; "
              f"vs BF16-storage cos {_cos(g[k], eg[k]):.7f} rel {_rel(g[k], eg[k]):.2e}")
        assert _cos(g[k], eg[k]) > 0.99999 and _rel(g[k], eg[k]) < 2e-3, k
        # the distance from the oracle is the one BF16 storage explains
        assert _rel(g[k], og[k]) <= _rel(eg[k], og[k]) + 2e-3, k
        if B == 32:  # the data the fixed bound was measured on
            assert _cos(g[k], og[k]) > 0.998 and _rel(g[k], og[k]) < 6e-2, k


def test_adam_step_matches_oracle(setup):
    dpt, net, p = setup
    net.set_params(p)  # resets the Adam state
    pairs, tgt = _data(8, seed=2)
    p0 = dpt.cnn_unflatten(net.get_params().astype(np.float64))
    net.train_step(pairs, tgt, lr=1e-3)
    g = dpt.cnn_unflatten(net.get_grads().astype(np.float64))
    p1 = dpt.cnn_unflatten(net.get_params().astype(np.float64))
    m = {k: np.zeros_like(v) for k, v in p0.items()}
    v = {k: np.zeros_like(x) for k, x in p0.items()}
    ref = {k: x.copy() for k, x in p0.items()}
    ocnn.adam_step(ref, g, m, v, 1)
    for k in ocnn.PARAM_NAMES:
        np.testing.assert_allclose(p1[k], ref[k], rtol=1e-5, atol=1e-6)
    net.set_params(p)


def test_training_reduces_loss(setup):
    dpt, net, p = setup
    net.set_params(p)
    pairs, tgt = _data(64, seed=3)
    first = net.train_step(pairs, tgt, lr=1e-3)
    for _ in range(60):
        last = net.train_step(pairs, tgt, lr=1e-3)
    assert last < 0.5 * first
    net.set_params(p)
