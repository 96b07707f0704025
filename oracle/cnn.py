"""FP64 NumPy oracle of the learned pose initialiser (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP kernels.

The network is not in the paper; it replaces the start pose of the paper's
coarse-to-fine Gauss-Newton (Sec. IV-A) with a learned guess.  Shape:
input 2 x 60 x 94 (reference and current coarsest pyramid level, (I - 128) / 64),
four 3x3 stride-2 padding-1 convolutions with ReLU (2-16-32-64-64 channels:
30x47, 15x24, 8x12, 4x6), global average pool, FC 64-64 with ReLU, FC 64-6.
The output is the reference-to-current twist (omega, v) divided by
(5 deg, 5 deg, 5 deg, 0.1 m, 0.1 m, 0.1 m).  Loss: mean squared error over
the 6 outputs and the batch.  Optimiser: Adam.

Everything here is written directly from those definitions: a convolution is
the explicit sum over input channels and the 3x3 window of the zero-padded
input, its gradients are the same sums taken with respect to each operand.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 16, 32, 64, 64)
HIDDEN = 64
OUT = 6
TWIST_SCALE = np.array([np.deg2rad(5.0)] * 3 + [0.1] * 3)
PARAM_NAMES = ("w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4", "fw1", "fb1", "fw2", "fb2")


def conv_out(n: int) -> int:
    """Output size of a 3x3, stride-2, padding-1 convolution."""
    return (n + 2 - 3) // 2 + 1


def init_params(seed: int = 0) -> dict:
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for i in range(4):
        ci, co = CHANNELS[i], CHANNELS[i + 1]
        p[f"w{i + 1}"] = rng.normal(0.0, np.sqrt(2.0 / (ci * 9)), (co, ci, 3, 3))
        p[f"b{i + 1}"] = np.zeros(co)
    p["fw1"] = rng.normal(0.0, np.sqrt(2.0 / 64), (HIDDEN, 64))
    p["fb1"] = np.zeros(HIDDEN)
    p["fw2"] = rng.normal(0.0, np.sqrt(1.0 / HIDDEN), (OUT, HIDDEN))
    p["fb2"] = np.zeros(OUT)
    return p


def normalise(pair_u8: np.ndarray) -> np.ndarray:
    """uint8 (B, 2, 60, 94) -> (I - 128) / 64."""
    return (pair_u8.astype(np.float64) - 128.0) / 64.0


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, o, i, j] = b[o] + sum_{c, u, v} w[o, c, u, v] xp[n, c, 2i + u, 2j + v], xp = x zero-padded by 1."""
    N, C, H, W = x.shape
    O = w.shape[0]
    Ho, Wo = conv_out(H), conv_out(W)
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    y = np.zeros((N, O, Ho, Wo)) + b[None, :, None, None]
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2]  # (N, C, Ho, Wo)
            y += np.einsum("oc,ncij->noij", w[:, :, u, v], patch)
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, dy: np.ndarray):
    """Gradients of conv_forward with respect to x, w and b."""
    N, C, H, W = x.shape
    Ho, Wo = dy.shape[2], dy.shape[3]
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2]
            dw[:, :, u, v] = np.einsum("noij,ncij->oc", dy, patch)
            dxp[:, :, u:u + 2 * Ho:2, v:v + 2 * Wo:2] += np.einsum("oc,noij->ncij", w[:, :, u, v], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, db


def forward(p: dict, x: np.ndarray):
    """Network output (B, 6) and the activations backward() needs."""
    acts = [x]
    h = x
    for i in range(4):
        z = conv_forward(h, p[f"w{i + 1}"], p[f"b{i + 1}"])
        h = np.maximum(z, 0.0)
        acts.append(h)
    g = h.mean(axis=(2, 3))  # global average pool
    z1 = g @ p["fw1"].T + p["fb1"]
    h1 = np.maximum(z1, 0.0)
    out = h1 @ p["fw2"].T + p["fb2"]
    return out, {"acts": acts, "g": g, "h1": h1}


def mse(out: np.ndarray, target: np.ndarray):
    """Mean squared error over batch and outputs, and its gradient."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(p: dict, cache: dict, dout: np.ndarray) -> dict:
    g, h1, acts = cache["g"], cache["h1"], cache["acts"]
    grads = {"fw2": dout.T @ h1, "fb2": dout.sum(axis=0)}
    dh1 = dout @ p["fw2"]
    dz1 = dh1 * (h1 > 0)
    grads["fw1"] = dz1.T @ g
    grads["fb1"] = dz1.sum(axis=0)
    dg = dz1 @ p["fw1"]
    h = acts[4]
    dh = np.broadcast_to(dg[:, :, None, None] / (h.shape[2] * h.shape[3]), h.shape).copy()
    for i in range(3, -1, -1):
        dz = dh * (acts[i + 1] > 0)
        dx, dw, db = conv_backward(acts[i], p[f"w{i + 1}"], dz)
        grads[f"w{i + 1}"], grads[f"b{i + 1}"] = dw, db
        dh = dx
    return grads


def adam_step(p: dict, grads: dict, m: dict, v: dict, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t counts from 1."""
    for k in PARAM_NAMES:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def n_params(p: dict) -> int:
    return int(sum(p[k].size for k in PARAM_NAMES))
