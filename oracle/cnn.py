"""FP64 oracle of the warm-start CNN (test infrastructure only).

The network maps a normalised dirty plane to a reconstruction: four 3x3
convolutions 1 -> F -> F -> F -> 1 with circular padding, bias, ReLU after the
first three layers, and the positive-orthant projection applied to its output
when it is used as a starting point.  Convolutions are cross-correlations:

    y[b, o, i, j] = bias[o] + sum_c sum_{a, e in {-1, 0, 1}} w[o, c, a+1, e+1] x[b, c, i+a, j+e]

with indices taken modulo N.  Each function is the plain sum over the nine taps,
one channel contraction per tap, in FP64.  Inputs that the GPU holds in BF16
are passed in already rounded (``bf16_round``), so the two sides see the same
operands and differ only in accumulation order.
"""
from __future__ import annotations

import numpy as np

TAPS = [(a, e) for a in (-1, 0, 1) for e in (-1, 0, 1)]


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via the FP32 bit pattern; returns float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _shift(x: np.ndarray, a: int, e: int) -> np.ndarray:
    """s[..., i, j] = x[..., i + a, j + e] (periodic)."""
    return np.roll(x, shift=(-a, -e), axis=(-2, -1))


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x (B, C, N, N), w (O, C, 3, 3), b (O,) -> (B, O, N, N)."""
    B, C, N, _ = x.shape
    O = w.shape[0]
    y = np.broadcast_to(b[None, :, None, None], (B, O, N, N)).astype(np.float64).copy()
    for a, e in TAPS:
        xs = _shift(x, a, e)
        y += np.einsum("oc,bcij->boij", w[:, :, a + 1, e + 1], xs)
    return y


def conv_data_grad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Transpose of conv_forward in x: dx[b, c, i, j] = sum_o sum_taps w[o, c, a, e] dy[b, o, i-a, j-e]."""
    B, O, N, _ = dy.shape
    C = w.shape[1]
    dx = np.zeros((B, C, N, N))
    for a, e in TAPS:
        dys = _shift(dy, -a, -e)
        dx += np.einsum("oc,boij->bcij", w[:, :, a + 1, e + 1], dys)
    return dx


def conv_weight_grad(x: np.ndarray, dy: np.ndarray):
    """(dw, db): dw[o, c, a, e] = sum_{b,i,j} dy[b, o, i, j] x[b, c, i+a, j+e], db[o] = sum dy[:, o]."""
    O, C = dy.shape[1], x.shape[1]
    dw = np.zeros((O, C, 3, 3))
    for a, e in TAPS:
        dw[:, :, a + 1, e + 1] = np.einsum("boij,bcij->oc", dy, _shift(x, a, e))
    return dw, dy.sum(axis=(0, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(F: int = 32, seed: int = 0):
    """He-normal weights, zero biases, for the 1 -> F -> F -> F -> 1 network."""
    rng = np.random.default_rng(seed)
    shapes = [(F, 1), (F, F), (F, F), (1, F)]
    params = []
    for o, c in shapes:
        std = np.sqrt(2.0 / (9 * c))
        params.append((rng.normal(0.0, std, size=(o, c, 3, 3)), np.zeros(o)))
    return params


def forward(params, x: np.ndarray, bf16: bool = True):
    """Network forward on (B, 1, N, N); returns (output, list of layer inputs).

    With ``bf16`` the weights, the input and every hidden activation are rounded
    to bfloat16 (the layer output is accumulated in full precision first); the
    final output stays unrounded.
    """
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = rnd(x)
    acts = []
    n = len(params)
    for i, (w, b) in enumerate(params):
        acts.append(h)
        z = conv_forward(h, rnd(w), b)
        h = rnd(relu(z)) if i < n - 1 else z
    return h, acts


def mse(pred: np.ndarray, target: np.ndarray):
    """(loss, dloss/dpred) of mean((pred - target)^2)."""
    r = pred - target
    return float(np.mean(r * r)), 2.0 * r / r.size


def backward(params, acts, dout: np.ndarray, bf16: bool = True):
    """Gradients of every (w, b) given d(loss)/d(output); ReLU masks come from the stored inputs."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(params)
    g = rnd(dout)
    for i in reversed(range(len(params))):
        w, _ = params[i]
        x = acts[i]
        grads[i] = conv_weight_grad(x, g)
        if i > 0:
            g = conv_data_grad(g, rnd(w))
            g = g * (x > 0)  # x = relu(previous pre-activation), so x > 0 marks the active units
            g = rnd(g) if bf16 else g
    return grads


def adam_update(param, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on FP64 arrays; returns (param, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v
