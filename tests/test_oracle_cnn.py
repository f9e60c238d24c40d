"""Pins of the warm-start CNN oracle: FFT correlation, adjoint identities, brute-force
weight gradients, finite differences, bfloat16 rounding and the first Adam step."""
import numpy as np
import pytest
import torch

from oracle import cnn


def rng(s=0):
    return np.random.default_rng(s)


def test_conv_forward_equals_fft_circular_correlation():
    B, C, O, N = 2, 3, 4, 8
    x = rng(1).normal(size=(B, C, N, N))
    w = rng(2).normal(size=(O, C, 3, 3))
    b = rng(3).normal(size=O)
    y = cnn.conv_forward(x, w, b)
    ref = np.zeros_like(y)
    X = np.fft.fft2(x)
    for o in range(O):
        acc = np.zeros((B, N, N), dtype=complex)
        for c in range(C):
            k = np.zeros((N, N))
            for a in (-1, 0, 1):
                for e in (-1, 0, 1):
                    k[a % N, e % N] = w[o, c, a + 1, e + 1]
            acc += X[:, c] * np.conj(np.fft.fft2(k))
        ref[:, o] = np.real(np.fft.ifft2(acc)) + b[o]
    np.testing.assert_allclose(y, ref, atol=1e-12)


def test_conv_tap_orientation():
    """A single tap w[0, 0, 0, 2] (a = -1, e = +1) reads x[i - 1, j + 1]."""
    N = 6
    x = rng(4).normal(size=(1, 1, N, N))
    w = np.zeros((1, 1, 3, 3))
    w[0, 0, 0, 2] = 1.0
    y = cnn.conv_forward(x, w, np.zeros(1))
    for i in range(N):
        for j in range(N):
            assert y[0, 0, i, j] == x[0, 0, (i - 1) % N, (j + 1) % N]


def test_data_grad_is_adjoint():
    B, C, O, N = 2, 3, 5, 8
    x = rng(5).normal(size=(B, C, N, N))
    w = rng(6).normal(size=(O, C, 3, 3))
    dy = rng(7).normal(size=(B, O, N, N))
    lhs = np.sum(cnn.conv_forward(x, w, np.zeros(O)) * dy)
    rhs = np.sum(x * cnn.conv_data_grad(dy, w))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_weight_grad_brute_force():
    B, C, O, N = 2, 2, 3, 6
    x = rng(8).normal(size=(B, C, N, N))
    dy = rng(9).normal(size=(B, O, N, N))
    dw, db = cnn.conv_weight_grad(x, dy)
    for o in range(O):
        for c in range(C):
            for a in range(3):
                for e in range(3):
                    E = np.zeros((O, C, 3, 3))
                    E[o, c, a, e] = 1.0
                    ref = np.sum(cnn.conv_forward(x, E, np.zeros(O)) * dy)
                    assert dw[o, c, a, e] == pytest.approx(ref, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 2, 3)), rtol=1e-12)


def test_network_backward_matches_finite_differences():
    params = cnn.init_params(F=4, seed=3)
    x = rng(10).normal(size=(2, 1, 6, 6))
    target = rng(11).normal(size=(2, 1, 6, 6))

    def loss(ps):
        out, _ = cnn.forward(ps, x, bf16=False)
        return cnn.mse(out, target)[0]

    out, acts = cnn.forward(params, x, bf16=False)
    _, dout = cnn.mse(out, target)
    grads = cnn.backward(params, acts, dout, bf16=False)
    h = 1e-6
    r = rng(12)
    for li in range(len(params)):
        for which in (0, 1):
            for _ in range(3):
                arr = params[li][which]
                idx = tuple(r.integers(0, s) for s in arr.shape)
                plus = [(w.copy(), b.copy()) for w, b in params]
                minus = [(w.copy(), b.copy()) for w, b in params]
                plus[li][which][idx] += h
                minus[li][which][idx] -= h
                fd = (loss(plus) - loss(minus)) / (2 * h)
                an = grads[li][which][idx]
                assert an == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_bf16_round_matches_torch_and_ties_to_even():
    v = rng(13).normal(scale=10.0, size=10000)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(v), ref)
    assert cnn.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    assert cnn.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_first_adam_step_has_learning_rate_size():
    g = np.array([3.0, -0.02, 1e-3])
    p, m, v = cnn.adam_update(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
