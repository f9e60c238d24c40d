"""Pins of oracle pieces that the solver pins do not reach: the generic primal-dual step (one step
worked by hand), the SNR of Sec. 4 (closed forms), the two-step calibration of Sec. 4 (closed-form
minimisers of each step) and Adam beyond its first step (Kingma and Ba's recursion worked by hand)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cnn
from oracle import muffin as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_primal_dual_step_worked_by_hand():
    """Scalar problem f(x) = (x - 3)^2 / 2, K = 2, g = indicator of x >= 0, h = |.|, from x = 1,
    y = 0.5 with tau = 0.1, sigma = 0.2, rho = 0.5:
      p = max(1 - 0.1 ((1 - 3) + 2 * 0.5), 0) = 1.1
      q = clip(0.5 + 0.2 * 2 * (2 * 1.1 - 1), -1, 1) = 0.98
      x' = 0.5 * 1.1 + 0.5 * 1 = 1.05,  y' = 0.5 * 0.98 + 0.5 * 0.5 = 0.74.
    Using p or x' in place of the extrapolated point 2p - x, or dropping the relaxation, changes
    the result."""
    x, (y,) = om.primal_dual_step(np.array(1.0), (np.array(0.5),), lambda v: v - 3.0, lambda v: (2.0 * v,),
                                  lambda u: 2.0 * u, om.positive, om.l1_conj_prox, 0.1, 0.2, 0.5)
    assert float(x) == pytest.approx(1.05, abs=1e-15)
    assert float(y) == pytest.approx(0.74, abs=1e-15)


def test_primal_dual_step_converges_to_soft_threshold():
    """min (x - a)^2 / 2 + lam |x| over x >= 0 has the minimiser max(a - lam, 0) entry by entry."""
    a = np.array([2.0, 0.3, -1.0, 0.75])
    lam = 0.5
    x, y = np.zeros(4), (np.zeros(4),)
    for _ in range(3000):
        x, y = om.primal_dual_step(x, y, lambda v: v - a, lambda v: (lam * v,), lambda u: lam * u, om.positive,
                                   om.l1_conj_prox, 0.5, 1.0, 1.0)
    np.testing.assert_allclose(x, np.maximum(a - lam, 0.0), atol=1e-10)


def test_snr_closed_forms():
    # ||X*||^2 = 25, ||X - X*||^2 = 0.25: 10 log10(100) = 20 dB
    assert om.snr_db(np.array([3.0, 4.5]), np.array([3.0, 4.0])) == pytest.approx(20.0, abs=1e-12)
    r = np.random.default_rng(0)
    T = r.normal(size=(3, 8, 8))
    for eps in (0.1, -0.03, 1e-4):
        assert om.snr_db((1.0 + eps) * T, T) == pytest.approx(-20.0 * np.log10(abs(eps)), rel=1e-10)
    # an error orthogonal to the truth of a chosen energy
    E = r.normal(size=T.shape)
    E -= np.sum(E * T) / np.sum(T * T) * T
    E *= np.sqrt(np.sum(T * T) / 1000.0) / np.linalg.norm(E)  # ||E||^2 = ||T||^2 / 1000
    assert om.snr_db(T + E, T) == pytest.approx(30.0, rel=1e-10)
    # the truth is the reference: swapping the arguments changes the value
    assert om.snr_db(T, 2.0 * T) != pytest.approx(om.snr_db(2.0 * T, T))


def test_adam_three_steps_worked_by_hand():
    g = json.load(open(os.path.join(GOLDEN, "adam_three_steps.json")))
    frac = lambda s: float(Fraction(s))
    theta = 0.0
    ref = []
    for t in range(3):
        theta -= g["lr"] * frac(g["mhat"][t]) / np.sqrt(frac(g["vhat"][t]))
        ref.append(theta)
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t, gr in enumerate(g["grads"], start=1):
        p, m, v = cnn.adam_update(p, np.array([gr]), m, v, t=t, lr=g["lr"], b1=g["b1"], b2=g["b2"], eps=g["eps"])
        assert m[0] == pytest.approx(frac(g["m"][t - 1]), abs=1e-15)
        assert v[0] == pytest.approx(frac(g["v"][t - 1]), abs=1e-15)
        assert p[0] == pytest.approx(ref[t - 1], rel=1e-13)
    # the pin separates the two moment rates: with them swapped step 2 already differs
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t, gr in enumerate(g["grads"][:2], start=1):
        p, m, v = cnn.adam_update(p, np.array([gr]), m, v, t=t, lr=g["lr"], b1=g["b2"], b2=g["b1"], eps=g["eps"])
    assert abs(p[0] - ref[1]) > 1e-3


def delta_psf(L, N):
    psf = np.zeros((L, N, N))
    psf[:, N // 2, N // 2] = 1.0
    return psf


def test_two_step_calibration_reaches_each_steps_closed_form():
    """delta PSF, mu_s = 0: step 1 (mu_lambda = 0) converges to (Y)_+; step 2 (mu_lambda > 0, from
    step 1's X) converges to the per-pixel soft threshold of the cosine coefficients when the
    positivity constraint is inactive (Y on a large positive offset)."""
    r = np.random.default_rng(3)
    L, N = 4, 8
    Y = 5.0 + r.normal(size=(L, N, N))
    p = om.Problem(dirty=Y, psf=delta_psf(L, N), J=2, mu_s=0.0, mu_l=0.4, sigma=1.0)
    st1, st2 = om.two_step_calibration(p, 50, 2000, tau1=0.9)
    np.testing.assert_allclose(st1.X, np.maximum(Y, 0.0), atol=1e-9)
    ref = om.spectral_adjoint(om.soft(om.spectral(Y), 0.4))
    np.testing.assert_allclose(st2.X, ref, atol=1e-8)
    # step 2 starts from step 1's X with fresh duals: one step from there equals iterate on init_state(X1)
    tau2 = om.step_sizes(p)[0]
    st1b, st2b = om.two_step_calibration(p, 50, 1, tau1=0.9)
    one = om.iterate(p, om.init_state(p, st1b.X), tau2)
    np.testing.assert_array_equal(st2b.X, one.X)
