"""Pins of the union-of-bases oracle (oracle/uob.py): Daubechies' published closed forms, the
defining properties of each filter, orthonormality of the periodic transform by brute force, the
tight frame, the adjoint, a one-level Haar example by hand, and the solver with this prior against
an independent QP solve."""
import numpy as np
import pytest
import scipy.optimize

from oracle import muffin as om
from oracle import uob


def test_haar_and_db2_closed_forms():
    np.testing.assert_allclose(uob.daubechies_lowpass(1), [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    s3 = np.sqrt(3.0)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))  # Daubechies (1988)
    np.testing.assert_allclose(uob.daubechies_lowpass(2), ref, atol=1e-14)


@pytest.mark.parametrize("n", range(1, 9))
def test_filter_properties(n):
    """length 2n, sum sqrt(2), orthonormal to its even shifts, n vanishing wavelet moments, and the
    frequency response |m0(w)|^2 + |m0(w + pi)|^2 = 1 with m0 = sum h_k e^{-ikw} / sqrt(2)."""
    h = uob.daubechies_lowpass(n)
    assert len(h) == 2 * n
    assert h.sum() == pytest.approx(np.sqrt(2.0), abs=1e-13)
    for m in range(n):
        assert np.dot(h[:len(h) - 2 * m], h[2 * m:]) == pytest.approx(1.0 if m == 0 else 0.0, abs=1e-12)
    k = np.arange(len(h))
    for p in range(n):
        assert abs(np.sum((-1.0) ** k * k ** p * h)) <= 1e-12 * max(1.0, (2 * n) ** p)
    w = np.linspace(0, np.pi, 33)
    m0 = lambda w: (h[None, :] * np.exp(-1j * np.outer(w, k))).sum(axis=1) / np.sqrt(2.0)
    np.testing.assert_allclose(np.abs(m0(w)) ** 2 + np.abs(m0(w + np.pi)) ** 2, 1.0, atol=1e-12)
    # the wavelet filter annihilates constants and is orthogonal to the scaling filter's even shifts
    g = uob.highpass(h)
    assert abs(g.sum()) < 1e-12
    for m in range(-(n - 1), n):
        a = np.sum([h[i] * g[i + 2 * m] for i in range(len(h)) if 0 <= i + 2 * m < len(h)])
        assert abs(a) < 1e-12


def test_one_level_haar_by_hand():
    """Rows then columns with h = (1, 1)/sqrt 2, g = (1, -1)/sqrt 2 on [[a, b], [c, d]]."""
    a, b, c, d = 1.0, 2.0, 5.0, 11.0
    out = uob.dwt2(np.array([[a, b], [c, d]]), uob.daubechies_lowpass(1), 1)
    np.testing.assert_allclose(out, [[(a + b + c + d) / 2, (a - b + c - d) / 2],
                                     [(a + b - c - d) / 2, (a - b - c + d) / 2]], atol=1e-15)


@pytest.mark.parametrize("n", [1, 3, 8])
def test_one_level_is_orthogonal_by_brute_force(n):
    """The periodic one-level analysis as an explicit 16 x 16 matrix (built column by column from
    its definition) is orthogonal, also where the filter is longer than the signal."""
    h = uob.daubechies_lowpass(n)
    for size in (16, 4):
        cols = []
        for i in range(size):
            e = np.zeros(size)
            e[i] = 1.0
            lo, hi = uob.analysis_1d(e, h, axis=0)
            cols.append(np.concatenate([lo, hi]))
        M = np.array(cols).T
        np.testing.assert_allclose(M @ M.T, np.eye(size), atol=1e-12)


def test_multilevel_transform_perfect_reconstruction_and_energy():
    r = np.random.default_rng(1)
    x = r.normal(size=(32, 32))
    for h in uob.filters():
        c = uob.dwt2(x, h, 3)
        assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)
        np.testing.assert_allclose(uob.idwt2(c, h, 3), x, atol=1e-12)


def test_constant_image():
    """A constant c has zero details; each 2-D level multiplies the mean by 2, so the J-level
    approximation block holds c 2^J."""
    for h in uob.filters():
        out = uob.dwt2(np.full((16, 16), 0.7), h, 2)
        np.testing.assert_allclose(out[:4, :4], 0.7 * 4, atol=1e-12)
        out[:4, :4] = 0.0
        assert np.max(np.abs(out)) < 1e-12


def test_union_is_a_tight_frame_and_adjoint():
    r = np.random.default_rng(2)
    x = r.normal(size=(16, 16))
    u = r.normal(size=(8, 16, 16))
    W = uob.uob(x, 2)
    assert W.shape == (8, 16, 16)
    np.testing.assert_allclose(uob.uob_adjoint(W, 2), x, atol=1e-12)  # W^T W = I
    assert np.sum(W * u) == pytest.approx(np.sum(x * uob.uob_adjoint(u, 2)), rel=1e-12)
    # ||W||^2 = 1: the largest singular value of the explicit matrix at 8 x 8
    cols = []
    for i in range(64):
        e = np.zeros(64)
        e[i] = 1.0
        cols.append(uob.uob(e.reshape(8, 8), 2).ravel())
    Wm = np.array(cols).T
    assert np.linalg.norm(Wm, 2) ** 2 == pytest.approx(1.0, abs=1e-12)


def test_solver_with_union_of_bases_matches_qp():
    """The oracle's iteration with the union-of-bases prior (N = 4, J = 1, L = 2) reaches the
    minimum of min 1/2||Hx - y||^2 + ||Kx||_1, x >= 0, solved as a smooth QP on dense matrices."""
    r = np.random.default_rng(11)
    L, N, J = 2, 4, 1
    psf = np.abs(r.normal(size=(L, N, N))) * 0.3
    psf[:, N // 2, N // 2] = 1.0
    x_true = np.abs(r.normal(size=(L, N, N)))
    y = om.apply_H(psf, x_true) + 0.05 * r.normal(size=(L, N, N)) - 0.3
    p = om.Problem(dirty=y, psf=psf, J=J, mu_s=0.3, mu_l=0.6, prior="uob")
    n = L * N * N
    K = []
    H = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        X = e.reshape(L, N, N)
        ks = np.concatenate([p.mu_s * uob.uob(X[l], J).ravel() for l in range(L)])
        K.append(np.concatenate([ks, p.mu_l * om.spectral(X).ravel()]))
        H.append(om.apply_H(psf, X).ravel())
    K, H = np.array(K).T, np.array(H).T
    assert om.op_norm_sq(p) == pytest.approx(np.linalg.norm(K, 2) ** 2, rel=1e-10)
    yv = y.ravel()
    m = K.shape[0]

    def f(z):
        res = H @ z[:n] - yv
        return 0.5 * res @ res + z[n:].sum()

    def g(z):
        out = np.ones_like(z)
        out[:n] = H.T @ (H @ z[:n] - yv)
        return out

    hess = np.zeros((n + m, n + m))
    hess[:n, :n] = H.T @ H
    A = np.vstack([np.hstack([-K, np.eye(m)]), np.hstack([K, np.eye(m)])])
    x0 = np.maximum(yv, 0)
    z0 = np.concatenate([x0, np.abs(K @ x0) + 1e-3])
    res = scipy.optimize.minimize(f, z0, jac=g, hess=lambda z: hess, method="trust-constr",
                                  bounds=scipy.optimize.Bounds([0.0] * n + [-np.inf] * m, np.inf),
                                  constraints=[scipy.optimize.LinearConstraint(A, 0.0, np.inf)],
                                  options={"maxiter": 20000, "gtol": 1e-12, "xtol": 1e-14})
    assert res.success, res.message
    st, _ = om.solve(p, 6000)
    assert st.U.shape == (L, 8, N, N)
    assert om.objective(p, st.X)[0] == pytest.approx(res.fun, rel=1e-8)
