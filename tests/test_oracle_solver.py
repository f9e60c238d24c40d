"""Pins of the oracle's Algorithm 1 against closed-form minimisers, exact invariants,
an independent QP solve and the optimality (KKT) conditions."""
import numpy as np
import pytest
import scipy.optimize

from oracle import muffin as om


def delta_psf(L, N):
    psf = np.zeros((L, N, N))
    psf[:, N // 2, N // 2] = 1.0
    return psf


def peaked_psf(L, N, seed=0, side=0.25):
    """A nonnegative PSF: unit peak at the origin plus small random sidelobes."""
    r = np.random.default_rng(seed)
    psf = side * r.uniform(0, 1, size=(L, N, N))
    psf[:, N // 2, N // 2] = 1.0
    return psf


def prob(dirty, psf, J=1, mu_s=0.0, mu_l=0.0, **kw):
    return om.Problem(dirty=dirty, psf=psf, J=J, mu_s=mu_s, mu_l=mu_l, **kw)


# ---------------------------------------------------------------- closed forms
def test_delta_psf_no_prior_gives_positive_part():
    r = np.random.default_rng(1)
    Y = r.normal(size=(3, 8, 8))
    st, _ = om.solve(prob(Y, delta_psf(3, 8)), 1500)
    np.testing.assert_allclose(st.X, np.maximum(Y, 0), atol=1e-10)


def test_delta_psf_single_channel_spectral_prior_soft_thresholds():
    """L = 1: W_lambda = [1], so the minimiser is (y - mu_lambda)_+."""
    r = np.random.default_rng(2)
    Y = r.normal(scale=2.0, size=(1, 8, 8))
    mu = 0.7
    st, _ = om.solve(prob(Y, delta_psf(1, 8), mu_l=mu), 4000)
    np.testing.assert_allclose(st.X, np.maximum(Y - mu, 0), atol=1e-8)


def test_delta_psf_spectral_prior_inactive_positivity():
    """With positivity inactive the minimiser is IDCT(soft(DCT(y), mu_lambda)) per pixel."""
    r = np.random.default_rng(3)
    L = 5
    Y = 50.0 + r.normal(size=(L, 4, 4))
    mu = 0.4
    st, _ = om.solve(prob(Y, delta_psf(L, 4), mu_l=mu), 4000)
    W = om.dct_matrix(L)
    coef = np.tensordot(W.T, Y, axes=(1, 0))
    expect = np.tensordot(W, om.soft(coef, mu), axes=(1, 0))
    np.testing.assert_allclose(st.X, expect, atol=1e-8)


# ---------------------------------------------------------------- invariants
def small_problem(seed=4, L=3, N=8, J=2, gen=2, mu_s=0.25, mu_l=0.5):
    r = np.random.default_rng(seed)
    psf = peaked_psf(L, N, seed)
    X_true = np.maximum(r.normal(size=(L, N, N)), 0)
    Y = om.apply_H(psf, X_true) + 0.05 * r.normal(size=(L, N, N))
    return prob(Y, psf, J=J, mu_s=mu_s, mu_l=mu_l, gen=gen)


def test_scaling_invariance_is_exact():
    """(Y, mu_s, mu_l, tau, sigma) -> (cY, c mu_s, c mu_l, tau, sigma/c^2) scales X by c; U, V unchanged."""
    p = small_problem()
    tau = om.step_sizes(p)[0]
    c = 4.0
    q = prob(c * p.dirty, p.psf, J=p.J, mu_s=c * p.mu_s, mu_l=c * p.mu_l, sigma=p.sigma / c ** 2)
    a, _ = om.solve(p, 30, tau=tau)
    b, _ = om.solve(q, 30, tau=tau)
    np.testing.assert_allclose(b.X, c * a.X, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(b.U, a.U, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(b.V, a.V, rtol=1e-12, atol=1e-14)


def test_spatial_shift_equivariance():
    p = small_problem()
    tau = om.step_sizes(p)[0]
    q = prob(np.roll(p.dirty, (3, -2), axis=(-2, -1)), p.psf, J=p.J, mu_s=p.mu_s, mu_l=p.mu_l)
    a, _ = om.solve(p, 25, tau=tau)
    b, _ = om.solve(q, 25, tau=tau)
    np.testing.assert_allclose(b.X, np.roll(a.X, (3, -2), axis=(-2, -1)), atol=1e-12)


def test_channel_reversal_equivariance():
    p = small_problem()
    tau = om.step_sizes(p)[0]
    q = prob(p.dirty[::-1].copy(), p.psf[::-1].copy(), J=p.J, mu_s=p.mu_s, mu_l=p.mu_l)
    a, _ = om.solve(p, 25, tau=tau)
    b, _ = om.solve(q, 25, tau=tau)
    np.testing.assert_allclose(b.X, a.X[::-1], atol=1e-12)


def test_no_spectral_prior_separates_channels():
    """mu_lambda = 0 decouples the channels (Sec. 4, first calibration step)."""
    p = small_problem(mu_l=0.0)
    tau = om.step_sizes(p)[0]
    a, _ = om.solve(p, 25, tau=tau)
    for l in range(p.L):
        ql = prob(p.dirty[l:l + 1], p.psf[l:l + 1], J=p.J, mu_s=p.mu_s, mu_l=0.0)
        b, _ = om.solve(ql, 25, tau=tau)
        np.testing.assert_allclose(b.X[0], a.X[l], atol=1e-13)


# ---------------------------------------------------------------- step sizes
def explicit_K(p):
    """Dense K = [mu_s W_s (per channel); mu_lambda W_lambda (per pixel)] built from unit vectors."""
    L, N, J = p.L, p.N, p.J
    n = L * N * N
    rows = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        X = e.reshape(L, N, N)
        ks = np.concatenate([p.mu_s * om.iuwt(X[l], J, p.gen).ravel() for l in range(L)])
        kl = p.mu_l * om.spectral(X).ravel()
        rows.append(np.concatenate([ks, kl]))
    return np.array(rows).T


def explicit_H(p):
    L, N = p.L, p.N
    n = L * N * N
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(om.apply_H(p.psf, e.reshape(L, N, N)).ravel())
    return np.array(cols).T


def test_operator_norm_matches_dense_matrix():
    p = small_problem(N=4, J=1, L=3)
    K = explicit_K(p)
    assert om.op_norm_sq(p) == pytest.approx(np.linalg.norm(K, 2) ** 2, rel=1e-10)
    H = explicit_H(p)
    assert om.lipschitz(p.psf) == pytest.approx(np.linalg.norm(H, 2) ** 2, rel=1e-10)


def test_step_sizes_satisfy_convergence_condition_and_reject_bad_tau():
    p = small_problem()
    tau, sigma, rho, beta, k2 = om.step_sizes(p)
    assert 1 / tau - sigma * k2 > beta / 2
    bad = prob(p.dirty, p.psf, J=p.J, mu_s=p.mu_s, mu_l=p.mu_l, tau=2.5 / beta)
    with pytest.raises(ValueError):
        om.step_sizes(bad)


# ---------------------------------------------------------------- optimality
def tiny_problem():
    """N=4, L=2, J=1; the offset makes 8 of the 32 minimiser pixels zero."""
    p = small_problem(seed=11, L=2, N=4, J=1, mu_s=0.3, mu_l=0.6)
    p.dirty = p.dirty - 0.3
    return p


def test_matches_independent_qp_solution():
    """min 1/2||Hx - y||^2 + ||Kx||_1, x >= 0, solved as a smooth QP (z >= |Kx|) by scipy's
    trust-constr on dense matrices; the oracle's objective must reach the same minimum."""
    p = tiny_problem()
    H = explicit_H(p)
    K = explicit_K(p)
    y = p.dirty.ravel()
    n, m = H.shape[1], K.shape[0]

    def f(z):
        r = H @ z[:n] - y
        return 0.5 * r @ r + z[n:].sum()

    def g(z):
        out = np.ones_like(z)
        out[:n] = H.T @ (H @ z[:n] - y)
        return out

    hess = np.zeros((n + m, n + m))
    hess[:n, :n] = H.T @ H
    A = np.vstack([np.hstack([-K, np.eye(m)]), np.hstack([K, np.eye(m)])])
    x0 = np.maximum(y, 0)
    z0 = np.concatenate([x0, np.abs(K @ x0) + 1e-3])
    res = scipy.optimize.minimize(
        f, z0, jac=g, hess=lambda z: hess, method="trust-constr",
        bounds=scipy.optimize.Bounds([0.0] * n + [-np.inf] * m, np.inf),
        constraints=[scipy.optimize.LinearConstraint(A, 0.0, np.inf)],
        options={"maxiter": 20000, "gtol": 1e-12, "xtol": 1e-14})
    assert res.success, res.message
    st, _ = om.solve(p, 6000)
    f_oracle = om.objective(p, st.X)[0]
    assert f_oracle == pytest.approx(res.fun, rel=1e-8)


def test_converged_iterate_satisfies_kkt():
    """At the fixed point: (U, V) lie in the unit box and are subgradients of ||.||_1 at Kx;
    the primal residual grad f + K^T (U, V) vanishes where x > 0 and is >= 0 where x = 0."""
    p = tiny_problem()
    st, _ = om.solve(p, 6000)
    X, U, V = st.X, st.U, st.V
    g = om.data_gradient(p.psf, X, p.dirty)
    r = g + p.mu_s * np.stack([om.iuwt_adjoint(U[l], p.J, p.gen) for l in range(p.L)]) \
        + p.mu_l * om.spectral_adjoint(V)
    pos = X > 1e-9
    assert np.max(np.abs(r[pos])) < 1e-6
    assert np.any(~pos)
    assert np.min(r[~pos]) > -1e-6
    assert np.all(np.abs(U) <= 1.0) and np.all(np.abs(V) <= 1.0)
    ws = np.stack([om.iuwt(X[l], p.J, p.gen) for l in range(p.L)])
    act = np.abs(ws) > 1e-6
    np.testing.assert_allclose(U[act], np.sign(ws[act]), atol=1e-6)
    wl = om.spectral(X)
    act = np.abs(wl) > 1e-6
    np.testing.assert_allclose(V[act], np.sign(wl[act]), atol=1e-6)


def test_objective_behaviour():
    """f_k approaches the long-run value; fixed-point residuals vanish (no per-step monotonicity)."""
    p = small_problem(N=8, L=3, J=2)
    tau = om.step_sizes(p)[0]
    st = om.init_state(p)
    fs, dx = [], []
    for _ in range(1500):
        nxt = om.iterate(p, st, tau)
        dx.append(np.linalg.norm(nxt.X - st.X))
        st = nxt
        fs.append(om.objective(p, st.X)[0])
    fs = np.array(fs)
    f_end = fs[-1]
    assert abs(fs[100] - f_end) > abs(fs[-200] - f_end)
    assert abs(fs[-200] - f_end) / abs(f_end) < 1e-3
    assert dx[-1] < 1e-3 * max(dx[:10])
    assert om.objective(p, st.X)[0] < om.objective(p, np.zeros_like(st.X))[0]
