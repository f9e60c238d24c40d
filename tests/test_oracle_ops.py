"""Pins of the FP64 oracle's operators against brute force, closed forms and library routines.

Each test checks the oracle against something other than itself, chosen so a
plausible slip (a dropped term, a wrong sign, index or tap, a transposed
operand) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import muffin as om


def rng(seed=0):
    return np.random.default_rng(seed)


def rand_psf(L, N, seed=1):
    return rng(seed).uniform(0.0, 1.0, size=(L, N, N))


# ---------------------------------------------------------------- data term
def test_H_equals_direct_circular_convolution():
    """H_l x_l == sum_q psf_l[q] x_l[p - (q - N/2)] written as an explicit O(N^4) loop."""
    L, N = 2, 6
    psf = rand_psf(L, N)
    x = rng(2).normal(size=(L, N, N))
    out = np.zeros((L, N, N))
    for l in range(L):
        for p0 in range(N):
            for p1 in range(N):
                acc = 0.0
                for q0 in range(N):
                    for q1 in range(N):
                        acc += psf[l, q0, q1] * x[l, (p0 - q0 + N // 2) % N, (p1 - q1 + N // 2) % N]
                out[l, p0, p1] = acc
    np.testing.assert_allclose(om.apply_H(psf, x), out, rtol=1e-12, atol=1e-12)


def test_H_delta_psf_is_identity():
    L, N = 3, 8
    psf = np.zeros((L, N, N))
    psf[:, N // 2, N // 2] = 1.0
    x = rng(3).normal(size=(L, N, N))
    np.testing.assert_allclose(om.apply_H(psf, x), x, atol=1e-13)
    np.testing.assert_allclose(om.apply_Ht(psf, x), x, atol=1e-13)


def test_H_shifted_delta_is_shift():
    """A delta PSF one pixel right of the origin shifts the image by one pixel to the right."""
    N = 8
    psf = np.zeros((1, N, N))
    psf[0, N // 2, N // 2 + 1] = 1.0
    x = rng(4).normal(size=(1, N, N))
    np.testing.assert_allclose(om.apply_H(psf, x), np.roll(x, 1, axis=-1), atol=1e-13)


def test_H_adjoint_dot():
    L, N = 3, 16
    psf = rand_psf(L, N)
    x = rng(5).normal(size=(L, N, N))
    y = rng(6).normal(size=(L, N, N))
    lhs = np.sum(om.apply_H(psf, x) * y)
    rhs = np.sum(x * om.apply_Ht(psf, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_lipschitz_equals_squared_psf_sum_for_nonnegative_psf():
    """|H(k)| <= H(0) = sum psf for a nonnegative PSF, so ||H||^2 = (sum psf)^2."""
    L, N = 4, 16
    psf = rand_psf(L, N)
    w = np.array([1.0, 0.5, 2.0, 0.25])
    expect = max(w[l] * psf[l].sum() ** 2 for l in range(L))
    assert om.lipschitz(psf, w) == pytest.approx(expect, rel=1e-12)


def test_lipschitz_matches_power_iteration():
    """Power iteration on H^T H (signed PSF, so the maximum is not at DC)."""
    N = 16
    psf = rng(7).normal(size=(1, N, N))
    v = rng(8).normal(size=(1, N, N))
    for _ in range(3000):
        v = om.apply_Ht(psf, om.apply_H(psf, v))
        v /= np.linalg.norm(v)
    rq = np.sum(v * om.apply_Ht(psf, om.apply_H(psf, v)))
    assert om.lipschitz(psf) == pytest.approx(rq, rel=1e-6)


def test_gradient_is_derivative_of_data_term():
    L, N = 2, 8
    psf = rand_psf(L, N)
    w = np.array([0.7, 1.3])
    x = rng(9).normal(size=(L, N, N))
    y = rng(10).normal(size=(L, N, N))
    dx = rng(11).normal(size=(L, N, N))
    h = 1e-6
    fd = (om.data_term(psf, x + h * dx, y, w) - om.data_term(psf, x - h * dx, y, w)) / (2 * h)
    an = np.sum(om.data_gradient(psf, x, y, w) * dx)
    assert fd == pytest.approx(an, rel=1e-7)


# ---------------------------------------------------------------- IUWT
@pytest.mark.parametrize("N,J", [(16, 1), (16, 2), (32, 3), (8, 3)])
def test_iuwt_gen1_planes_sum_to_image(N, J):
    x = rng(12).normal(size=(N, N))
    np.testing.assert_allclose(om.iuwt(x, J, 1).sum(axis=0), x, atol=1e-13)


@pytest.mark.parametrize("N,J", [(16, 1), (32, 3), (8, 3)])
def test_iuwt_gen2_recursive_synthesis_reconstructs(N, J):
    """Second generation: c_j = w_{j+1} + H_j c_{j+1} recovers x; the plain sum does not."""
    x = rng(13).normal(size=(N, N))
    u = om.iuwt(x, J, 2)
    np.testing.assert_allclose(om.iuwt_synthesis(u, J, 2), x, atol=1e-13)
    assert np.max(np.abs(u.sum(axis=0) - x)) > 1e-3


@pytest.mark.parametrize("gen", [1, 2])
@pytest.mark.parametrize("N,J", [(16, 2), (32, 4), (8, 3)])
def test_iuwt_adjoint_dot(gen, N, J):
    x = rng(14).normal(size=(N, N))
    u = rng(15).normal(size=(J + 1, N, N))
    lhs = np.sum(om.iuwt(x, J, gen) * u)
    rhs = np.sum(x * om.iuwt_adjoint(u, J, gen))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("gen", [1, 2])
def test_iuwt_adjoint_is_explicit_matrix_transpose(gen):
    N, J = 8, 2
    n = N * N
    A = np.zeros(((J + 1) * n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = om.iuwt(e.reshape(N, N), J, gen).ravel()
    At = np.zeros((n, (J + 1) * n))
    for i in range((J + 1) * n):
        e = np.zeros((J + 1) * n)
        e[i] = 1.0
        At[:, i] = om.iuwt_adjoint(e.reshape(J + 1, N, N), J, gen).ravel()
    np.testing.assert_allclose(At, A.T, atol=1e-14)


def test_iuwt_constant_image():
    N, J = 16, 3
    for gen in (1, 2):
        u = om.iuwt(np.full((N, N), 2.5), J, gen)
        np.testing.assert_allclose(u[:J], 0.0, atol=1e-14)
        np.testing.assert_allclose(u[J], 2.5, atol=1e-14)


@pytest.mark.parametrize("j", [0, 1, 2])
def test_b3_smoothing_eigenvalue(j):
    """cos(w1 m) cos(w2 n) is an eigenimage of H_j with eigenvalue b(2^j w1) b(2^j w2),
    b(w) = 3/8 + cos(w)/2 + cos(2w)/8, the response of the [1,4,6,4,1]/16 filter."""
    N = 32
    k1, k2 = 3, 5
    w1, w2 = 2 * np.pi * k1 / N, 2 * np.pi * k2 / N
    m = np.arange(N)
    img = np.outer(np.cos(w1 * m), np.cos(w2 * m))
    b = lambda w: 3 / 8 + np.cos(w) / 2 + np.cos(2 * w) / 8
    np.testing.assert_allclose(om.smooth(img, j), b(2 ** j * w1) * b(2 ** j * w2) * img, atol=1e-13)


def test_b3_taps_on_delta():
    """The smoothing of a delta is the outer product of [1,4,6,4,1]/16 at dilation 2^j."""
    N = 16
    d = np.zeros((N, N))
    d[8, 8] = 1.0
    out = om.smooth(d, 1)
    h = np.array([1, 4, 6, 4, 1]) / 16
    expect = np.zeros((N, N))
    for a in range(5):
        for e in range(5):
            expect[8 + 2 * (a - 2), 8 + 2 * (e - 2)] = h[a] * h[e]
    np.testing.assert_allclose(out, expect, atol=1e-15)


@pytest.mark.parametrize("gen", [1, 2])
def test_frame_symbol_matches_plane_wave_energy(gen):
    """||W_s c||^2 / ||c||^2 for a cosine eigenimage equals the closed-form symbol at its frequency."""
    N, J = 32, 3
    m = np.arange(N)
    sym = om.frame_symbol(N, J, gen)
    for k1, k2 in [(0, 0), (1, 0), (3, 7), (16, 16), (5, 11)]:
        img = np.outer(np.cos(2 * np.pi * k1 * m / N), np.cos(2 * np.pi * k2 * m / N))
        e = np.sum(om.iuwt(img, J, gen) ** 2) / np.sum(img ** 2)
        assert e == pytest.approx(sym[k1, k2], rel=1e-12)


@pytest.mark.parametrize("gen", [1, 2])
def test_frame_bound_is_one_and_power_iteration_agrees(gen):
    N, J = 32, 3
    assert np.max(om.frame_symbol(N, J, gen)) == pytest.approx(1.0, abs=1e-14)
    v = rng(16).normal(size=(N, N))
    for _ in range(200):
        v = om.iuwt_adjoint(om.iuwt(v, J, gen), J, gen)
        v /= np.linalg.norm(v)
    rq = np.sum(om.iuwt(v, J, gen) ** 2)
    assert 0.99 < rq <= 1.0 + 1e-12


# ---------------------------------------------------------------- DCT
@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 15, 64])
def test_spectral_matches_scipy_dct(L):
    X = rng(17).normal(size=(L, 4, 3))
    np.testing.assert_allclose(om.spectral(X), scipy.fft.dct(X, type=2, norm="ortho", axis=0),
                               atol=1e-13)
    np.testing.assert_allclose(om.spectral_adjoint(X), scipy.fft.idct(X, type=2, norm="ortho", axis=0),
                               atol=1e-13)


@pytest.mark.parametrize("L", [1, 4, 7, 16])
def test_dct_orthonormal_and_constant(L):
    W = om.dct_matrix(L)
    np.testing.assert_allclose(W @ W.T, np.eye(L), atol=1e-13)
    c = np.full((L, 1, 1), 1.5)
    out = om.spectral(c)[:, 0, 0]
    np.testing.assert_allclose(out, np.r_[np.sqrt(L) * 1.5, np.zeros(L - 1)], atol=1e-13)


# ---------------------------------------------------------------- prox maps
def test_sat_is_projection_on_unit_interval_brute_force():
    grid = np.linspace(-1, 1, 200001)
    for z in [-3.2, -1.0, -0.4, 0.0, 0.73, 1.0, 5.0]:
        best = grid[np.argmin((grid - z) ** 2)]
        assert om.sat(np.array(z)) == pytest.approx(best, abs=1e-5)


def test_soft_brute_force_and_moreau():
    grid = np.linspace(-6, 6, 600001)
    for z in [-3.2, -0.4, 0.0, 0.73, 5.0]:
        for t in [0.5, 1.0, 2.0]:
            best = grid[np.argmin(0.5 * (grid - z) ** 2 + t * np.abs(grid))]
            assert om.soft(np.array(z), t) == pytest.approx(best, abs=2e-5)
    z = rng(18).normal(scale=2.0, size=1000)
    np.testing.assert_allclose(om.sat(z) + om.soft(z, 1.0), z, atol=1e-15)


def test_positive_part():
    x = np.array([-2.0, -0.0, 0.0, 3.0])
    np.testing.assert_array_equal(om.positive(x), [0.0, 0.0, 0.0, 3.0])
