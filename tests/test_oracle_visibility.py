"""Pins of the visibility-domain oracle (Sec. 2, eq. (viseq)) against what fixes it independently:
the 2-D DFT it reduces to on a grid with w = 0, the geometric phase of a point source, adjointness,
Hermitian symmetry, finite differences of the data term, and a dense eigen-solver for beta."""
import numpy as np
import pytest

from oracle import muffin as om
from oracle import visibility as ov
from paper_1602_08847_amd import synth


def rng_uvw(rng, K, b):
    return np.column_stack([rng.uniform(-b, b, K), rng.uniform(-b, b, K), rng.uniform(-b / 2, b / 2, K)])


def test_grid_baselines_with_w_zero_are_the_dft_of_x_over_n():
    # u = p lambda / (N cell), v = q lambda / (N cell), w = 0: the phase of pixel (i, j) is
    # p (j - N/2) / N + q (i - N/2) / N, so Phi x = (-1)^(p+q) FFT2(x / n)[q, p] (N even)
    N, cell, lam = 16, 0.01, 0.7
    rng = np.random.default_rng(3)
    x = rng.normal(size=(1, N, N))
    pq = [(1, 3), (3, 1), (0, 5), (-4, 2), (7, -6), (0, 0)]
    uvw = np.array([[p * lam / (N * cell), q * lam / (N * cell), 0.0] for p, q in pq])
    # n of every pixel, computed here from its own grid
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    n = np.sqrt(1.0 - ((jj - N / 2) * cell) ** 2 - ((ii - N / 2) * cell) ** 2)
    F = np.fft.fft2(x[0] / n)
    want = np.array([(-1.0) ** (p + q) * F[q % N, p % N] for p, q in pq])
    got = ov.phi(x, uvw, np.array([lam]), cell)[0]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-10)


def test_point_source_phase_is_the_geometric_path_difference():
    # a unit source in the direction of the unit vector s (polar angle th, azimuth ph): its
    # visibility on baseline b is exp(-2 pi i b.s / lambda) / cos(th) (s_z = n = cos th)
    N, cell = 32, 0.02
    i0, j0 = 7, 27
    l0, m0 = (j0 - N / 2) * cell, (i0 - N / 2) * cell
    th = np.arcsin(np.hypot(l0, m0))
    ph = np.arctan2(m0, l0)
    s = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    rng = np.random.default_rng(5)
    uvw = rng_uvw(rng, 9, 300.0)
    lam = np.array([0.9, 1.3])
    x = np.zeros((2, N, N))
    x[:, i0, j0] = 1.0
    got = ov.phi(x, uvw, lam, cell)
    for c in range(2):
        want = np.exp(-2j * np.pi * (uvw @ s) / lam[c]) / np.cos(th)
        assert np.allclose(got[c], want, rtol=1e-12, atol=1e-12)


def test_phase_centre_source_sees_only_w():
    N = 8
    x = np.zeros((1, N, N))
    x[0, N // 2, N // 2] = 2.5
    uvw = np.array([[10.0, -3.0, 0.0], [4.0, 8.0, 0.25], [0.0, 0.0, 1.5]])
    got = ov.phi(x, uvw, np.array([0.5]), 0.05)[0]
    assert np.allclose(got, 2.5 * np.exp(-2j * np.pi * uvw[:, 2] / 0.5), rtol=1e-13)


def test_adjoint_and_hermitian_symmetry():
    N, L, K = 12, 3, 40
    rng = np.random.default_rng(11)
    uvw = rng_uvw(rng, K, 60.0)
    lam = np.array([1.0, 0.8, 0.6])
    cell = 0.01
    x = rng.normal(size=(L, N, N))
    r = rng.normal(size=(L, K)) + 1j * rng.normal(size=(L, K))
    lhs = np.sum(np.real(np.conj(ov.phi(x, uvw, lam, cell)) * r))
    rhs = np.sum(x * ov.phi_adjoint(r, uvw, lam, cell, N))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1)
    # real sky: the mirrored baseline sees the conjugate visibility
    assert np.allclose(ov.phi(x, -uvw, lam, cell), np.conj(ov.phi(x, uvw, lam, cell)), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("w", [None, (0.5, 3.0)])
def test_gradient_matches_finite_differences(w):
    N, L, K = 8, 2, 30
    rng = np.random.default_rng(2)
    uvw = rng_uvw(rng, K, 40.0)
    d = ov.VisData(uvw=uvw, lam=np.array([1.0, 0.75]), cell=0.02,
                   vis=rng.normal(size=(L, K)) + 1j * rng.normal(size=(L, K)), N=N, w=w)
    x = rng.normal(size=(L, N, N))
    e = rng.normal(size=(L, N, N))
    h = 1e-5
    fd = (ov.vis_data_term(x + h * e, d) - ov.vis_data_term(x - h * e, d)) / (2 * h)
    an = np.sum(ov.vis_gradient(x, d) * e)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_channel_weights_scale_each_channel_alone():
    # a channel's weight scales its own data term and gradient and leaves the other channel alone
    N, L, K = 8, 2, 20
    rng = np.random.default_rng(6)
    uvw = rng_uvw(rng, K, 40.0)
    vis = rng.normal(size=(L, K)) + 1j * rng.normal(size=(L, K))
    x = rng.normal(size=(L, N, N))
    d1 = ov.VisData(uvw=uvw, lam=np.array([1.0, 0.75]), cell=0.02, vis=vis, N=N)
    d2 = ov.VisData(uvw=uvw, lam=np.array([1.0, 0.75]), cell=0.02, vis=vis, N=N, w=np.array([1.0, 4.0]))
    g1, g2 = ov.vis_gradient(x, d1), ov.vis_gradient(x, d2)
    assert np.allclose(g2[0], g1[0], rtol=1e-13, atol=1e-13) and np.allclose(g2[1], 4.0 * g1[1], rtol=1e-13)
    one = ov.VisData(uvw=uvw, lam=np.array([0.75]), cell=0.02, vis=vis[1:], N=N)
    assert np.isclose(ov.vis_data_term(x, d2) - ov.vis_data_term(x, d1), 3.0 * ov.vis_data_term(x[1:], one),
                      rtol=1e-12)


def test_power_estimate_against_dense_eigensolver():
    N, K = 6, 25
    rng = np.random.default_rng(8)
    uvw = rng_uvw(rng, K, 30.0)
    lam = np.array([1.0, 0.7, 0.55])
    cell = 0.03
    tops = []
    for l in lam:
        # Re Phi^H Phi, its columns from unit images
        cols = [ov.phi_adjoint(ov.phi(np.eye(N * N)[p].reshape(1, N, N), uvw, np.array([l]), cell), uvw,
                               np.array([l]), cell, N).ravel() for p in range(N * N)]
        tops.append(float(np.max(np.linalg.eigvalsh(np.array(cols)))))
    top = max(tops)
    # the three channels' top eigenvalues lie close together, which slows the iteration down
    est = ov.power_estimate(uvw, lam, cell, N, iters=200)
    assert est <= top * (1 + 1e-12)
    assert est >= top * (1 - 1e-4)
    assert ov.power_estimate(uvw, lam, cell, N) >= top * (1 - 1e-2)
    d = ov.VisData(uvw=uvw, lam=lam, cell=cell, vis=np.zeros((3, K), complex), N=N)
    assert ov.vis_lipschitz(d) >= top
    # channel weights: the weighted eigenvalues, the dense way
    w = np.array([0.2, 1.0, 2.5])
    topw = max(w[c] * tops[c] for c in range(3))
    estw = ov.power_estimate(uvw, lam, cell, N, iters=200, w=w)
    assert topw * (1 - 1e-4) <= estw <= topw * (1 + 1e-12)


def test_pixel_outside_the_unit_disc_is_rejected():
    with pytest.raises(ValueError):
        ov.direction_cosines(64, 0.03)


def test_solver_with_visibilities_decreases_the_objective():
    vi = synth.make_vis_inputs(synth.VisSpec(N=16, L=4, K=120, n_sources=3, seed=1))
    vis = ov.phi(vi.sky, vi.uvw, vi.lam, vi.cell) + vi.noise
    d = ov.VisData(uvw=vi.uvw, lam=vi.lam, cell=vi.cell, vis=vis, N=16)
    p = om.Problem(dirty=None, psf=None, J=2, mu_s=1.0, mu_l=2.0, vis=d)
    assert p.L == 4 and p.N == 16
    st, hist = om.solve(p, 60, record_every=10)
    assert np.all(np.diff(hist) < 0)
    assert om.snr_db(st.X, vi.sky) > 5.0
