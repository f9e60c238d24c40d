"""The channel-sampled two-pass evaluation used by the full-size GPU parity test equals two calls of
the oracle's whole-cube iteration on the sampled channels (and in full for X1 and V1)."""
import numpy as np
import pytest

from oracle import muffin as om
from paper_1602_08847_amd import synth
from two_step_oracle import data_gradient_threaded, two_passes_sampled


@pytest.mark.parametrize("rho,pc,gen", [(1.0, True, 2), (0.7, False, 2), (1.0, True, 1)])
def test_sampled_two_passes_equal_whole_cube_iteration(rho, pc, gen):
    c = synth.make_cube(synth.CubeSpec(N=32, L=7, J=3, n_sources=4, n_baselines=80, seed=3))
    dirty, psf = c.dirty.astype(np.float64), c.psf.astype(np.float64)
    omega = np.ones(4)
    omega[3] = 1.0 if pc else 0.0
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=3.0, gen=gen, omega=omega, sigma=2.0, rho=rho)
    tau = om.step_sizes(p)[0]
    X0 = np.random.default_rng(4).normal(size=dirty.shape) * 0.5 + 0.2  # negative entries: clipped at init
    s1 = om.iterate(p, om.init_state(p, X0), tau)
    s2 = om.iterate(p, s1, tau)
    chans = [0, 4, 6]
    got = two_passes_sampled(dirty, psf, X0, 3, 0.25, 3.0, tau, chans, sigma=2.0, rho=rho, omega=omega, gen=gen,
                             workers=3)
    np.testing.assert_allclose(got["X1"], s1.X, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["V1"], s1.V, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["U1"], s1.U[chans], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["X2"], s2.X[chans], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got["U2"], s2.U[chans], rtol=1e-12, atol=1e-14)
    # the case is not degenerate: both branches of each clip are taken
    assert 0 < np.mean(s2.X == 0) < 1
    assert 0 < np.mean(np.abs(s1.V) == rho) < 1  # V0 = 0: saturated entries are +-rho


def test_threaded_gradient_is_the_oracle_gradient():
    r = np.random.default_rng(5)
    x, y, psf = r.random((10, 16, 16)), r.random((10, 16, 16)), r.random((10, 16, 16))
    np.testing.assert_array_equal(data_gradient_threaded(psf, x, y, workers=3, chunk=3),
                                  om.data_gradient(psf, x, y))
