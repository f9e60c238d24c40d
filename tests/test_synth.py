"""The seeded generator: determinism, PSF layout and the paper's printed step sizes."""
import json
import os

import numpy as np

from oracle import muffin as om
from paper_1602_08847_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def test_generator_is_deterministic_and_psf_peaks_at_centre():
    spec = synth.CubeSpec(N=32, L=4, J=2, n_sources=3, n_baselines=40, seed=5)
    a = synth.make_cube(spec)
    b = synth.make_cube(spec)
    np.testing.assert_array_equal(a.dirty, b.dirty)
    for l in range(4):
        assert np.argmax(a.psf[l]) == 16 * 32 + 16
        assert a.psf[l].max() == 1.0 and a.psf[l].min() >= 0.0
    assert np.all(a.sky > 0)
    # the first channel has nu = nu_0, so its source peaks are exactly U[0.5, 1] draws
    assert a.sky[0].max() <= 1.0 + 1e-12


def test_dirty_is_psf_convolved_sky_plus_noise():
    spec = synth.CubeSpec(N=32, L=3, J=2, n_sources=4, n_baselines=60, seed=9, noise_sigma=0.0)
    c = synth.make_cube(spec)
    np.testing.assert_allclose(om.apply_H(c.psf, c.sky), c.dirty, atol=1e-10)


def test_paper_step_sizes_satisfy_convergence_condition_on_synthetic_cube():
    """With peak-normalised PSFs the paper's printed (rho, sigma, tau) = (1, 1, 1e-5), Sec. 4,
    satisfy the primal-dual convergence condition on the small synthetic cube."""
    g = json.load(open(GOLDEN))
    cube = synth.make_cube(synth.WORKLOADS["cube64_L8_J3"])
    p = om.Problem(dirty=cube.dirty, psf=cube.psf, J=3, mu_s=g["mu_s"]["value"],
                   mu_l=g["mu_lambda"]["value"], tau=g["tau"]["value"], sigma=g["sigma"]["value"],
                   rho=g["rho"]["value"])
    tau, sigma, rho, beta, k2 = om.step_sizes(p)
    assert tau == 1e-5 and 1 / tau - sigma * k2 > beta / 2


def test_cubes_drawn_by_worker_processes_match_the_serial_draw():
    """The warm-start training set may be drawn by forked host processes (--gen-workers): the cubes
    depend only on their spec and seed, so they equal the serial draw bit for bit."""
    import multiprocessing as mp
    spec = synth.CubeSpec(N=32, L=4, J=2, n_sources=3, n_baselines=40)
    specs = [synth.CubeSpec(**{**spec.__dict__, "seed": 10000 + i}) for i in range(4)]
    with mp.get_context("fork").Pool(2) as pool:
        got = [r.get() for r in [pool.apply_async(synth.make_cube, (s, np.float32, False)) for s in specs]]
    for g, s in zip(got, specs):
        ref = synth.make_cube(s, dtype=np.float32, with_sky=False)
        np.testing.assert_array_equal(g.dirty, ref.dirty)
        np.testing.assert_array_equal(g.psf, ref.psf)
