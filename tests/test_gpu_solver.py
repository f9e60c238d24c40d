"""Iteration-level parity of the HIP path against the FP64 oracle, closed-form special cases,
checkpoint/resume, error paths and graph replay."""
import numpy as np
import pytest

from oracle import muffin as om
from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def small():
    c = synth.make_cube(synth.WORKLOADS["cube64_L8_J3"])
    return c


@pytest.mark.parametrize("gen", [2, 1])
def test_trajectory_matches_oracle_small_cube(lib, small, gen):
    """64x64x8, J=3, 50 iterations of Algorithm 1 from X = U = V = 0 with the same tau."""
    c = small
    dirty, psf = f32(c.dirty), f32(c.psf)
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=3.0, gen=gen)
    tau = om.step_sizes(p)[0]
    st, _ = om.solve(p, 50, tau=tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, iuwt_gen=gen, tau=tau) as m:
        m.step(50)
        X = m.get_x().double().cpu().numpy()
        U = m.get_u().double().cpu().numpy()
        V = m.get_v().double().cpu().numpy()
        f = m.objective()[0]
    f_ref = om.objective(p, st.X)[0]
    assert rel(X, st.X) < 1e-4
    assert rel(U, st.U) < 1e-4
    assert rel(V, st.V) < 1e-4
    assert abs(f - f_ref) / abs(f_ref) < 1e-4


@pytest.mark.parametrize("penalize_coarse,rho", [(False, 1.0), (True, 0.8)])
def test_trajectory_coarse_plane_and_relaxation(lib, small, penalize_coarse, rho):
    """The last analysis scale updates the coarse dual in the same launch; check it with the coarse
    plane unpenalised (omega = 0 there, its dual stays 0) and with relaxation rho < 1."""
    c = small
    dirty, psf = f32(c.dirty), f32(c.psf)
    omega = np.ones(4)
    omega[3] = 1.0 if penalize_coarse else 0.0
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=3.0, omega=omega, sigma=10.0, rho=rho)
    tau = om.step_sizes(p)[0]
    st, _ = om.solve(p, 20, tau=tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, penalize_coarse=penalize_coarse, tau=tau,
                    sigma=10.0, rho=rho) as m:
        m.step(20)
        X = m.get_x().double().cpu().numpy()
        U = m.get_u().double().cpu().numpy()
        V = m.get_v().double().cpu().numpy()
    assert rel(X, st.X) < 1e-4
    assert rel(U, st.U) < 1e-4
    assert rel(V, st.V) < 1e-4
    if not penalize_coarse:
        assert np.all(U[:, 3] == 0)


def test_single_iteration_matches_oracle_tightly(lib, small):
    c = small
    dirty, psf = f32(c.dirty), f32(c.psf)
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=3.0)
    tau = om.step_sizes(p)[0]
    x0 = f32(np.abs(np.random.default_rng(5).normal(size=dirty.shape)))
    st = om.iterate(p, om.init_state(p, x0), tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        m.set_x(x0)
        m.step(1)
        assert rel(m.get_x().double().cpu().numpy(), st.X) < 1e-5
        assert rel(m.get_u().double().cpu().numpy(), st.U) < 1e-5
        assert rel(m.get_v().double().cpu().numpy(), st.V) < 1e-5


SPECTRAL_PATHS = [
    # Bluestein DFTs (flag 64) through FFTs of length M = 64, 96, 128, 192, 256, 384, 512, 768, 1024
    (16, 17, 64), (16, 37, 64), (16, 50, 64), (16, 70, 64), (16, 100, 64), (16, 150, 64), (16, 200, 64),
    (16, 300, 64), (8, 511, 64),
    # the cosine-table paths (flag 32): dense products for L <= 256 (kernels for up to 128 and 256
    # channels), the direct kernel beyond
    (16, 100, 32), (16, 200, 32), (16, 260, 32),
    # by default: dense products (L = 11, 100), Bluestein (L = 120, 260), an FFT with a radix-3 plan
    (16, 11, 0), (16, 100, 0), (16, 120, 0), (16, 260, 0), (16, 384, 0),
    # radix-3 plans with 16 and 8 transforms per block; the largest power-of-two plan
    (16, 48, 0), (16, 96, 0), (16, 192, 0), (8, 512, 0),
]


@pytest.mark.parametrize("N,L,flags", SPECTRAL_PATHS)
def test_single_iteration_spectral_paths(lib, N, L, flags):
    """Two iterations with the spectral step on each of its paths against the oracle: flags 64
    (FLAG_SPECTRAL_BLUESTEIN) and 32 (FLAG_SPECTRAL_DENSE) force the form of the cosine transforms
    for channel counts without an FFT plan; 0 takes the default choice."""
    c = synth.make_cube(synth.CubeSpec(N=N, L=L, J=2, n_sources=3, n_baselines=40, seed=L))
    dirty, psf = f32(c.dirty), f32(c.psf)
    p = om.Problem(dirty=dirty, psf=psf, J=2, mu_s=0.25, mu_l=3.0)
    tau = om.step_sizes(p)[0]
    r = np.random.default_rng(6)
    x0 = f32(np.abs(r.normal(size=dirty.shape)))
    st = om.iterate(p, om.init_state(p, x0), tau)
    st = om.iterate(p, st, tau)
    with lib.Muffin(dirty, psf, J=2, mu_s=0.25, mu_lambda=3.0, tau=tau, flags=flags) as m:
        m.set_x(x0)
        m.step(2)
        assert rel(m.get_x().double().cpu().numpy(), st.X) < 1e-5
        assert rel(m.get_u().double().cpu().numpy(), st.U) < 1e-5
        assert rel(m.get_v().double().cpu().numpy(), st.V) < 1e-5


def delta_psf(L, N):
    psf = np.zeros((L, N, N))
    psf[:, N // 2, N // 2] = 1.0
    return psf


def test_closed_form_positive_part(lib):
    Y = f32(np.random.default_rng(6).normal(size=(3, 16, 16)))
    with lib.Muffin(Y, delta_psf(3, 16), J=2, mu_s=0.0, mu_lambda=0.0) as m:
        m.step(1500)
        # tau = 1.98 makes x <- -0.98 x + 1.98 y a 0.98-contraction, which amplifies the FFT
        # rounding of H^T H x (about 1e-7 max|x|, spread over every pixel) by 1.98 / 0.02 = 100
        np.testing.assert_allclose(m.get_x().cpu().numpy(), np.maximum(Y, 0), rtol=0,
                                   atol=3e-5 * np.abs(Y).max())


def test_closed_form_single_channel_soft_threshold(lib):
    Y = f32(np.random.default_rng(7).normal(scale=2.0, size=(1, 16, 16)))
    with lib.Muffin(Y, delta_psf(1, 16), J=2, mu_s=0.0, mu_lambda=0.7) as m:
        m.step(4000)
        np.testing.assert_allclose(m.get_x().cpu().numpy(), np.maximum(Y - 0.7, 0), atol=1e-5)


def test_closed_form_spectral_soft_threshold(lib):
    L = 5
    Y = f32(50.0 + np.random.default_rng(8).normal(size=(L, 8, 8)))
    with lib.Muffin(Y, delta_psf(L, 8), J=1, mu_s=0.0, mu_lambda=0.4) as m:
        m.step(4000)
        W = om.dct_matrix(L)
        expect = np.tensordot(W, om.soft(np.tensordot(W.T, Y, axes=(1, 0)), 0.4), axes=(1, 0))
        np.testing.assert_allclose(m.get_x().cpu().numpy(), expect, atol=2e-4)


# with the fused tail (J = 4 and 5, flag 4) the checkpoint is taken with its planes in the second
# buffer (7 iterations), and the carried adjoint sum is rebuilt after set_state
@pytest.mark.parametrize("J,flags", [(3, 0), (5, 2), (4, 4), (5, 4)])
def test_checkpoint_resume_is_bitwise(lib, small, J, flags):
    c = small
    kw = dict(J=J, mu_s=0.25, mu_lambda=3.0, flags=flags)
    with lib.Muffin(c.dirty, c.psf, **kw) as a:
        a.step(7)
        blob = a.get_state()
        a.step(5)
        xa = a.get_x().cpu().numpy()
    with lib.Muffin(c.dirty, c.psf, **kw) as b:
        b.set_state(blob)
        assert b.info()["iter"] == 7
        b.step(5)
        xb = b.get_x().cpu().numpy()
    np.testing.assert_array_equal(xa, xb)


def test_checkpoint_rejects_other_parameters(lib, small):
    c = small
    with lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=3.0) as a:
        blob = a.get_state()
    with lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.5, mu_lambda=3.0) as b:
        with pytest.raises(lib.MuffinError) as e:
            b.set_state(blob)
        assert e.value.code == lib.ESTATE


@pytest.mark.parametrize("J,flags,gen", [(3, 0, 2), (5, 2, 2), (5, 4, 2), (5, 0, 1)])
def test_graph_replay_equals_eager_launches(lib, small, J, flags, gen):
    c = small
    kw = dict(J=J, mu_s=0.25, mu_lambda=3.0, flags=flags, iuwt_gen=gen)
    with lib.Muffin(c.dirty, c.psf, **kw) as a, lib.Muffin(c.dirty, c.psf, **kw) as b:
        a.step(5)
        b.profile(5)
        np.testing.assert_array_equal(a.get_x().cpu().numpy(), b.get_x().cpu().numpy())
        np.testing.assert_array_equal(a.get_u().cpu().numpy(), b.get_u().cpu().numpy())
        np.testing.assert_array_equal(a.get_v().cpu().numpy(), b.get_v().cpu().numpy())
        a.step(2)  # the two paths also continue alike
        b.step(2)
        np.testing.assert_array_equal(a.get_x().cpu().numpy(), b.get_x().cpu().numpy())


def test_error_paths(lib, small):
    c = small
    bad = np.array(c.dirty, dtype=np.float32)
    bad[3, 5, 7] = np.nan
    with pytest.raises(lib.MuffinError) as e:
        lib.Muffin(bad, c.psf, J=3, mu_s=0.25, mu_lambda=3.0)
    assert e.value.code == lib.ENONFINITE
    with pytest.raises(lib.MuffinError) as e:
        lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=1.0)
    assert e.value.code == lib.ESTEP
    with pytest.raises(lib.MuffinError) as e:
        lib.Muffin(c.dirty, c.psf, J=9, mu_s=0.25, mu_lambda=3.0)
    assert e.value.code == lib.EINVAL
    with pytest.raises(lib.MuffinError) as e:
        lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=3.0, rho=1.9)
    assert e.value.code == lib.ESTEP
