"""Per-operator parity of the HIP path against the FP64 oracle (relative L2 <= 1e-5 in FP32).

Every operator is called through the C ABI (muffin_apply_op) on seeded inputs and compared
element by element with the oracle on the same inputs.
"""
import numpy as np
import pytest

from oracle import muffin as om
from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5  # relative L2 per operator, FP32 against FP64


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


SHAPES = [
    # (N, L, J, gen): the small parity cube, ragged and degenerate cases, radix-3 sizes,
    # scales whose taps wrap around the image
    (64, 8, 3, 2), (64, 8, 3, 1), (8, 1, 3, 2), (8, 3, 1, 1), (12, 5, 2, 2), (16, 2, 3, 2),
    (96, 7, 3, 2), (128, 17, 4, 2), (384, 3, 4, 2), (256, 64, 4, 2), (32, 33, 2, 1), (48, 48, 3, 2),
    # channel counts above 256 without an FFT plan, and a radix-3 plan
    (8, 260, 2, 2), (8, 384, 2, 2),
    # the largest image sides: 512, the radix-3 768 and 1024 (at J = 6: scale triples 0-2 and 3-5)
    (512, 2, 5, 2), (768, 2, 4, 1), (1024, 2, 6, 2),
]


def make(N, L, J, seed=0):
    spec = synth.CubeSpec(N=N, L=L, J=J, n_sources=max(2, N // 16), n_baselines=max(8, N * 2), seed=seed)
    return synth.make_cube(spec)


@pytest.fixture(scope="module")
def ctxs(lib):
    cache = {}

    def get(N, L, J, gen):
        key = (N, L, J, gen)
        if key not in cache:
            c = make(N, L, J)
            m = lib.Muffin(f32(c.dirty), f32(c.psf), J=J, mu_s=0.25, mu_lambda=3.0, iuwt_gen=gen)
            cache[key] = (c, m)
        return cache[key]
    yield get
    for _, m in cache.values():
        m.close()


@pytest.mark.parametrize("N,L,J,gen", SHAPES)
def test_convolution_ops(lib, ctxs, N, L, J, gen):
    c, m = ctxs(N, L, J, gen)
    psf = f32(c.psf)
    x = f32(np.random.default_rng(1).normal(size=(L, N, N)))
    assert rel(m.apply_op(lib.OP_H, x).cpu().numpy(), om.apply_H(psf, x)) < TOL
    assert rel(m.apply_op(lib.OP_HT, x).cpu().numpy(), om.apply_Ht(psf, x)) < TOL
    g = om.data_gradient(psf, x, f32(c.dirty))
    assert rel(m.apply_op(lib.OP_GRAD, x).cpu().numpy(), g) < TOL


@pytest.mark.parametrize("N,L,J,gen", SHAPES)
def test_iuwt_ops(lib, ctxs, N, L, J, gen):
    c, m = ctxs(N, L, J, gen)
    r = np.random.default_rng(2)
    x = f32(r.normal(size=(L, N, N)))
    ref = np.stack([om.iuwt(x[l], J, gen) for l in range(L)])
    assert rel(m.apply_op(lib.OP_IUWT, x).cpu().numpy(), ref) < TOL
    u = f32(r.normal(size=(L, J + 1, N, N)))
    ref = np.stack([om.iuwt_adjoint(u[l], J, gen) for l in range(L)])
    assert rel(m.apply_op(lib.OP_IUWT_ADJ, u).cpu().numpy(), ref) < TOL


def check_iuwt_sched(lib, m, N, L, J, gen, seed):
    x = f32(0.05 * np.random.default_rng(seed).normal(size=(L, N, N)))
    ref = np.stack([om.iuwt(x[l], J, gen) for l in range(L)])
    assert np.max(np.abs(ref)) < 1.0  # the dual step's saturation stays inactive
    got = m.apply_op(lib.OP_IUWT_SCHED, x).cpu().numpy()
    assert rel(got, ref) < TOL
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,L,J,gen", SHAPES)
def test_iuwt_through_the_iteration_kernels(lib, ctxs, N, L, J, gen):
    """W_s through the analysis launches the iteration itself runs (scale triples and pairs with the
    dual step on zero planes), not the operator-only smoothing kernels."""
    c, m = ctxs(N, L, J, gen)
    check_iuwt_sched(lib, m, N, L, J, gen, 12)


@pytest.mark.parametrize("N,L,J", [(64, 8, 4), (128, 17, 4), (64, 5, 5), (256, 64, 4), (32, 3, 2)])
def test_iuwt_through_the_fused_tail(lib, N, L, J):
    """The same with the fused tail forced on: the last two scales and the coarse plane come from the
    fused analysis + next-adjoint launch."""
    c = make(N, L, J, seed=5)
    with lib.Muffin(f32(c.dirty), f32(c.psf), J=J, mu_s=0.25, mu_lambda=3.0, flags=lib.FLAG_FUSED_TAIL) as m:
        check_iuwt_sched(lib, m, N, L, J, 2, 13)


@pytest.mark.parametrize("N,L,J,gen", SHAPES)
def test_dct_ops(lib, ctxs, N, L, J, gen):
    c, m = ctxs(N, L, J, gen)
    x = f32(np.random.default_rng(3).normal(size=(L, N, N)))
    assert rel(m.apply_op(lib.OP_DCT, x).cpu().numpy(), om.spectral(x)) < TOL
    assert rel(m.apply_op(lib.OP_IDCT, x).cpu().numpy(), om.spectral_adjoint(x)) < TOL


@pytest.mark.parametrize("N,L,J,gen", SHAPES[:6])
def test_step_size_constants(lib, ctxs, N, L, J, gen):
    c, m = ctxs(N, L, J, gen)
    p = om.Problem(dirty=f32(c.dirty), psf=f32(c.psf), J=J, mu_s=0.25, mu_l=3.0, gen=gen)
    tau, sigma, rho, beta, k2 = om.step_sizes(p)
    info = m.info()
    assert info["beta"] == pytest.approx(beta, rel=1e-6)
    assert info["Ws2"] == pytest.approx(1.0, abs=1e-12)
    assert info["K2"] == pytest.approx(k2, rel=1e-6)
    assert info["tau"] == pytest.approx(tau, rel=1e-6)


@pytest.mark.parametrize("N,L,J,gen", [(64, 8, 3, 2), (96, 7, 3, 1), (8, 1, 3, 2)])
def test_objective_evaluation(lib, ctxs, N, L, J, gen):
    """FP64 objective reductions at a fixed X against the oracle's objective at the same X."""
    c, m = ctxs(N, L, J, gen)
    x = f32(np.abs(np.random.default_rng(4).normal(size=(L, N, N))))
    m.set_x(x)
    got = m.objective()
    p = om.Problem(dirty=f32(c.dirty), psf=f32(c.psf), J=J, mu_s=0.25, mu_l=3.0, gen=gen)
    ref = om.objective(p, x)
    np.testing.assert_allclose(got, ref, rtol=1e-6)
