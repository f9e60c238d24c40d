"""Parity of the warm-start CNN (BF16 MFMA kernels) against the FP64 oracle on BF16-rounded
operands: per layer forward, input gradient and weight gradient, the whole-network loss and
gradient, Adam over several steps, inference and the warm start."""
import numpy as np
import pytest

from oracle import cnn as oc
from oracle import muffin as om
from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def net(lib):
    with lib.Cnn(seed=3) as n:
        yield n


def rnd(shape, seed, scale=1.0):
    return np.random.default_rng(seed).normal(scale=scale, size=shape)


@pytest.mark.parametrize("layer", [1, 2, 3, 4])
@pytest.mark.parametrize("N", [32, 64, 96])
def test_layer_forward_and_backward(lib, net, layer, N):
    B = 2
    cin, cout = (1 if layer == 1 else 32), (1 if layer == 4 else 32)
    params = lib.cnn_params_to_oracle(net.get_params())
    w, b = params[layer - 1]
    x = rnd((B, cin, N, N), 10 + layer)
    dz = rnd((B, cout, N, N), 20 + layer, 1e-2)
    xr, wr, dzr = oc.bf16_round(x), oc.bf16_round(w), oc.bf16_round(dz)
    z = net.layer(layer, 0, x).double().cpu().numpy()
    # only the FP32 accumulation order differs from the oracle on identical BF16 operands
    assert rel(z, oc.conv_forward(xr, wr, b)) < 1e-5
    dx, dp = net.layer(layer, 1, x, dz)
    dw_ref, db_ref = oc.conv_weight_grad(xr, dzr)
    nw = cout * cin * 9
    assert rel(dp[:nw].reshape(w.shape), dw_ref) < 1e-5
    assert rel(dp[nw:], db_ref) < 1e-5
    if layer > 1:
        assert rel(dx.double().cpu().numpy(), oc.conv_data_grad(dzr, wr)) < 1e-5


def test_network_loss_and_gradient(lib, net):
    B, N = 2, 64
    x = np.abs(rnd((B, N, N), 31))
    t = np.abs(rnd((B, N, N), 32, 0.5))
    params = lib.cnn_params_to_oracle(net.get_params())
    out, acts = oc.forward(params, x[:, None], bf16=True)
    loss_ref, dout = oc.mse(out, t[:, None])
    grads = oc.backward(params, acts, dout, bf16=True)
    loss, g = net.loss_grad(x, t)
    assert loss == pytest.approx(loss_ref, rel=1e-4)
    # hidden activations are rounded to BF16 after an FP32 (GPU) or FP64 (oracle) sum, so a few
    # round-half decisions can differ; each such flip moves one activation by one BF16 ulp
    assert rel(g, lib.cnn_params_from_oracle(grads)) < 2e-3
    pred = net.predict(x).double().cpu().numpy()
    assert rel(pred, out[:, 0]) < 2e-3


def bf16_round(a):
    """FP32 -> nearest BF16 (ties to even), returned as FP32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def test_inference_equals_the_layer_chain_bitwise(lib, net):
    """predict runs layers 1 and 2 in one pass (a1 stays in LDS); chaining the single-layer launches
    on the host, with the same ReLU and BF16 rounding between them, must give the same bits."""
    B, N = 2, 64
    x = np.abs(rnd((B, N, N), 41)).astype(np.float32)
    pred = net.predict(x).cpu().numpy()
    a = x[:, None]
    for layer in (1, 2, 3):
        z = net.layer(layer, 0, a).cpu().numpy()
        a = bf16_round(np.maximum(z, 0.0))
    z4 = net.layer(4, 0, a).cpu().numpy()[:, 0]
    np.testing.assert_array_equal(pred, z4)


def test_adam_steps_match_oracle(lib):
    """Four Adam steps (Kingma and Ba's recursion with bias correction, beta 0.9 / 0.999): the
    parameters after each step against the oracle's update chained from the same gradients, with
    the moments carried over (at t = 1 the moments cancel out of the update; from t = 2 on they
    do not)."""
    B, N = 2, 32
    x = np.abs(rnd((B, N, N), 41))
    t = np.abs(rnd((B, N, N), 42, 0.5))
    with lib.Cnn(seed=7) as n:
        p = n.get_params().astype(np.float64)
        m = np.zeros_like(p)
        v = np.zeros_like(p)
        for step in range(1, 5):
            _, g = n.loss_grad(x, t)
            n.train_step(x, t, lr=1e-3)
            got = n.get_params().astype(np.float64)
            p, m, v = oc.adam_update(p, g.astype(np.float64), m, v, t=step, lr=1e-3)
            np.testing.assert_allclose(got, p, rtol=1e-5, atol=1e-8, err_msg=f"step {step}")
            p = got  # the next gradient is taken at the GPU's parameters


def test_training_reduces_loss(lib):
    B, N = 4, 32
    x = np.abs(rnd((B, N, N), 51))
    t = 0.5 * x
    with lib.Cnn(seed=9) as n:
        first = n.train_step(x, t, lr=3e-3)
        for _ in range(60):
            last = n.train_step(x, t, lr=3e-3)
    assert last < 0.2 * first


def test_warm_start_sets_positive_part_of_prediction(lib, net):
    """The warm start's input is y_l / g_l (g_l the PSF's 9 x 9 main-lobe sum); X becomes the
    positive part of the network's output on exactly that input, bit for bit, with U = V = 0."""
    c = synth.make_cube(synth.CubeSpec(N=64, L=4, J=2, n_sources=4, n_baselines=100, seed=3))
    with lib.Muffin(c.dirty, c.psf, J=2, mu_s=0.25, mu_lambda=3.0) as m:
        inp = m.warm_input()
        m.warm_start(net)
        X = m.get_x().cpu().numpy()
        assert np.all(m.get_u().cpu().numpy() == 0) and np.all(m.get_v().cpu().numpy() == 0)
    N, h = c.dirty.shape[-1], 4
    psf = c.psf.astype(np.float32).astype(np.float64)
    gain = psf[:, N // 2 - h:N // 2 + h + 1, N // 2 - h:N // 2 + h + 1].sum(axis=(1, 2))
    ref_in = c.dirty.astype(np.float32).astype(np.float64) / gain[:, None, None]
    assert rel(inp.double().cpu().numpy(), ref_in) < 1e-6
    pred = np.maximum(net.predict(inp).cpu().numpy(), 0)
    np.testing.assert_array_equal(X, pred)
    assert np.mean(X > 0) > 0.05


def test_trained_warm_start_gains_over_cold_start(lib):
    """A network trained by the library's own kernels on plain-solver solutions of small cubes
    starts a held-out cube at a lower objective and stays ahead at equal iteration counts."""
    from paper_1602_08847_amd import warmstart as ws
    spec = synth.CubeSpec(N=64, L=8, J=3, n_sources=5, n_baselines=200)
    inputs, targets = ws.build_training_set(12, spec, 1500, sigma=100.0, seed0=20000, log=None)
    with lib.Cnn(seed=2) as n:
        hist = ws.train(n, inputs, targets, epochs=25, batch=8, lr=1e-3, log=None)
        assert hist[-1] < 0.2 * hist[0]
        cube = synth.make_cube(synth.CubeSpec(N=64, L=8, J=3, n_sources=5, n_baselines=200, seed=31))
        f = {}
        for mode in ("cold", "warm"):
            with lib.Muffin(cube.dirty, cube.psf, J=3, mu_s=ws.MU_S, mu_lambda=ws.MU_L, sigma=100.0) as m:
                if mode == "warm":
                    m.warm_start(n)
                f[mode] = [m.objective()[0]]
                for k in (200, 800):
                    m.step(k)
                    f[mode].append(m.objective()[0])
        # the fixed-budget comparison: the warm start reaches the cold run's 1000-iteration objective sooner
        b = ws.compare_budget(n, cube, 3, 100.0, budget=1000, check_every=50)
    assert all(w < c for w, c in zip(f["warm"], f["cold"])), f
    assert b["f_target"] == pytest.approx(f["cold"][-1], rel=1e-12)
    assert b["warm_reached"] and b["warm_iters"] < b["cold_iters"] and b["warm_f"] <= b["f_target"], b


def test_time_to_tolerance_runs_through_muffin_solve(lib):
    """The warm-start study's clock: time_to_tolerance stops where a plain step/objective loop with
    the same checks first meets the gap (the library's f_ref rule), for the cold start and for the
    two-step protocol of Sec. 4 (mu_lambda = 0 first, then the full method from its X)."""
    from paper_1602_08847_amd import warmstart as ws
    cube = synth.make_cube(synth.CubeSpec(N=64, L=8, J=3, n_sources=5, n_baselines=200, seed=33))
    f_ref = ws.reference_objective(cube, 3, 100.0, 4000)
    tol, every = 1e-2, 20
    cold = ws.compare_cold(cube, 3, 100.0, tol, f_ref, every, 4000)
    with lib.Muffin(cube.dirty, cube.psf, J=3, mu_s=ws.MU_S, mu_lambda=ws.MU_L, sigma=100.0) as m:
        it, f = 0, m.objective()[0]
        while (f - f_ref) / abs(f_ref) > tol:
            m.step(every)
            it += every
            f = m.objective()[0]
    assert cold["cold_iters"] == it and cold["cold_f"] == f
    assert (cold["cold_f"] - f_ref) / abs(f_ref) <= tol
    two = ws.compare_two_step(cube, 3, 100.0, tol, f_ref, 200, every, 4000)
    assert (two["two_step_f"] - f_ref) / abs(f_ref) <= tol and two["two_step_iters"] > 0
    assert two["snr0_two_step_db"] > 0
