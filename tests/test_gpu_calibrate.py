"""The two-step calibration of Sec. 4 on the library (paper_1602_08847_amd.calibrate): the mu_s sweep
runs every value at once as a batch with mu_lambda = 0, and each value's iterate equals a separate
context's bit for bit; the scores are the FP64 SNR against the truth and the noise discrepancy; step 2
from the chosen value's X matches the oracle's two-step run."""
import numpy as np
import pytest

from oracle import muffin as om
from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_mu_s_sweep_and_second_step(lib):
    from paper_1602_08847_amd import calibrate
    spec = synth.WORKLOADS["cube64_L8_J3"]
    c = synth.make_cube(spec, dtype=np.float32)
    truth = c.sky.astype(np.float32)
    mus, n1, n2 = [0.05, 0.25, 1.0], 60, 40
    res = calibrate.sweep_mu_s(c, 3, mus, n1, truth=truth, noise_sigma=spec.noise_sigma)
    assert [r["mu_s"] for r in res] == mus
    for r in res:
        with lib.Muffin(c.dirty, c.psf, J=3, mu_s=r["mu_s"], mu_lambda=0.0) as m:
            assert m.info()["tau"] == r["tau"]
            m.step(n1)
            np.testing.assert_array_equal(m.get_x().cpu().numpy(), r["x"].cpu().numpy())
            assert m.snr(truth) == r["snr_db"]
            f = m.objective()
        assert r["data_term"] == f[1]
        e = 64 * 64 * 8 * spec.noise_sigma ** 2
        assert r["discrepancy"] == pytest.approx(abs(2 * f[1] - e) / e, rel=1e-12)
    best = calibrate.choose(res)
    assert best["snr_db"] == max(r["snr_db"] for r in res)
    assert calibrate.choose([{k: v for k, v in r.items() if k != "snr_db"} for r in res])["discrepancy"] == min(
        r["discrepancy"] for r in res)
    two = calibrate.step_two(c, 3, best["mu_s"], 3.0, best["x"], n2, truth=truth)
    p = om.Problem(dirty=c.dirty.astype(np.float64), psf=c.psf.astype(np.float64), J=3, mu_s=best["mu_s"], mu_l=3.0)
    st1, st2 = om.two_step_calibration(p, n1, n2)
    assert rel(best["x"].double().cpu().numpy(), st1.X) < 1e-4
    assert rel(two["x"].double().cpu().numpy(), st2.X) < 1e-4
    assert two["snr_db"] == pytest.approx(om.snr_db(st2.X, truth.astype(np.float64)), abs=1e-3)
