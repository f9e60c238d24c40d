"""The library's stopping machinery against the FP64 oracle: convergence norms of a monitored
iteration, the SNR of Sec. 4, both stopping rules of muffin_solve, and the mu_lambda = 0 path that
the first calibration step of Sec. 4 uses (the primal step in the gradient's last pass), with the
two-step calibration of Sec. 4 on the GPU."""
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
    dirty, psf = f32(c.dirty), f32(c.psf)
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=3.0)
    return c, dirty, psf, p, om.step_sizes(p)[0]


def norms(a, b):
    return np.linalg.norm(a - b), np.linalg.norm(a)


def test_monitored_norms_are_the_fp64_norms_of_the_iterates(lib, small):
    """The reduction itself: FP64 sums over the GPU's own iterates (read back before and after the
    monitored iteration), at both parities of the fused tail's alternating planes and without the
    fused tail; and n > 1 monitors only the last of its n iterations."""
    c, dirty, psf, p, tau = small

    def state(m):
        return [t.double().cpu().numpy() for t in (m.get_x(), m.get_u(), m.get_v())]

    for flags in (lib.FLAG_FUSED_TAIL, lib.FLAG_NO_FUSED_TAIL):
        with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau, flags=flags) as m:
            for n in (1, 2, 1):  # the iteration count changes parity between the monitored iterations
                if n > 1:
                    m.step(n - 1)
                before = state(m)
                r = m.step_monitored(1)
                after = state(m)
                for key, a, b in zip(("X", "U", "V"), after, before):
                    d, nrm = norms(a, b)
                    assert d > 0
                    assert r["d" + key] == pytest.approx(d, rel=1e-12), (flags, n, key)
                    assert r[key] == pytest.approx(nrm, rel=1e-12), (flags, n, key)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m1, \
            lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m2:
        r1 = m1.step_monitored(5)
        m2.step(4)
        r2 = m2.step_monitored(1)
        assert r1 == r2
        assert m1.info()["iter"] == m2.info()["iter"] == 5


def test_monitored_norms_match_the_oracle_trajectory(lib, small):
    """After 20 iterations from zero: the changes of the last iteration against the oracle's
    (a difference of two nearby iterates loses digits, so the bound is 1e-3 against 1e-4 for
    the iterates themselves)."""
    c, dirty, psf, p, tau = small
    st19, _ = om.solve(p, 19, tau=tau)
    st20 = om.iterate(p, st19, tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        r = m.step_monitored(20)
        assert m.info()["iter"] == 20
    for key, a, b in (("X", st20.X, st19.X), ("U", st20.U, st19.U), ("V", st20.V, st19.V)):
        d, nrm = norms(a, b)
        assert r["d" + key] == pytest.approx(d, rel=1e-3), key
        assert r[key] == pytest.approx(nrm, rel=1e-4), key


def test_snr_against_a_truth(lib, small):
    c, dirty, psf, p, tau = small
    sky = f32(c.sky)
    st, _ = om.solve(p, 30, tau=tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        m.step(30)
        X = m.get_x().double().cpu().numpy()
        s = m.snr(sky)
        m.set_x(sky)
        assert m.snr(sky) == np.inf
    assert s == pytest.approx(om.snr_db(X, sky), abs=1e-9)  # the FP64 reduction over the GPU's X
    assert s == pytest.approx(om.snr_db(st.X, sky), abs=1e-3)  # and the oracle's iterate


def test_solve_stops_on_the_objective_gap(lib, small):
    """f_ref mode: the run stops at the first check where (f - f_ref)/|f_ref| <= tol.  tol is
    placed halfway between the oracle's gaps at two consecutive checks, far from both, so the
    oracle fixes the stopping iteration; f_final is the objective there."""
    c, dirty, psf, p, tau = small
    every, n = 10, 120
    st, hist = om.solve(p, n, tau=tau, record_every=every)
    f_ref = hist[-1] * (1 - 1e-3)
    gaps = (hist - f_ref) / abs(f_ref)
    k = int(np.argmax(gaps < 0.1 * gaps[0]))  # the first check well below the first gap
    assert k > 0 and np.all(gaps[:k] > gaps[k])
    tol = 0.5 * (gaps[k] + np.min(gaps[:k]))
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        it, f = m.solve(n, check_every=every, tol=tol, f_ref=f_ref)
        assert it == (k + 1) * every
        assert f == pytest.approx(hist[k], rel=1e-4)
        assert m.objective()[0] == f
        # relative change of f between checks, no reference: stops where the oracle's change drops
        # below a tol placed between two consecutive changes
        m.set_x(np.zeros(dirty.shape))
    ch = np.abs(np.diff(hist)) / np.abs(hist[1:])
    j = int(np.argmax(ch < 0.5 * ch[0]))  # first check whose change is well below the first one
    assert j > 0 and np.all(ch[:j] > ch[j])
    tol2 = 0.5 * (ch[j] + np.min(ch[:j]))
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        it2, f2 = m.solve(n, check_every=every, tol=tol2)
    assert it2 == (j + 2) * every  # change j compares checks j and j + 1 (1-based: j + 2)
    assert f2 == pytest.approx(hist[j + 1], rel=1e-4)


def test_solve_stops_on_the_change_of_the_iterates(lib, small):
    """MUFFIN_STOP_CHANGE: the oracle's relative changes of X, U, V over the last iteration of each
    window fix the stopping window (tol halfway between two windows' values); the partial last
    window and max_iter = 0 are exercised too."""
    c, dirty, psf, p, tau = small
    every, n = 7, 70
    st = om.init_state(p)
    ratios = []
    for it in range(1, n + 1):
        nxt = om.iterate(p, st, tau)
        if it % every == 0:
            r = [np.linalg.norm(a - b) / np.linalg.norm(a) for a, b in ((nxt.X, st.X), (nxt.U, st.U), (nxt.V, st.V))]
            ratios.append(max(r))
        st = nxt
    ratios = np.array(ratios)
    k = int(np.argmax(ratios < 0.6 * ratios[0]))
    assert k > 0 and np.all(ratios[:k] > ratios[k])
    tol = 0.5 * (ratios[k] + np.min(ratios[:k]))
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        it, f = m.solve(n, check_every=every, tol=tol, rule=lib.STOP_CHANGE)
        assert it == (k + 1) * every
        assert f == pytest.approx(om.objective(p, om.solve(p, it, tau=tau)[0].X)[0], rel=1e-4)
        assert m.objective()[0] == f
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau) as m:
        # a tolerance never met: runs max_iter with a shorter last window
        it, f = m.solve(16, check_every=every, tol=0.0, rule=lib.STOP_CHANGE)
        assert it == 16 and m.info()["iter"] == 16
        it0, f0 = m.solve(0, check_every=every, tol=0.0, rule=lib.STOP_CHANGE)
        assert it0 == 0 and f0 == m.objective()[0]
        with pytest.raises(lib.MuffinError):
            m.solve(5, check_every=every, tol=0.0, rule=7)


@pytest.mark.parametrize("gen,rho", [(2, 1.0), (1, 1.0), (2, 0.8)])
def test_spectral_weight_zero_trajectory_matches_oracle(lib, small, gen, rho):
    """mu_lambda = 0 runs the primal step in the gradient's last pass and skips the spectral kernel:
    50 iterations against the oracle (one iteration at 1e-5), V stays 0."""
    c, dirty, psf, _, _ = small
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=0.0, gen=gen, rho=rho, sigma=5.0)
    tau = om.step_sizes(p)[0]
    x0 = f32(np.abs(np.random.default_rng(8).normal(size=dirty.shape)))
    one = om.iterate(p, om.init_state(p, x0), tau)
    st, _ = om.solve(p, 50, tau=tau)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=0.0, iuwt_gen=gen, rho=rho, sigma=5.0, tau=tau) as m:
        m.set_x(x0)
        m.step(1)
        assert rel(m.get_x().double().cpu().numpy(), one.X) < 1e-5
        assert rel(m.get_u().double().cpu().numpy(), one.U) < 1e-5
        m.set_x(np.zeros(dirty.shape))
        m.step(50)
        X = m.get_x().double().cpu().numpy()
        U = m.get_u().double().cpu().numpy()
        assert np.all(m.get_v().cpu().numpy() == 0)
        f = m.objective()
    assert rel(X, st.X) < 1e-4 and rel(U, st.U) < 1e-4
    assert f[3] == 0.0
    assert f[0] == pytest.approx(om.objective(p, st.X)[0], rel=1e-4)


def test_spectral_weight_zero_is_separable_bit_for_bit(lib, small):
    """With mu_lambda = 0 the problem separates over the channels (Sec. 4, step 1): the cube's
    iterates equal those of one context per channel, bit for bit (same tau)."""
    c, dirty, psf, _, _ = small
    p = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=0.0)
    tau = om.step_sizes(p)[0]
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=0.0, tau=tau) as m:
        m.step(25)
        X = m.get_x().cpu().numpy()
        U = m.get_u().cpu().numpy()
    for l in range(dirty.shape[0]):
        with lib.Muffin(dirty[l:l + 1], psf[l:l + 1], J=3, mu_s=0.25, mu_lambda=0.0, tau=tau) as m1:
            m1.step(25)
            np.testing.assert_array_equal(m1.get_x().cpu().numpy()[0], X[l])
            np.testing.assert_array_equal(m1.get_u().cpu().numpy()[0], U[l])


def test_spectral_weight_zero_in_a_batch(lib):
    """Cubes with mu_lambda = 0 in a batch group take the same path, each with its own tau, and
    equal separate contexts bit for bit; a group mixing mu_lambda = 0 with mu_lambda > 0 keeps
    the spectral kernel and still matches separate contexts within 1e-5."""
    cs = [synth.make_cube(synth.CubeSpec(N=32, L=L, J=2, n_sources=3, n_baselines=60, seed=40 + L)) for L in (3, 5)]
    for mls in ([0.0, 0.0], [0.0, 2.0]):
        with lib.Batch([(c.dirty, c.psf) for c in cs], J=2, mu_s=0.3, mu_lambda=mls) as b:
            b.step(15)
            got = [b.get_x(i).cpu().numpy() for i in range(2)]
            taus = [b.info(i)["tau"] for i in range(2)]
        for i, c in enumerate(cs):
            with lib.Muffin(c.dirty, c.psf, J=2, mu_s=0.3, mu_lambda=mls[i], tau=taus[i]) as m:
                m.step(15)
                ref = m.get_x().cpu().numpy()
            if mls == [0.0, 0.0]:
                np.testing.assert_array_equal(got[i], ref)
            else:
                assert rel(got[i], ref) < 1e-5


def test_two_step_calibration_matches_oracle(lib, small):
    """Sec. 4 calibration on the GPU: step 1 with mu_lambda = 0 (40 iterations), then the full
    method (mu_lambda = 3, same mu_s) started from step 1's X with fresh duals (30 iterations),
    against the oracle's two-step run with the same step sizes."""
    c, dirty, psf, p, tau2 = small
    p1 = om.Problem(dirty=dirty, psf=psf, J=3, mu_s=0.25, mu_l=0.0)
    tau1 = om.step_sizes(p1)[0]
    st1, st2 = om.two_step_calibration(p, 40, 30, tau1=tau1, tau2=tau2)
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=0.0, tau=tau1) as m1:
        m1.step(40)
        X1 = m1.get_x()
    with lib.Muffin(dirty, psf, J=3, mu_s=0.25, mu_lambda=3.0, tau=tau2) as m2:
        m2.set_x(X1)
        m2.step(30)
        X2 = m2.get_x().double().cpu().numpy()
        f2 = m2.objective()[0]
    assert rel(X1.double().cpu().numpy(), st1.X) < 1e-4
    assert rel(X2, st2.X) < 1e-4
    assert f2 == pytest.approx(om.objective(p, st2.X)[0], rel=1e-4)
