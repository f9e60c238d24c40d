"""Uneven batches and the band-height autotuner: both must leave the arithmetic unchanged, so a
batch reproduces separate contexts bit for bit and a tuned context reproduces an untuned one."""
import json

import numpy as np
import pytest

from oracle import muffin as om
from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu

SPECS = [synth.CubeSpec(N=64, L=8, J=3, n_sources=4, n_baselines=100, seed=1),
         synth.CubeSpec(N=96, L=5, J=3, n_sources=4, n_baselines=150, seed=2),
         synth.CubeSpec(N=64, L=3, J=3, n_sources=3, n_baselines=80, seed=3),
         synth.CubeSpec(N=128, L=17, J=3, n_sources=6, n_baselines=300, seed=4)]


@pytest.fixture(scope="module")
def cubes():
    return [synth.make_cube(s, dtype=np.float32) for s in SPECS]


@pytest.mark.parametrize("gen", [2, 1])
def test_batch_matches_separate_contexts_bitwise(lib, cubes, gen):
    mls = [3.0, 2.0, 3.0, 1.5]
    with lib.Batch([(c.dirty, c.psf) for c in cubes], J=3, mu_s=0.25, mu_lambda=mls, sigma=10.0, iuwt_gen=gen) as b:
        b.step(12)
        for i, c in enumerate(cubes):
            with lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=mls[i], sigma=10.0, iuwt_gen=gen) as m:
                assert b.info(i)["tau"] == m.info()["tau"]
                m.step(12)
                np.testing.assert_array_equal(b.get_x(i).cpu().numpy(), m.get_x().cpu().numpy())
                np.testing.assert_allclose(b.objective(i), m.objective(), rtol=1e-12)


@pytest.mark.parametrize("gen", [2, 1])
def test_batch_step_matches_oracle_per_cube(lib, cubes, gen):
    with lib.Batch([(c.dirty, c.psf) for c in cubes[:2]], J=3, mu_s=0.25, mu_lambda=3.0, iuwt_gen=gen) as b:
        b.step(5)
        for i, c in enumerate(cubes[:2]):
            p = om.Problem(dirty=c.dirty.astype(np.float64), psf=c.psf.astype(np.float64), J=3, mu_s=0.25,
                           mu_l=3.0, gen=gen)
            st, _ = om.solve(p, 5, tau=b.info(i)["tau"])
            x = b.get_x(i).double().cpu().numpy()
            assert np.linalg.norm(x - st.X) / np.linalg.norm(st.X) < 1e-4


def test_autotune_keeps_results_and_reports_choices(lib, cubes):
    c = cubes[3]
    with lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=3.0) as a:
        a.step(6)
        xa = a.get_x().cpu().numpy()
    with lib.Muffin(c.dirty, c.psf, J=3, mu_s=0.25, mu_lambda=3.0) as t:
        rep = json.loads(t.autotune(reps=2))
        # J = 3: the three analysis scales in one launch, the three adjoint steps in another
        assert rep["N"] == 128 and len(rep["scales"]) == 2
        assert [(s["j"], s["kernel"]) for s in rep["scales"]] == [(0, "analysis triple"), (0, "adjoint triple")]
        for s in rep["scales"]:
            assert 128 % s["rows"] == 0 and f'{s["rows"]}x{s["class_groups"]}' in s["candidates_ms"]
            # the triples start at scale 0: one residue class, so one group
            assert s["class_groups"] == 1 and s["family"] in (lib.FAMILY_TRIPLE_ANALYSIS, lib.FAMILY_TRIPLE_ADJOINT)
        t.step(6)
        np.testing.assert_array_equal(t.get_x().cpu().numpy(), xa)


@pytest.mark.parametrize("shape,flags", [("small", 0), ("small", 4), ("wide", 0)])
def test_autotune_chooses_the_fused_tail(lib, cubes, shape, flags):
    """The autotuner times the fused tail against the two launches it replaces and keeps the faster
    one (flag 4 keeps it fused); the iterates do not change either way.  The small cube starts
    without it (too few channels); the wide one (256 channels of 256^2, J = 4) starts with it, its
    planes in the second buffer when the autotuner may switch it off."""
    if shape == "small":
        c, J = cubes[3], 5
    else:
        c, J = synth.make_cube(synth.CubeSpec(N=256, L=256, J=4, n_sources=8, n_baselines=400, seed=5)), 4
    kw = dict(J=J, mu_s=0.25, mu_lambda=3.0)
    with lib.Muffin(c.dirty, c.psf, flags=2, **kw) as a:
        a.step(5)
        xa, ua = a.get_x().cpu().numpy(), a.get_u().cpu().numpy()
    with lib.Muffin(c.dirty, c.psf, flags=flags, **kw) as t:
        t.step(3)  # odd: a fused tail's planes sit in its second buffer when the choice is made
        rep = json.loads(t.autotune(reps=1))
        kernels = [s["kernel"] for s in rep["scales"]]
        assert "analysis pair + next adjoint pair" in kernels and "adjoint pair" in kernels
        for s in rep["scales"]:
            # every band height with 1, 2, 4 or 8 class groups (up to 2^j)
            g = s["class_groups"]
            assert f'{s["rows"]}x{g}' in s["candidates_ms"] and 1 <= g <= min(8, 1 << s["j"])
        assert isinstance(rep["fused_tail"], bool)
        assert rep["fused_tail"] == (flags == 4 or rep["fused_ms"] < rep["separate_ms"])
        t.step(2)
        np.testing.assert_array_equal(t.get_x().cpu().numpy(), xa)
        np.testing.assert_array_equal(t.get_u().cpu().numpy(), ua)
