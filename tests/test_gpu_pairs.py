"""Two or three IUWT scales per launch, and the last analysis pair fused with the next iteration's
first adjoint pair, against one scale per launch: the fused kernels perform the same operations in
the same order, so the iterates agree bit for bit, for every J (schedules of singles, pairs and
triples, each with or without the coarse plane), for both generations of the transform, with and
without the coarse plane's penalty, with relaxation, and for image sides where the coarse taps
wrap around the image several times."""
import numpy as np
import pytest

from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu

CASES = [
    # N, L, J, penalize_coarse, rho
    (64, 8, 1, True, 1.0),
    (64, 8, 2, True, 1.0),
    (64, 8, 3, True, 1.0),
    (64, 8, 4, False, 0.8),
    (96, 5, 5, True, 0.9),
    (128, 4, 6, True, 1.0),
    (16, 3, 4, True, 1.0),
    (8, 2, 3, False, 1.0),
    (12, 3, 5, True, 1.0),
    (256, 3, 5, True, 1.0),
    # N = 8: the fused pair's taps (scales 2, 3 at J = 4; 3, 4 at J = 5) span or exceed the side
    (8, 2, 4, True, 1.0),
    (8, 2, 5, True, 0.9),
]


@pytest.mark.parametrize("N,L,J,pc,rho", CASES)
def test_pairs_match_single_scale_bitwise(lib, N, L, J, pc, rho):
    c = synth.make_cube(synth.CubeSpec(N=N, L=L, J=J, n_sources=max(2, N // 16), n_baselines=max(8, N * 2),
                                       seed=N + J))
    out = {}
    for flags in (lib.FLAG_FUSED_TAIL, lib.FLAG_NO_FUSED_TAIL, lib.FLAG_SINGLE_SCALE):
        with lib.Muffin(c.dirty, c.psf, J=J, mu_s=0.25, mu_lambda=3.0, penalize_coarse=pc, sigma=10.0, rho=rho,
                        flags=flags) as m:
            m.step(7)  # odd: the fused tail's planes end in its second buffer
            out[flags] = (m.get_x().cpu().numpy(), m.get_u().cpu().numpy(), m.get_v().cpu().numpy())
    for flags in (lib.FLAG_FUSED_TAIL, lib.FLAG_NO_FUSED_TAIL):
        for a, b in zip(out[flags], out[lib.FLAG_SINGLE_SCALE]):
            np.testing.assert_array_equal(a, b)


# first generation: pairs only ({1, 2}, {2, 2}, {1, 2, 2}, {2, 2, 2} scales per launch)
G1_CASES = [
    # N, L, J, penalize_coarse, rho
    (64, 8, 2, True, 1.0),
    (64, 8, 3, True, 1.0),
    (64, 8, 4, False, 0.8),
    (96, 5, 5, True, 0.9),
    (128, 4, 6, True, 1.0),
    (16, 3, 4, True, 1.0),
    (8, 2, 3, False, 1.0),
    (12, 3, 5, True, 1.0),
    (8, 2, 5, True, 0.9),
]


@pytest.mark.parametrize("N,L,J,pc,rho", G1_CASES)
def test_first_generation_pairs_match_single_scale_bitwise(lib, N, L, J, pc, rho):
    c = synth.make_cube(synth.CubeSpec(N=N, L=L, J=J, n_sources=max(2, N // 16), n_baselines=max(8, N * 2),
                                       seed=N + J + 100))
    out = {}
    for flags in (0, lib.FLAG_SINGLE_SCALE):
        with lib.Muffin(c.dirty, c.psf, J=J, mu_s=0.25, mu_lambda=3.0, iuwt_gen=1, penalize_coarse=pc, sigma=10.0,
                        rho=rho, flags=flags) as m:
            m.step(7)
            out[flags] = (m.get_x().cpu().numpy(), m.get_u().cpu().numpy(), m.get_v().cpu().numpy())
    for a, b in zip(out[0], out[lib.FLAG_SINGLE_SCALE]):
        np.testing.assert_array_equal(a, b)


# Class groups: a launch may split a band's residue classes mod 2^j over several workgroups. Each
# class still runs through the same steps, so the iterates agree bit for bit with one workgroup per
# band, for every kernel family (one scale, pairs, triples, the fused tail), both generations, whole-
# channel and short bands, with and without relaxation.
FAMILIES = {2: (0, 1, 5, 6, 7, 8, 9), 1: (2, 3, 10, 11)}


def _set_tiles(lib, N, J, gen, rows, groups):
    for j in range(J):
        for f in FAMILIES[gen]:
            lib.set_band_tiles(N, j, f, rows, min(groups, 1 << j, 8) if groups else 0)


@pytest.mark.parametrize("N,L,J,gen,pc,rho,rows,groups", [
    (64, 6, 4, 2, True, 1.0, 16, 4), (64, 6, 4, 2, False, 0.8, 64, 2), (64, 6, 4, 1, True, 1.0, 32, 4),
    (96, 4, 5, 2, True, 0.9, 96, 8), (96, 4, 5, 1, True, 1.0, 32, 8), (128, 3, 5, 2, True, 1.0, 128, 8),
    (128, 3, 6, 2, True, 1.0, 64, 8), (64, 4, 3, 2, True, 1.0, 64, 4), (64, 4, 2, 2, True, 1.0, 32, 2),
    (16, 3, 4, 2, True, 1.0, 16, 4), (8, 2, 5, 1, True, 1.0, 8, 8), (8, 2, 5, 2, True, 0.9, 8, 8)])
def test_class_groups_match_one_workgroup_per_band_bitwise(lib, N, L, J, gen, pc, rho, rows, groups):
    c = synth.make_cube(synth.CubeSpec(N=N, L=L, J=J, n_sources=max(2, N // 16), n_baselines=max(8, N * 2),
                                       seed=N + J + 200))
    kw = dict(J=J, mu_s=0.25, mu_lambda=3.0, iuwt_gen=gen, penalize_coarse=pc, sigma=10.0, rho=rho)
    flag_sets = (lib.FLAG_FUSED_TAIL, lib.FLAG_NO_FUSED_TAIL, lib.FLAG_SINGLE_SCALE) if gen == 2 else \
        (0, lib.FLAG_SINGLE_SCALE)

    def run(flags):
        with lib.Muffin(c.dirty, c.psf, flags=flags, **kw) as m:
            m.step(7)  # odd: the fused tail's planes end in its second buffer
            return m.get_x().cpu().numpy(), m.get_u().cpu().numpy(), m.get_v().cpu().numpy()

    try:
        _set_tiles(lib, N, J, gen, rows, 1)
        ref = run(lib.FLAG_SINGLE_SCALE)
        _set_tiles(lib, N, J, gen, rows, groups)
        got = {f: run(f) for f in flag_sets}
    finally:
        _set_tiles(lib, N, J, gen, 0, 0)
    for f in flag_sets:
        for a, b in zip(got[f], ref):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("flags,gen", [(0, 2), (2, 2), (4, 2), (0, 1)])
def test_pairs_autotuned_match_single_scale(lib, flags, gen):
    c = synth.make_cube(synth.CubeSpec(N=128, L=6, J=5, n_sources=6, n_baselines=300, seed=9))
    kw = dict(J=5, mu_s=0.25, mu_lambda=3.0, sigma=10.0, iuwt_gen=gen)
    with lib.Muffin(c.dirty, c.psf, flags=flags, **kw) as a, \
            lib.Muffin(c.dirty, c.psf, flags=lib.FLAG_SINGLE_SCALE, **kw) as b:
        a.autotune(reps=1)
        a.step(5)
        b.step(5)
        np.testing.assert_array_equal(a.get_u().cpu().numpy(), b.get_u().cpu().numpy())


# launch kinds: 0 one analysis scale, 1 one adjoint step, 2 last analysis scale with the coarse plane,
# 3/4/5 the same for pairs, 6/7/8 for triples, 9 the last analysis pair fused with the next
# iteration's first adjoint pair (coarse plane penalised, last group a pair; flag 4 forces it, flag 2
# turns it off, and by default a cube of 4 channels is too small for it)
@pytest.mark.parametrize("J,pc,flags,counts", [
    (5, True, 2, {6: 1, 5: 1, 4: 1, 7: 1}), (4, True, 2, {3: 1, 4: 2, 5: 1}), (2, True, 2, {5: 1, 4: 1}),
    (5, True, 0, {6: 1, 5: 1, 4: 1, 7: 1}),
    (3, True, 0, {8: 1, 7: 1}), (6, True, 0, {6: 1, 8: 1, 7: 2}), (1, True, 0, {2: 1, 1: 1}),
    (5, True, 4, {6: 1, 9: 1, 7: 1}), (4, True, 4, {3: 1, 9: 1, 4: 1}), (2, True, 4, {9: 1}),
    (5, False, 4, {6: 1, 3: 1, 4: 1, 7: 1}), (3, True, 4, {8: 1, 7: 1})])
def test_profile_reports_the_launch_schedule(lib, J, pc, flags, counts):
    c = synth.make_cube(synth.CubeSpec(N=128, L=4, J=J, n_sources=3, n_baselines=100, seed=2))
    with lib.Muffin(c.dirty, c.psf, J=J, mu_s=0.25, mu_lambda=3.0, penalize_coarse=pc, flags=flags) as m:
        ms = m.profile(4)
    assert len(ms) == 32 and np.all(ms[5:8] == 0)
    for k in range(12):
        assert ms[9 + 2 * k] == counts.get(k, 0), (k, ms)
        assert (ms[8 + 2 * k] > 0) == (k in counts)
    assert ms[0] == pytest.approx(sum(ms[1:5]), rel=1e-6)
