"""Workloads run against the bounds-checked build of the library (test infrastructure).

Run as a child process by tests/test_gpu_checked.py with MUFFIN_LIBRARY set to
paper_1602_08847_amd/libmuffin_checked.so.  It drives every instrumented kernel family (the IUWT
band, pair, triple and fused-tail kernels of both generations, also with class groups forced, the
FFT passes, the spectral step in its planned, Bluestein and cosine-table forms, the union-of-bases
kernels in both workgroup layouts, the visibility data term's kernels, an uneven batch) over ragged
and wrapping shapes, then prints one JSON line with the number of out-of-bounds indices the device
caught.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_1602_08847_amd import muffin, synth  # noqa: E402


def cube(N, L, J, seed=0):
    c = synth.make_cube(synth.CubeSpec(N=N, L=L, J=J, n_sources=max(2, N // 16), n_baselines=max(8, 2 * N),
                                       seed=seed), dtype=np.float32)
    return c.dirty, c.psf


def run(N, L, J, steps=3, **kw):
    dirty, psf = cube(N, L, J, seed=N + L)
    with muffin.Muffin(dirty, psf, J=J, mu_s=0.25, mu_lambda=3.0, **kw) as m:
        m.set_x(np.abs(np.random.default_rng(N).normal(size=dirty.shape)).astype(np.float32))
        m.step(steps)
        m.objective()
        if kw.get("prior") == muffin.PRIOR_UOB:
            x = np.random.default_rng(1).normal(size=(L, N, N)).astype(np.float32)
            m.apply_op(muffin.OP_IUWT, x)
            m.apply_op(muffin.OP_IUWT_ADJ, np.random.default_rng(2).normal(size=(L, 8, N, N)).astype(np.float32))
            m.apply_op(muffin.OP_IUWT_SCHED, 0.05 * x)
        else:
            x = np.random.default_rng(1).normal(size=(L, N, N)).astype(np.float32)
            for op in (muffin.OP_H, muffin.OP_HT, muffin.OP_GRAD):
                m.apply_op(op, x)


def main():
    assert muffin.debug_oob() == 0  # raises on a library built without the checks
    cases = []
    # IUWT, both generations, the launch forms: fused tail on and off, one scale per launch
    for N, L, J, gen, flags in [(64, 8, 3, 2, 0), (64, 8, 3, 1, 0), (8, 3, 1, 1, 0), (12, 5, 2, 2, 0),
                                (96, 7, 3, 2, 0), (128, 17, 4, 2, 4), (128, 17, 4, 2, 2), (256, 64, 4, 2, 4),
                                (256, 64, 4, 1, 0), (64, 5, 5, 2, 1), (384, 3, 4, 2, 0), (48, 48, 3, 2, 0)]:
        run(N, L, J, iuwt_gen=gen, flags=flags)
        cases.append(f"iuwt N={N} L={L} J={J} gen={gen} flags={flags}")
    # class groups forced on every IUWT family, with bands no taller than the coarsest residue step
    fams = {2: (0, 1, 5, 6, 7, 8, 9), 1: (2, 3, 10, 11)}
    for N, L, J, gen, flags in [(64, 4, 5, 2, 4), (64, 4, 5, 2, 2), (64, 4, 5, 2, 1), (64, 4, 5, 1, 0)]:
        try:
            for j in range(J):
                for f in fams[gen]:
                    muffin.set_band_tiles(N, j, f, 16, min(8, 1 << j))
            run(N, L, J, iuwt_gen=gen, flags=flags)
        finally:
            for j in range(J):
                for f in fams[gen]:
                    muffin.set_band_tiles(N, j, f, 0, 0)
        cases.append(f"iuwt class groups N={N} L={L} J={J} gen={gen} flags={flags}")
    # the spectral step: Bluestein (64), cosine tables (32), default choice; planned radix-3 sizes
    for L, flags in [(17, 64), (37, 64), (70, 64), (100, 64), (150, 64), (300, 64), (100, 32), (260, 32),
                     (120, 0), (96, 0), (192, 0)]:
        run(16, L, 2, steps=2, flags=flags)
        cases.append(f"spectral L={L} flags={flags}")
    # union of bases, both workgroup layouts, small levels and the all-bases layout
    for N, L, J, flags in [(64, 8, 3, 0), (32, 3, 5, 0), (96, 5, 3, 8), (128, 17, 4, 8), (16, 2, 4, 0),
                           (256, 4, 5, 8), (256, 4, 5, 16)]:
        run(N, L, J, prior=muffin.PRIOR_UOB, flags=flags)
        cases.append(f"uob N={N} L={L} J={J} flags={flags}")
    # the visibility data term: ragged visibility counts, one visibility, image sides 3 * 2^a
    for N, L, K in [(16, 3, 50), (24, 2, 65), (64, 2, 1), (48, 3, 130), (8, 2, 200)]:
        rng = np.random.default_rng(N + K)
        uvw = np.column_stack([rng.uniform(-2 * N, 2 * N, K), rng.uniform(-2 * N, 2 * N, K), rng.uniform(-N, N, K)])
        lam = np.linspace(1.0, 0.7, L)
        vis = (rng.normal(size=(L, K)) + 1j * rng.normal(size=(L, K))).astype(np.complex64)
        with muffin.Muffin.from_visibilities(vis, uvw, lam, 1.0 / (12 * N), N=N, J=2, mu_s=0.5, mu_lambda=1.0,
                                             power_iters=3) as m:
            m.set_x(np.abs(rng.normal(size=(L, N, N))).astype(np.float32))
            m.step(2)
            m.objective()
            x = rng.normal(size=(L, N, N)).astype(np.float32)
            m.apply_op(muffin.OP_PHI, x)
            m.apply_op(muffin.OP_PHI_ADJ, rng.normal(size=(L, K, 2)).astype(np.float32))
            m.apply_op(muffin.OP_GRAD, x)
            m.vis_residual()
        cases.append(f"vis N={N} L={L} K={K}")
    # an uneven batch (groups by image side)
    specs = [(64, 9), (128, 20), (64, 33), (96, 7)]
    data = [cube(N, L, 3, seed=i) for i, (N, L) in enumerate(specs)]
    with muffin.Batch(data, J=3, mu_s=0.25, mu_lambda=3.0) as b:
        b.step(3)
    cases.append("batch")
    print(json.dumps({"cases": len(cases), "oob": muffin.debug_oob()}), flush=True)


if __name__ == "__main__":
    main()
