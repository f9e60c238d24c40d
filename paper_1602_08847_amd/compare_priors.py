"""The paper's comparison of the two spatial priors (Sec. 4, Fig. 3): the reconstruction SNR along the
iterations for the IUWT and for the union of the first eight Daubechies bases, both run through
the calibration protocol of Sec. 4 (mu_lambda = 0 for the first n1 iterations, then the full method
with mu_lambda > 0 from that X), on seeded synthetic cubes standing in for the paper's simulated
M31 cube (its data are not available).

python -m paper_1602_08847_amd.compare_priors --help
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import muffin, synth


def snr_curve(cube, J: int, prior: int, mu_s: float, mu_l: float, n1: int, n2: int, every: int,
              sigma: float = 1.0) -> dict:
    """SNR against the cube's sky every ``every`` iterations through both steps; device ms per
    iteration of each step."""
    import torch
    truth = cube.sky.astype(np.float32)
    out = {"prior": "uob" if prior == muffin.PRIOR_UOB else "iuwt", "snr": [], "mu_s": mu_s, "mu_lambda": mu_l}
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=mu_s, mu_lambda=0.0, sigma=sigma, prior=prior) as m:
        ms = 0.0
        for it in range(every, n1 + 1, every):
            ms += m.step_timed(every)
            out["snr"].append((it, m.snr(truth)))
        out["step1_ms_per_iter"] = ms / n1
        x1 = m.get_x()
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=mu_s, mu_lambda=mu_l, sigma=sigma, prior=prior) as m:
        m.set_x(x1)
        ms = 0.0
        for it in range(every, n2 + 1, every):
            ms += m.step_timed(every)
            out["snr"].append((n1 + it, m.snr(truth)))
        out["step2_ms_per_iter"] = ms / n2
        out["objective"] = float(m.objective()[0])
    torch.cuda.synchronize()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--L", type=int, default=15)
    ap.add_argument("--J", type=int, default=4)
    ap.add_argument("--sources", type=int, default=20)
    ap.add_argument("--baselines", type=int, default=2000)
    ap.add_argument("--seeds", default="0,1,2")
    ap.add_argument("--mu-s", type=float, default=0.25)
    ap.add_argument("--mu-lambda", type=float, default=3.0)
    ap.add_argument("--n1", type=int, default=2000)
    ap.add_argument("--n2", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    runs = []
    for seed in [int(v) for v in a.seeds.split(",")]:
        spec = synth.CubeSpec(N=a.N, L=a.L, J=a.J, n_sources=a.sources, n_baselines=a.baselines, seed=seed)
        cube = synth.make_cube(spec, dtype=np.float32)
        for prior in (muffin.PRIOR_IUWT, muffin.PRIOR_UOB):
            t0 = time.time()
            r = snr_curve(cube, a.J, prior, a.mu_s, a.mu_lambda, a.n1, a.n2, a.every, a.sigma)
            r["seed"] = seed
            log(f"[priors] seed {seed} {r['prior']}: SNR {r['snr'][a.n1 // a.every - 1][1]:.2f} dB after step 1, "
                f"{r['snr'][-1][1]:.2f} dB after step 2 ({time.time() - t0:.1f}s; "
                f"{r['step1_ms_per_iter']:.3f} / {r['step2_ms_per_iter']:.3f} ms per iteration)")
            runs.append(r)
    out = {"N": a.N, "L": a.L, "J": a.J, "n1": a.n1, "n2": a.n2, "sigma": a.sigma, "runs": runs}
    line = json.dumps(out)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
