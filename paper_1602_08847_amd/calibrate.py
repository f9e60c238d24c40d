"""The paper's two-step calibration of the regularisation weights (Sec. 4), on the library.

Step 1 sets mu_lambda = 0: the problem separates over the channels, each channel iterates on its
own (the library then skips the spectral step and runs the primal step in the gradient's last
pass), and several values of mu_s are cheap to try.  Here every value runs at once: the sweep is
one batch of copies of the cube, one copy per mu_s, and the batch API gives each copy its own group
and stream.  Step 2 keeps the chosen mu_s and runs the full method with mu_lambda > 0 from step 1's
X (U = V = 0).

The paper picks its weights by the reconstruction quality it reports (SNR against the sky truth,
Fig. 3) and suggests cross-validation.  The sweep scores each mu_s on what is held out of the
solver: with a truth, the SNR of Sec. 4 against it; without one, the discrepancy between the
data residual and the expected noise energy (Morozov's principle: ||H x - y||^2 against
N^2 L sigma_n^2), both reduced in FP64 on the GPU.

python -m paper_1602_08847_amd.calibrate --help
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import muffin, synth


def sweep_mu_s(cube, J: int, mus, iters: int, sigma: float = 1.0, truth=None, noise_sigma: float | None = None,
               log=None) -> list[dict]:
    """Step 1 for every mu_s in ``mus`` (mu_lambda = 0, ``iters`` iterations from zero), run together as
    one batch.  Returns per value: mu_s, tau, the data term (eq. (reg), FP64), the SNR against the
    truth if given, the relative discrepancy |2 data - N^2 L sigma_n^2| / (N^2 L sigma_n^2) if the noise
    level is given, and the final X (a device tensor)."""
    import torch
    mus = [float(m) for m in mus]
    copies = [(cube.dirty, cube.psf)] * len(mus)
    out = []
    with muffin.Batch(copies, J=J, mu_s=mus, mu_lambda=0.0, sigma=sigma) as b:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        L, N = b.shapes[0]
        for i, mu in enumerate(mus):
            f = b.objective(i)
            r = {"mu_s": mu, "tau": b.info(i)["tau"], "data_term": float(f[1]), "objective": float(f[0]),
                 "x": b.get_x(i)}
            if truth is not None:
                r["snr_db"] = b.snr(i, truth)
            if noise_sigma:
                e = N * N * L * noise_sigma ** 2
                r["discrepancy"] = abs(2.0 * f[1] - e) / e
            out.append(r)
    if log:
        log(f"[calibrate] step 1: {len(mus)} values of mu_s x {iters} iterations in {dt:.2f}s")
    for r in out:
        r["sweep_s"] = dt
    return out


def choose(results: list[dict]) -> dict:
    """The best mu_s: highest SNR when a truth was given, else the smallest discrepancy."""
    if all("snr_db" in r for r in results):
        return max(results, key=lambda r: r["snr_db"])
    return min(results, key=lambda r: r["discrepancy"])


def step_two(cube, J: int, mu_s: float, mu_lambda: float, x1, iters: int, sigma: float = 1.0, truth=None) -> dict:
    """Step 2: the full method with the chosen mu_s and mu_lambda from step 1's X, U = V = 0."""
    import torch
    with muffin.Muffin(cube.dirty, cube.psf, J=J, mu_s=mu_s, mu_lambda=mu_lambda, sigma=sigma) as m:
        m.set_x(x1)
        r = {"mu_s": mu_s, "mu_lambda": mu_lambda, "tau": m.info()["tau"]}
        if truth is not None:
            r["snr0_db"] = m.snr(truth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(iters)
        torch.cuda.synchronize()
        r["step2_s"] = time.perf_counter() - t0
        r["objective"] = float(m.objective()[0])
        if truth is not None:
            r["snr_db"] = m.snr(truth)
        r["x"] = m.get_x()
    return r


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--cube", default="cube256_L64_J4", help="workload name")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mus", default="0.01,0.05,0.1,0.25,0.5,1.0")
    ap.add_argument("--mu-lambda", type=float, default=3.0)
    ap.add_argument("--n1", type=int, default=2000, help="step 1 iterations (mu_lambda = 0)")
    ap.add_argument("--n2", type=int, default=2000, help="step 2 iterations")
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--criterion", choices=["snr", "discrepancy"], default="snr")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    spec = synth.CubeSpec(**{**synth.WORKLOADS[a.cube].__dict__, "seed": a.seed})
    cube = synth.make_cube(spec, dtype=np.float32)
    truth = cube.sky.astype(np.float32) if a.criterion == "snr" else None
    res = sweep_mu_s(cube, spec.J, [float(v) for v in a.mus.split(",")], a.n1, a.sigma, truth=truth,
                     noise_sigma=spec.noise_sigma, log=log)
    best = choose(res)
    log(f"[calibrate] chosen mu_s {best['mu_s']}")
    two = step_two(cube, spec.J, best["mu_s"], a.mu_lambda, best["x"], a.n2, a.sigma,
                   truth=cube.sky.astype(np.float32))
    out = {"cube": a.cube, "seed": a.seed, "n1": a.n1, "n2": a.n2, "sigma": a.sigma, "criterion": a.criterion,
           "sweep": [{k: v for k, v in r.items() if k != "x"} for r in res], "chosen_mu_s": best["mu_s"],
           "step2": {k: v for k, v in two.items() if k != "x"}}
    line = json.dumps(out)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
