"""Writes tests/golden/c2_objective.json: the FP64 oracle's trajectory on the 256 x 256 x 64, J = 4
parity cube (20 sources, 2000 baselines, seed 0; inputs rounded to FP32 as the GPU receives them),
200 iterations of the MUFFIN iteration (Algorithm 1) from X = U = V = 0 with mu_s = 0.25,
mu_lambda = 3 (Sec. 4), sigma = rho = 1, tau by the convergence condition; the objective of
eq. (reg) + eq. (RegAll) every 20 iterations, and norms of the final X, U, V.

Calls only the oracle (and the seeded input generator).  Run from the repository root:
    python tests/golden/make_c2_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import muffin as om  # noqa: E402
from paper_1602_08847_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_objective.json")


def main():
    spec = synth.WORKLOADS["cube256_L64_J4"]
    c = synth.make_cube(spec)
    dirty = c.dirty.astype(np.float32).astype(np.float64)
    psf = c.psf.astype(np.float32).astype(np.float64)
    p = om.Problem(dirty=dirty, psf=psf, J=spec.J, mu_s=0.25, mu_l=3.0)
    tau = om.step_sizes(p)[0]
    t0 = time.time()
    st = om.init_state(p)
    f = []
    for it in range(1, 201):
        st = om.iterate(p, st, tau)
        if it % 20 == 0:
            f.append([it, float(om.objective(p, st.X)[0])])
            print(f"iteration {it}: f = {f[-1][1]:.12e} ({time.time() - t0:.0f}s)", flush=True)
    out = {
        "what": "FP64 oracle, 256x256x64 J=4 cube (seed 0, inputs rounded to FP32), mu_s=0.25, mu_lambda=3, "
                "sigma=rho=1, 200 iterations from zero",
        "tau": tau,
        "objective_every_20": f,
        "objective_terms_200": [float(v) for v in om.objective(p, st.X)],
        "norm_X": float(np.linalg.norm(st.X)),
        "norm_U": float(np.linalg.norm(st.U)),
        "norm_V": float(np.linalg.norm(st.V)),
        "script": "tests/golden/make_c2_golden.py",
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
