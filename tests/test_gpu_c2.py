"""The 256 x 256 x 64, J = 4 parity cube (20 sources, 2000 baselines, seed 0): 200 iterations of the
HIP path against the FP64 oracle's objective trajectory, stored by tests/golden/make_c2_golden.py
(a script that calls only the oracle): the objective every 20 iterations and the final one within
1e-4, and the norms of the final X, U and V."""
import json
import os

import numpy as np
import pytest

from paper_1602_08847_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_objective.json")


def test_c2_two_hundred_iterations_match_oracle_objective(lib):
    g = json.load(open(GOLDEN))
    spec = synth.WORKLOADS["cube256_L64_J4"]
    c = synth.make_cube(spec)
    with lib.Muffin(c.dirty.astype(np.float32), c.psf.astype(np.float32), J=4, mu_s=0.25, mu_lambda=3.0,
                    tau=g["tau"]) as m:
        done = 0
        for it, f_ref in g["objective_every_20"]:
            m.step(it - done)
            done = it
            f = m.objective()
            print(f"[c2] iteration {it}: f {f[0]:.10e} oracle {f_ref:.10e} rel {abs(f[0] - f_ref) / f_ref:.2e}",
                  flush=True)
            assert abs(f[0] - f_ref) / abs(f_ref) < 1e-4, it
        np.testing.assert_allclose(f, g["objective_terms_200"], rtol=1e-4)
        for key, t in (("norm_X", m.get_x()), ("norm_U", m.get_u()), ("norm_V", m.get_v())):
            assert float(np.linalg.norm(t.double().cpu().numpy())) == pytest.approx(g[key], rel=1e-4), key
