"""Two steps of the MUFFIN iteration from (X0, U = 0, V = 0), evaluated only where a full-size cube
(1024 x 1024 x 256 voxels, J = 5) stays affordable in FP64 on the host.

Both steps are the oracle's generic ``primal_dual_step`` applied to a restriction of the problem
that leaves the sampled results unchanged:

* the proximal maps (positive part, l-infinity projection) and the relaxation act entry by entry,
  so a dual variable may be restricted to any subset of its entries;
* the spatial half of the analysis operator acts on one channel at a time, the spectral half on
  one pixel spectrum at a time.

Step 1 therefore runs on the whole X with the dual restricted to (U on the sampled channels, all
of V); since U = V = 0 its adjoint term vanishes, so no wavelet transform beyond the sampled
channels is needed, only the data gradient of every channel (an FFT per channel, on a thread
pool).  Step 2 runs channel by channel on the sampled channels with the dual U_c; the spectral
dual V1 enters that channel's primal step only through the fixed term mu_lambda (V1 W_lambda^T)_c,
which is added to the gradient.  A CPU test pins this restriction to the oracle's whole-cube
``iterate`` on a small cube.

Test infrastructure only: it calls the oracle and nothing else.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import muffin as om


def data_gradient_threaded(psf, x, y, workers: int = 8, chunk: int = 4) -> np.ndarray:
    """The oracle's data gradient, channel block by channel block on a thread pool (the FFTs
    release the interpreter lock); each channel's gradient is the same computation as in one call."""
    L = x.shape[0]
    out = np.empty(x.shape, dtype=np.float64)

    def one(l0):
        l1 = min(L, l0 + chunk)
        out[l0:l1] = om.data_gradient(psf[l0:l1], x[l0:l1], y[l0:l1])

    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(one, range(0, L, chunk)))
    return out


def two_passes_sampled(dirty, psf, X0, J, mu_s, mu_l, tau, chans, sigma=1.0, rho=1.0, omega=None, gen=2,
                       workers: int = 8) -> dict:
    """X1 and V1 in full; U1, X2 and U2 on the channels ``chans`` (all FP64)."""
    K = om.AnalysisOperator(J=J, gen=gen, mu_s=mu_s, mu_l=mu_l, omega=om.plane_weights(J, omega))
    chans = list(chans)
    X0 = om.positive(np.asarray(X0, dtype=np.float64))  # the oracle's initial state clips X0
    L, N = X0.shape[0], X0.shape[1]

    # step 1: dual (U on the sampled channels, V) = 0
    def K1(X):
        return np.stack([K.spatial(X[c]) for c in chans]), mu_l * om.spectral(X)

    def K1_adj(Uc, V):
        assert not np.any(Uc) and not np.any(V)  # the restricted adjoint is exact only at 0
        return 0.0

    duals0 = (np.zeros((len(chans), J + 1, N, N)), np.zeros((L, N, N)))
    X1, (U1, V1) = om.primal_dual_step(X0, duals0, lambda x: data_gradient_threaded(psf, x, dirty, workers),
                                       K1, K1_adj, om.positive, om.l1_conj_prox, tau, sigma, rho)

    # step 2, one sampled channel at a time
    W = om.dct_matrix(L)
    out = {"X1": X1, "V1": V1, "U1": U1, "X2": [], "U2": []}
    for i, c in enumerate(chans):
        spec_c = mu_l * (W[c] @ V1.reshape(L, -1)).reshape(N, N)  # mu_lambda (V1 W_lambda^T)_c

        def grad_c(x, c=c, spec_c=spec_c):
            return om.data_gradient(psf[c:c + 1], x[None], dirty[c:c + 1])[0] + spec_c

        x2, (u2,) = om.primal_dual_step(X1[c], (U1[i],), grad_c, lambda x: (K.spatial(x),), K.spatial_adjoint,
                                        om.positive, om.l1_conj_prox, tau, sigma, rho)
        out["X2"].append(x2)
        out["U2"].append(u2)
    for k in ("X2", "U2"):
        out[k] = np.stack(out[k])
    return out
