"""Two passes of Algorithm 1 from (X0, U = 0, V = 0), evaluated only where a full-size cube
(1024 x 1024 x 256 voxels, J = 5) stays affordable in FP64 on the host.

Every per-channel operator of the iteration (the data gradient, the IUWT and its adjoint) acts on
one channel at a time, and the spectral operators act on one pixel spectrum at a time.  The first
pass therefore needs the data gradient of every channel (an FFT per channel, run on a thread pool)
but no wavelet transform beyond the sampled channels; the second pass needs the full spectral
dual V1 only through its adjoint, one cosine sum per sampled channel.  The steps are those of the
oracle's ``iterate`` in the same order, restricted to the sampled channels where the result allows
it (a CPU test pins this restriction to ``iterate`` itself on a small cube).

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
    """X1 and V1 in full; U1, X2 and U2 on the channels ``chans`` (all FP64).

    Pass 1 starts from U = V = 0, so its spatial and spectral adjoint terms vanish and
    X~1 = (X0 - tau grad(X0))_+.  The dual steps take D1 = 2 X~1 - X0 (Algorithm 1).
    Pass 2 at channel c: X~2 = (X1 - tau (grad_c(X1) + mu_s W_s^T(omega U1_c) + mu_l (V1 W_lambda^T)_c))_+,
    D2 = 2 X~2 - X1, U~2 = sat(U1_c + sigma mu_s omega W_s D2); then relaxation by rho.
    """
    om_w = om.plane_weights(J, omega)[:, None, None]
    r = rho
    X0 = om.positive(np.asarray(X0, dtype=np.float64))  # the oracle's initial state clips X0
    g0 = data_gradient_threaded(psf, X0, dirty, workers)
    Xt1 = om.positive(X0 - tau * g0)
    del g0
    D1 = 2.0 * Xt1 - X0
    V1 = r * om.sat(sigma * mu_l * om.spectral(D1))  # V0 = 0
    X1 = r * Xt1 + (1.0 - r) * X0
    del Xt1
    T1 = om.spectral_adjoint(V1)[chans]
    out = {"X1": X1, "V1": V1, "U1": [], "X2": [], "U2": []}
    for i, c in enumerate(chans):
        U1c = r * om.sat(sigma * mu_s * om_w * om.iuwt(D1[c], J, gen))  # U0 = 0
        grad = om.data_gradient(psf[c:c + 1], X1[c:c + 1], dirty[c:c + 1])[0]
        s = mu_s * om.iuwt_adjoint(om_w * U1c, J, gen)
        Xt2 = om.positive(X1[c] - tau * (grad + s + mu_l * T1[i]))
        D2 = 2.0 * Xt2 - X1[c]
        Ut2 = om.sat(U1c + sigma * mu_s * om_w * om.iuwt(D2, J, gen))
        out["U1"].append(U1c)
        out["X2"].append(r * Xt2 + (1.0 - r) * X1[c])
        out["U2"].append(r * Ut2 + (1.0 - r) * U1c)
    for k in ("U1", "X2", "U2"):
        out[k] = np.stack(out[k])
    return out
