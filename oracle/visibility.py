"""FP64 oracle of the visibility-domain data term (test infrastructure only).

Sec. 2, eq. (viseq), relates the sky image of one wavelength to the complex visibility of a
baseline (u, v, w) (metres, w along the line of sight): the integral over the direction cosines
(l, m) of x / n times exp(-2 pi i (u l + v m + w n) / lambda), with n = sqrt(1 - l^2 - m^2). The
w n term is the direction-dependent effect the image-plane model of eq. (model) leaves out. The
paper then writes all visibilities of a wavelength as v = Phi x + noise.

Discretisation read here (the paper fixes none of it):

* pixel (i, j) (row i, column j) of an N x N image sits at l = (j - N/2) cell, m = (i - N/2) cell,
  so that the phase centre is pixel (N/2, N/2), the origin of the PSF convention of the
  image-plane model; every pixel must satisfy l^2 + m^2 < 1;
* the integral becomes the sum over pixels, x being the flux of each pixel;
* the phase keeps the paper's w n (not the w (n - 1) of phase-tracked data; the two differ by a
  factor exp(-2 pi i w / lambda) per visibility, which cancels in the data term when the data
  were simulated with the same operator);
* channel l observes every baseline at its own wavelength lambda_l, so one set of K baselines
  gives K visibilities per channel;
* the data term is sum_l w_l/2 ||v_l - Phi_l x_l||^2 (eq. (reg) with Phi_l in place of H_l and
  its channel weights w_l = 1/sigma_l^2, 1 by default); x is real, so its gradient is
  w_l Re Phi_l^H (Phi_l x_l - v_l);
* beta, the Lipschitz constant of that gradient, is the largest eigenvalue of w_l Re Phi_l^H Phi_l
  over all channels. It has no closed form here: it is estimated by power iteration in FP64 from the
  all-ones cube (``power_iters`` steps), and the step sizes use ``BETA_MARGIN`` times the estimate.

Everything is plain numpy on dense phase matrices: sizes are kept small.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BETA_MARGIN = 1.01
POWER_ITERS = 40


@dataclass
class VisData:
    uvw: np.ndarray  # (K, 3) baselines in metres
    lam: np.ndarray  # (L,) wavelength of each channel, metres
    cell: float  # pixel size in direction-cosine units
    vis: np.ndarray  # (L, K) complex visibilities
    N: int  # image side
    w: np.ndarray | None = None  # (L,) channel weights 1/sigma_l^2, or None for 1


def direction_cosines(N: int, cell: float):
    """(l of each column, m of each row, n of each pixel) for an N x N image."""
    c = (np.arange(N) - N // 2) * float(cell)
    l = c[None, :]
    m = c[:, None]
    r2 = l * l + m * m
    if np.any(r2 >= 1.0):
        raise ValueError("every pixel needs l^2 + m^2 < 1")
    return c, c, np.sqrt(1.0 - r2)


def phase_matrix(N: int, cell: float, uvw: np.ndarray, lam: float) -> np.ndarray:
    """(K, N*N) matrix of Phi at one wavelength: exp(-2 pi i (u l + v m + w n) / lambda) / n."""
    lc, mc, n = direction_cosines(N, cell)
    l = np.broadcast_to(lc[None, :], (N, N)).ravel()
    m = np.broadcast_to(mc[:, None], (N, N)).ravel()
    nn = n.ravel()
    u, v, w = (np.asarray(uvw, dtype=np.float64)[:, k, None] / lam for k in range(3))
    return np.exp(-2j * np.pi * (u * l[None, :] + v * m[None, :] + w * nn[None, :])) / nn[None, :]


def phi(x: np.ndarray, uvw: np.ndarray, lam: np.ndarray, cell: float) -> np.ndarray:
    """Phi_l x_l for every channel: (L, N, N) real -> (L, K) complex (eq. (viseq), discretised)."""
    L, N = x.shape[0], x.shape[1]
    return np.stack([phase_matrix(N, cell, uvw, lam[l]) @ x[l].ravel() for l in range(L)])


def phi_adjoint(r: np.ndarray, uvw: np.ndarray, lam: np.ndarray, cell: float, N: int) -> np.ndarray:
    """Re Phi_l^H r_l for every channel: (L, K) complex -> (L, N, N) real."""
    L = r.shape[0]
    return np.stack([np.real(phase_matrix(N, cell, uvw, lam[l]).conj().T @ r[l]).reshape(N, N)
                     for l in range(L)])


def _weights(L: int, w) -> np.ndarray:
    return np.ones(L) if w is None else np.asarray(w, dtype=np.float64)


def vis_gradient(x: np.ndarray, d: VisData) -> np.ndarray:
    """Gradient of sum_l w_l/2 ||v_l - Phi_l x_l||^2 at the real cube x."""
    wl = _weights(x.shape[0], d.w)
    r = wl[:, None] * (phi(x, d.uvw, d.lam, d.cell) - d.vis)
    return phi_adjoint(r, d.uvw, d.lam, d.cell, d.N)


def vis_data_term(x: np.ndarray, d: VisData) -> float:
    """sum_l w_l/2 ||v_l - Phi_l x_l||^2."""
    wl = _weights(x.shape[0], d.w)
    r = phi(x, d.uvw, d.lam, d.cell) - d.vis
    return float(0.5 * np.sum(wl * np.sum(np.abs(r) ** 2, axis=1)))


def power_estimate(uvw: np.ndarray, lam: np.ndarray, cell: float, N: int, iters: int = POWER_ITERS,
                   w=None) -> float:
    """Largest eigenvalue of w_l Re Phi_l^H Phi_l over all channels, by power iteration from the
    all-ones cube: x <- A x / ||A x||; the estimate is ||A x|| of the last step."""
    L = len(lam)
    wl = _weights(L, w)
    x = np.ones((L, N, N))
    x /= np.linalg.norm(x)
    est = 0.0
    for _ in range(iters):
        y = phi_adjoint(wl[:, None] * phi(x, uvw, lam, cell), uvw, lam, cell, N)
        est = float(np.linalg.norm(y))
        x = y / est
    return est


def vis_lipschitz(d: VisData, iters: int = POWER_ITERS) -> float:
    """beta of the visibility data term: BETA_MARGIN times the power-iteration estimate."""
    return BETA_MARGIN * power_estimate(d.uvw, d.lam, d.cell, d.N, iters, d.w)
