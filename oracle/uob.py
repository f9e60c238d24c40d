"""FP64 oracle of the union-of-bases spatial prior (test infrastructure only).

The predecessor of MUFFIN's IUWT prior, which the paper compares against it (Sec. 3 and Sec. 4,
Fig. 3), is a union of orthonormal wavelet bases: the first eight Daubechies bases.  Here

    W_s x = (Psi_1 x, ..., Psi_8 x) / sqrt(8),

with Psi_n the J-level orthonormal 2-D discrete wavelet transform of Daubechies' filter with n
vanishing moments (Psi_1 = Haar), separable and periodic.  Each Psi_n is orthonormal, so
W_s^dagger W_s = I: W_s is a tight frame with ||W_s||^2 = 1, and W_s^dagger (u_1..u_8) =
sum_n Psi_n^T u_n / sqrt(8).

Coefficients sit in the usual pyramid layout of an N x N array: after level j (j = 1..J) the
approximation occupies the top-left (N/2^j)^2 block, and the horizontal-detail, vertical-detail and
diagonal-detail blocks of that level sit to its right, below it and diagonally.

Filters come from Daubechies' construction: |m0(w)|^2 = cos^{2n}(w/2) P_n(sin^2(w/2)) with
P_n(y) = sum_{k<n} C(n-1+k, k) y^k, factorised by keeping the roots inside the unit circle
(minimum phase).  Plain numpy throughout; every function is written from these definitions.
"""
from __future__ import annotations

from math import comb

import numpy as np

N_BASES = 8


def daubechies_lowpass(n: int) -> np.ndarray:
    """Scaling filter h (length 2n, sum sqrt(2), orthonormal to its even shifts) with n vanishing
    moments of the wavelet, minimum phase, ordered so that db2 reads (1+s3, 3+s3, 3-s3, 1-s3)/(4 sqrt 2)."""
    if n < 1:
        raise ValueError("n >= 1")
    # roots y_k of P_n(y) = sum_k C(n-1+k, k) y^k
    coeffs = [comb(n - 1 + k, k) for k in range(n)]  # increasing powers
    ys = np.roots(coeffs[::-1]) if n > 1 else np.array([])
    # y = (2 - z - 1/z)/4  <=>  z^2 - (2 - 4y) z + 1 = 0; keep the root inside the unit circle
    zs = []
    for y in ys:
        r = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        zs.append(r[np.argmin(np.abs(r))])
    # m0(z) proportional to (1 + z)^n prod_k (z - z_k), as a polynomial in z (coefficients of z^0..z^{2n-1})
    poly = np.array([1.0 + 0j])
    for _ in range(n):
        poly = np.convolve(poly, [1.0, 1.0])
    for zk in zs:
        poly = np.convolve(poly, [-zk, 1.0])
    h = np.real(poly)
    h = h * (np.sqrt(2.0) / h.sum())
    # orientation: the largest coefficients first (the published db2 ordering)
    if abs(h[0]) < abs(h[-1]):
        h = h[::-1].copy()
    return h


def highpass(h: np.ndarray) -> np.ndarray:
    """Wavelet filter g_k = (-1)^k h_{L-1-k} (the quadrature mirror of h)."""
    L = len(h)
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])


def analysis_1d(x: np.ndarray, h: np.ndarray, axis: int):
    """One periodic level along ``axis``: a_i = sum_k h_k x_{2i+k}, d_i = sum_k g_k x_{2i+k} (indices mod n)."""
    x = np.moveaxis(x, axis, -1)
    n = x.shape[-1]
    g = highpass(h)
    a = np.zeros(x.shape[:-1] + (n // 2,))
    d = np.zeros_like(a)
    idx = np.arange(n // 2)
    for k in range(len(h)):
        xs = x[..., (2 * idx + k) % n]
        a += h[k] * xs
        d += g[k] * xs
    return np.moveaxis(a, -1, axis), np.moveaxis(d, -1, axis)


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """Transpose of analysis_1d: x_m = sum_i (h_{m-2i} a_i + g_{m-2i} d_i) (indices mod n)."""
    a = np.moveaxis(a, axis, -1)
    d = np.moveaxis(d, axis, -1)
    half = a.shape[-1]
    n = 2 * half
    g = highpass(h)
    x = np.zeros(a.shape[:-1] + (n,))
    idx = np.arange(half)
    for k in range(len(h)):
        x[..., (2 * idx + k) % n] += h[k] * a + g[k] * d  # the n/2 indices 2i + k are distinct mod n
    return np.moveaxis(x, -1, axis)


def dwt2(x: np.ndarray, h: np.ndarray, J: int) -> np.ndarray:
    """J-level orthonormal 2-D DWT of an (N, N) image (rows filtered first, then columns), pyramid layout."""
    out = np.array(x, dtype=np.float64, copy=True)
    n = out.shape[-1]
    for _ in range(J):
        blk = out[:n, :n]
        lo, hi = analysis_1d(blk, h, axis=1)  # along rows (last axis)
        ll, lh = analysis_1d(lo, h, axis=0)
        hl, hh = analysis_1d(hi, h, axis=0)
        m = n // 2
        out[:m, :m] = ll
        out[:m, m:n] = hl
        out[m:n, :m] = lh
        out[m:n, m:n] = hh
        n = m
    return out


def idwt2(c: np.ndarray, h: np.ndarray, J: int) -> np.ndarray:
    """Inverse (= transpose, the transform being orthonormal) of dwt2."""
    out = np.array(c, dtype=np.float64, copy=True)
    N = out.shape[-1]
    for j in reversed(range(J)):
        n = N >> j
        m = n // 2
        ll, hl, lh, hh = out[:m, :m], out[:m, m:n], out[m:n, :m], out[m:n, m:n]
        lo = synthesis_1d(ll, lh, h, axis=0)
        hi = synthesis_1d(hl, hh, h, axis=0)
        out[:n, :n] = synthesis_1d(lo, hi, h, axis=1)
    return out


def filters(n_bases: int = N_BASES):
    return [daubechies_lowpass(n) for n in range(1, n_bases + 1)]


def uob(x: np.ndarray, J: int, n_bases: int = N_BASES) -> np.ndarray:
    """W_s x for one image: (n_bases, N, N), each basis's coefficients divided by sqrt(n_bases)."""
    s = 1.0 / np.sqrt(n_bases)
    return np.stack([s * dwt2(x, h, J) for h in filters(n_bases)])


def uob_adjoint(u: np.ndarray, J: int) -> np.ndarray:
    """W_s^dagger u = sum_n Psi_n^T u_n / sqrt(n_bases) for one channel's coefficients (n_bases, N, N)."""
    nb = u.shape[0]
    s = 1.0 / np.sqrt(nb)
    return sum(s * idwt2(u[i], h, J) for i, h in enumerate(filters(nb)))
