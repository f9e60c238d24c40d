"""Seeded synthetic radio-interferometric cubes (sky, PSF, dirty image).

This module is the only code shared between the FP64 oracle tests and the GPU
path: it draws the inputs and nothing else.  It holds none of the
reconstruction's arithmetic (no wavelet, cosine transform, proximal step or
iteration).  The observation itself, ``y_l = psf_l (*) x_l + n_l`` (the
image-plane model of Sec. 2, eq. (model)), is simulated here with numpy's FFT
because a dirty image is an input of the method, not a step of it.

Recipe (the paper's MeerKAT PSFs and M31 sky are not available, so these
synthetic cubes stand in for them):

* channels ``nu_l = nu_min + (nu_max - nu_min) * l / (L - 1)``, reference
  frequency ``nu_0 = nu_min`` (``L = 1`` gives ``nu = nu_min``);
* sky: ``S`` Gaussian sources with continuous centres uniform in ``[0, N)^2``,
  widths ``s ~ U[1, 4]`` px, peaks ``A ~ U[0.5, 1]`` and power-law spectra
  ``(nu_l / nu_0)^alpha`` with ``alpha ~ U[-1, 0]``; distances are periodic
  minimum-image distances;
* PSF of channel ``l``: ``B`` baselines ``(u, v) ~ U[-N/4, N/4)^2`` scaled by
  ``nu_l / nu_0`` and rounded; the uv mask holds each baseline, its Hermitian
  mirror and the origin; ``psf_l = fftshift(|IFFT2(mask_l)|)`` normalised to
  peak 1 (the paper quotes sidelobes as a fraction of the maximum, Fig. 1), so
  its origin sits at pixel ``(N/2, N/2)``;
* noise: i.i.d. ``N(0, noise_sigma^2)`` added to the dirty cube.

Draw order from ``numpy.random.default_rng(seed)``: source centres (2S), widths
(S), peaks (S), indices (S), baselines (2B), then the noise channel by channel.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class CubeSpec:
    """Shape and generator settings of one synthetic cube."""

    N: int
    L: int
    J: int
    n_sources: int
    n_baselines: int
    seed: int = 0
    noise_sigma: float = 0.01
    nu_min: float = 1.0
    nu_max: float = 1.5
    iters: int = 50


@dataclass
class Cube:
    spec: CubeSpec
    sky: np.ndarray  # (L, N, N)
    psf: np.ndarray  # (L, N, N), origin at (N/2, N/2)
    dirty: np.ndarray  # (L, N, N)
    nu: np.ndarray = field(default_factory=lambda: np.zeros(0))


# Named workloads (the shapes of the paper's Monte Carlo cubes scaled up to a
# single MI355X): small parity cube, medium parity cube, large throughput cube,
# and the CNN training cube shape.
WORKLOADS = {
    "cube64_L8_J3": CubeSpec(N=64, L=8, J=3, n_sources=5, n_baselines=200, seed=0, iters=50),
    "cube256_L64_J4": CubeSpec(N=256, L=64, J=4, n_sources=20, n_baselines=2000, seed=0, iters=200),
    "cube1024_L256_J5": CubeSpec(N=1024, L=256, J=5, n_sources=200, n_baselines=20000, seed=0,
                                 iters=200),
}


def uneven_batch_specs(n_cubes: int = 32, J: int = 4, seed: int = 7) -> list[CubeSpec]:
    """Side lengths from {128, 256, 384, 512}, L ~ U{16..128}; cube i uses seed 1000 + i."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([128, 256, 384, 512], size=n_cubes)
    Ls = rng.integers(16, 129, size=n_cubes)
    return [CubeSpec(N=int(sides[i]), L=int(Ls[i]), J=J, n_sources=20, n_baselines=2000,
                     seed=1000 + i, iters=200) for i in range(n_cubes)]


def channel_freqs(L: int, nu_min: float = 1.0, nu_max: float = 1.5) -> np.ndarray:
    if L == 1:
        return np.array([nu_min])
    return nu_min + (nu_max - nu_min) * np.arange(L) / (L - 1)


def _gauss_1d(N: int, centre: np.ndarray, width: np.ndarray) -> np.ndarray:
    """(S, N) periodic minimum-image Gaussian profiles along one axis."""
    grid = np.arange(N)[None, :]
    d = (grid - centre[:, None] + N / 2.0) % N - N / 2.0
    return np.exp(-(d * d) / (2.0 * width[:, None] ** 2))


def make_cube(spec: CubeSpec, dtype=np.float64, with_sky: bool = True) -> Cube:
    N, L, S, B = spec.N, spec.L, spec.n_sources, spec.n_baselines
    rng = np.random.default_rng(spec.seed)
    centres = rng.uniform(0.0, N, size=(2, S))
    widths = rng.uniform(1.0, 4.0, size=S)
    peaks = rng.uniform(0.5, 1.0, size=S)
    index = rng.uniform(-1.0, 0.0, size=S)
    uv = rng.uniform(-N / 4.0, N / 4.0, size=(B, 2))
    nu = channel_freqs(L, spec.nu_min, spec.nu_max)
    nu0 = spec.nu_min

    g0 = _gauss_1d(N, centres[0], widths)  # rows
    g1 = _gauss_1d(N, centres[1], widths)  # columns
    sky = np.empty((L, N, N), dtype=dtype) if with_sky else None
    psf = np.empty((L, N, N), dtype=dtype)
    dirty = np.empty((L, N, N), dtype=dtype)
    for l in range(L):
        amp = peaks * (nu[l] / nu0) ** index  # (S,)
        x = (g0.T * amp[None, :]) @ g1  # (N, N) = sum_s amp_s g0_s (x) g1_s
        ij = np.rint(uv * (nu[l] / nu0)).astype(np.int64)
        mask = np.zeros((N, N))
        mask[ij[:, 0] % N, ij[:, 1] % N] = 1.0
        mask[(-ij[:, 0]) % N, (-ij[:, 1]) % N] = 1.0
        mask[0, 0] = 1.0
        p0 = np.abs(np.fft.ifft2(mask))  # origin at (0, 0)
        p0 /= p0.max()
        # simulated observation: circular convolution with the origin-centred PSF
        y = np.fft.irfft2(np.fft.rfft2(x) * np.fft.rfft2(p0), s=(N, N))
        y += rng.normal(0.0, spec.noise_sigma, size=(N, N))
        psf[l] = np.fft.fftshift(p0)
        dirty[l] = y
        if with_sky:
            sky[l] = x
    return Cube(spec=spec, sky=sky, psf=psf, dirty=dirty, nu=nu)


# ------------------------------------------------------------------ visibility-domain inputs
@dataclass(frozen=True)
class VisSpec:
    """Inputs of the visibility-domain data term: a sky cube, K baselines and the channels'
    wavelengths (Sec. 2, eq. (viseq)).

    * wavelengths ``lambda_l = lambda_0 nu_0 / nu_l`` with the channel frequencies of the image
      cubes (``nu`` from ``nu_min`` to ``nu_max``, ``lambda_0 = 1`` metre at ``nu_0 = nu_min``);
    * baselines in metres: ``u, v ~ U[-b_max, b_max)`` and ``w ~ U[-w_frac b_max, w_frac b_max)``
      (``b_max`` in units of ``lambda_0``);
    * pixel size ``cell = lambda_min / (4 b_max)`` (direction cosines), so that the longest
      baseline at the highest frequency spans N/4 cycles across the image, as the uv masks of the
      image-plane cubes do;
    * sky: the Gaussian sources of ``make_cube`` with this spec's own draws;
    * noise: complex, i.i.d. ``N(0, noise_sigma^2)`` in each part, one value per visibility.

    Draw order from ``numpy.random.default_rng(seed)``: source centres (2S), widths (S), peaks
    (S), indices (S), baselines (3K), then the noise (real parts, imaginary parts).
    """

    N: int
    L: int
    K: int
    n_sources: int
    seed: int = 0
    b_max: float = 0.0  # 0: 2 N
    w_frac: float = 0.5
    noise_sigma: float = 0.01
    nu_min: float = 1.0
    nu_max: float = 1.5


@dataclass
class VisInputs:
    spec: VisSpec
    sky: np.ndarray  # (L, N, N)
    uvw: np.ndarray  # (K, 3) metres
    lam: np.ndarray  # (L,) metres
    cell: float
    noise: np.ndarray  # (L, K) complex


def make_vis_inputs(spec: VisSpec) -> VisInputs:
    N, L, S, K = spec.N, spec.L, spec.n_sources, spec.K
    rng = np.random.default_rng(spec.seed)
    centres = rng.uniform(0.0, N, size=(2, S))
    widths = rng.uniform(1.0, 4.0, size=S)
    peaks = rng.uniform(0.5, 1.0, size=S)
    index = rng.uniform(-1.0, 0.0, size=S)
    b_max = spec.b_max if spec.b_max > 0 else 2.0 * N
    uvw = np.empty((K, 3))
    uvw[:, 0:2] = rng.uniform(-b_max, b_max, size=(K, 2))
    uvw[:, 2] = rng.uniform(-spec.w_frac * b_max, spec.w_frac * b_max, size=K)
    nu = channel_freqs(L, spec.nu_min, spec.nu_max)
    lam = spec.nu_min / nu
    cell = float(lam.min() / (4.0 * b_max))
    g0 = _gauss_1d(N, centres[0], widths)
    g1 = _gauss_1d(N, centres[1], widths)
    sky = np.empty((L, N, N))
    for l in range(L):
        amp = peaks * (nu[l] / spec.nu_min) ** index
        sky[l] = (g0.T * amp[None, :]) @ g1
    noise = spec.noise_sigma * (rng.normal(size=(L, K)) + 1j * rng.normal(size=(L, K)))
    return VisInputs(spec=spec, sky=sky, uvw=uvw, lam=lam, cell=cell, noise=noise)
