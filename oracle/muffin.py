"""FP64 oracle of MUFFIN's operators and of Algorithm 1 (test infrastructure only).

Arrays follow the paper's notation with the channel axis first:

* ``X``  (L, N, N): column ``x_l`` of the paper's ``X`` is ``X[l]`` (Sec. 2);
* ``U``  (L, J+1, N, N): spatial dual, one IUWT decomposition per channel;
* ``V``  (L, N, N): spectral dual, ``V[k]`` is cosine coefficient ``k`` of
  every pixel spectrum;
* ``psf`` (L, N, N): PSF of each channel with its origin at pixel (N/2, N/2).

Readings of points the paper leaves open (each is listed with its reason in
the design notes of the repository):

* ``H_l`` is circular N x N convolution by ``psf_l`` (eq. (model));
* ``W_s`` is the B3-spline a trous IUWT with periodic boundary, taps
  ``[1, 4, 6, 4, 1] / 16`` at offsets ``k 2^j``; ``gen=2`` is the second
  generation the simulations use (Sec. 4), ``gen=1`` the first; J detail planes
  plus the coarse plane;
* ``W_lambda`` is the orthonormal DCT-II of each pixel spectrum (the "cosine
  decomposition" of Sec. 2), so ``W_lambda^dagger`` is its inverse;
* optional channel weights ``w_l = 1 / sigma_l^2`` (eq. (reg)); Algorithm 1
  has none, so the default is 1;
* ``omega`` weights the J+1 planes of the spatial prior: 1 everywhere, or 0 on
  the coarse plane to leave it unpenalised.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import uob as _uob
from . import visibility as _vis

B3_TAPS = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


# --------------------------------------------------------------------------
# Data term: H_l is convolution by the PSF of channel l (Sec. 2, eq. (model))
# --------------------------------------------------------------------------
def transfer(psf: np.ndarray) -> np.ndarray:
    """Transfer function of each H_l: the 2-D DFT of the origin-centred PSF."""
    return np.fft.fft2(np.fft.ifftshift(psf, axes=(-2, -1)), axes=(-2, -1))


def apply_H(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """H_l x_l for every channel (circular convolution)."""
    return np.real(np.fft.ifft2(transfer(psf) * np.fft.fft2(x, axes=(-2, -1)), axes=(-2, -1)))


def apply_Ht(psf: np.ndarray, y: np.ndarray) -> np.ndarray:
    """H_l^dagger y_l for every channel (circular correlation)."""
    return np.real(np.fft.ifft2(np.conj(transfer(psf)) * np.fft.fft2(y, axes=(-2, -1)),
                                axes=(-2, -1)))


def chan_weights(L: int, w=None) -> np.ndarray:
    return np.ones(L) if w is None else np.asarray(w, dtype=np.float64)


def data_gradient(psf, x, y, w=None) -> np.ndarray:
    """Gradient of the fidelity term: w_l H_l^dagger (H_l x_l - y_l) (Algorithm 1, eq. (grad))."""
    wl = chan_weights(x.shape[0], w)
    return wl[:, None, None] * apply_Ht(psf, apply_H(psf, x) - y)


def data_term(psf, x, y, w=None) -> float:
    """sum_l (w_l / 2) ||y_l - H_l x_l||^2 (eq. (reg))."""
    wl = chan_weights(x.shape[0], w)
    r = apply_H(psf, x) - y
    return float(0.5 * np.sum(wl * np.sum(r * r, axis=(-2, -1))))


# --------------------------------------------------------------------------
# Spatial prior: isotropic undecimated wavelet transform (Sec. 2, Sec. 4)
# --------------------------------------------------------------------------
def _atrous_1d(a: np.ndarray, j: int, axis: int) -> np.ndarray:
    s = 2 ** j
    out = np.zeros_like(a)
    for k, h in zip(range(-2, 3), B3_TAPS):
        out += h * np.roll(a, k * s, axis=axis)
    return out


def smooth(c: np.ndarray, j: int) -> np.ndarray:
    """H_j: separable B3-spline smoothing at dilation 2^j, periodic, on the last two axes."""
    return _atrous_1d(_atrous_1d(c, j, -2), j, -1)


def iuwt(x: np.ndarray, J: int, gen: int = 2) -> np.ndarray:
    """W_s x for one image (N, N) -> (J+1, N, N): detail planes w_1..w_J, then c_J.

    c_0 = x, c_{j+1} = H_j c_j; first generation w_{j+1} = c_j - c_{j+1},
    second generation w_{j+1} = c_j - H_j c_{j+1}.
    """
    planes = []
    c = x
    for j in range(J):
        c_next = smooth(c, j)
        planes.append(c - c_next if gen == 1 else c - smooth(c_next, j))
        c = c_next
    planes.append(c)
    return np.stack(planes)


def iuwt_adjoint(u: np.ndarray, J: int, gen: int = 2) -> np.ndarray:
    """W_s^dagger u for one decomposition (J+1, N, N) -> (N, N), the exact transpose.

    Every H_j is a symmetric circulant, so the transpose of
    w_{j+1} = (I - H_j^g) H_{j-1} ... H_0 x  (g = 1 or 2 by generation) is
    accumulated coarse-to-fine: a = u_{J+1};  a = (I - H_j^g) u_{j+1} + H_j a.
    """
    a = u[J]
    for j in reversed(range(J)):
        hu = smooth(u[j], j)
        if gen == 2:
            hu = smooth(hu, j)
        a = u[j] - hu + smooth(a, j)
    return a


def iuwt_synthesis(u: np.ndarray, J: int, gen: int = 2) -> np.ndarray:
    """Perfect-reconstruction inverse of ``iuwt`` (not the adjoint, Sec. 3 remark on eq. (adjointspat))."""
    if gen == 1:
        return u.sum(axis=0)
    c = u[J]
    for j in reversed(range(J)):
        c = u[j] + smooth(c, j)
    return c


def b3_response(omega: np.ndarray) -> np.ndarray:
    """Frequency response of the undilated 1-D B3 filter: 3/8 + cos(w)/2 + cos(2w)/8."""
    return 0.375 + 0.5 * np.cos(omega) + 0.125 * np.cos(2.0 * omega)


def frame_symbol(N: int, J: int, gen: int = 2, omega_w=None) -> np.ndarray:
    """Symbol of W_s^dagger diag(omega) W_s on the N x N DFT grid.

    W_s is a stack of circulants; plane k has symbol g_k, a product of dilated
    B3 responses, so W_s^dagger W_s is circulant with symbol sum_k omega_k |g_k|^2.
    """
    om = plane_weights(J, omega_w)
    f = 2.0 * np.pi * np.fft.fftfreq(N)
    w1, w2 = np.meshgrid(f, f, indexing="ij")
    prod = np.ones((N, N))
    total = np.zeros((N, N))
    for j in range(J):
        h = b3_response((2 ** j) * w1) * b3_response((2 ** j) * w2)
        g = prod * (1.0 - h if gen == 1 else 1.0 - h * h)
        total += om[j] * g * g
        prod = prod * h
    total += om[J] * prod * prod
    return total


def plane_weights(J: int, omega_w=None) -> np.ndarray:
    return np.ones(J + 1) if omega_w is None else np.asarray(omega_w, dtype=np.float64)


# --------------------------------------------------------------------------
# Spectral prior: orthonormal cosine decomposition of each pixel spectrum
# --------------------------------------------------------------------------
def dct_matrix(L: int) -> np.ndarray:
    """W_lambda with X W_lambda = orthonormal DCT-II of every row (pixel spectrum) of X.

    W[l, k] = s_k cos(pi (2l + 1) k / (2L)), s_0 = sqrt(1/L), s_k = sqrt(2/L).
    """
    l = np.arange(L)[:, None]
    k = np.arange(L)[None, :]
    s = np.where(k == 0, np.sqrt(1.0 / L), np.sqrt(2.0 / L))
    return s * np.cos(np.pi * (2 * l + 1) * k / (2.0 * L))


def spectral(X: np.ndarray) -> np.ndarray:
    """X W_lambda with the channel axis first: out[k] = sum_l W[l, k] X[l]."""
    W = dct_matrix(X.shape[0])
    return np.tensordot(W.T, X, axes=(1, 0))


def spectral_adjoint(V: np.ndarray) -> np.ndarray:
    """V W_lambda^dagger: out[l] = sum_k W[l, k] V[k]."""
    W = dct_matrix(V.shape[0])
    return np.tensordot(W, V, axes=(1, 0))


# --------------------------------------------------------------------------
# Proximal maps (Sec. 3)
# --------------------------------------------------------------------------
def sat(u):
    """sat(u): -1 below -1, 1 above 1, u otherwise (Sec. 3)."""
    return np.where(u < -1.0, -1.0, np.where(u > 1.0, 1.0, u))


def soft(z, t):
    """Soft threshold, the prox of t|.|; sat(z) = z - soft(z, 1) (Moreau)."""
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def positive(x):
    """(.)_+: projection on the positive orthant (Sec. 3)."""
    return np.maximum(x, 0.0)


# --------------------------------------------------------------------------
# Problem, objective, step sizes
# --------------------------------------------------------------------------
@dataclass
class Problem:
    dirty: np.ndarray  # (L, N, N)
    psf: np.ndarray  # (L, N, N)
    J: int
    mu_s: float
    mu_l: float
    gen: int = 2
    w: np.ndarray | None = None  # channel weights 1/sigma_l^2
    omega: np.ndarray | None = None  # (J+1,) plane weights of the spatial prior
    tau: float = 0.0
    sigma: float = 1.0
    rho: float = 1.0
    prior: str = "iuwt"  # spatial transform W_s: "iuwt", or "uob" (union of the first 8 Daubechies bases)
    # visibility-domain data term (Sec. 2, eq. (viseq)) in place of H: then dirty and psf are unused
    vis: _vis.VisData | None = None

    @property
    def L(self):
        return self.vis.vis.shape[0] if self.vis is not None else self.dirty.shape[0]

    @property
    def N(self):
        return self.vis.N if self.vis is not None else self.dirty.shape[1]


def problem_gradient(p: Problem, X: np.ndarray) -> np.ndarray:
    """Gradient of the problem's data term at X (image plane, or visibilities when p.vis is set)."""
    if p.vis is not None:
        return _vis.vis_gradient(X, p.vis)
    return data_gradient(p.psf, X, p.dirty, p.w)


def problem_data_term(p: Problem, X: np.ndarray) -> float:
    if p.vis is not None:
        return _vis.vis_data_term(X, p.vis)
    return data_term(p.psf, X, p.dirty, p.w)


def spatial_l1(X, J, gen=2, omega=None, prior="iuwt") -> float:
    """sum_l ||W_s x_l||_1 with plane weights omega (eq. (RegAll), second term without mu_s)."""
    if prior == "uob":
        return float(sum(np.sum(np.abs(_uob.uob(X[l], J))) for l in range(X.shape[0])))
    om = plane_weights(J, omega)
    tot = 0.0
    for l in range(X.shape[0]):
        tot += float(np.sum(om[:, None, None] * np.abs(iuwt(X[l], J, gen))))
    return tot


def spectral_l1(X) -> float:
    """sum_n ||W_lambda x^n||_1 (eq. (RegAll), third term without mu_lambda)."""
    return float(np.sum(np.abs(spectral(X))))


def objective(p: Problem, X: np.ndarray) -> np.ndarray:
    """[total, data, spatial, spectral] of eq. (reg) + eq. (RegAll) at X (inf if X has a negative entry)."""
    data = problem_data_term(p, X)
    spat = p.mu_s * spatial_l1(X, p.J, p.gen, p.omega, p.prior)
    spec = p.mu_l * spectral_l1(X)
    total = data + spat + spec
    if np.any(X < 0):
        total = np.inf
    return np.array([total, data, spat, spec])


def lipschitz(psf, w=None) -> float:
    """beta = max_l w_l ||H_l||^2 = max_l w_l max_k |H_l(k)|^2 (circulant spectrum)."""
    wl = chan_weights(psf.shape[0], w)
    return float(np.max(wl * np.max(np.abs(transfer(psf)) ** 2, axis=(-2, -1))))


def op_norm_sq(p: Problem) -> float:
    """||K||^2 for K = [mu_s W_s per channel; mu_lambda W_lambda per pixel].

    W_lambda is orthonormal, so K^dagger K = mu_s^2 (W_s^dagger W_s per channel) + mu_lambda^2 I.
    """
    # the union of orthonormal bases scaled by 1/sqrt(8) is a tight frame: W_s^dagger W_s = I
    ws2 = 1.0 if p.prior == "uob" else float(np.max(frame_symbol(p.N, p.J, p.gen, p.omega)))
    return p.mu_s ** 2 * ws2 + p.mu_l ** 2


def step_sizes(p: Problem):
    """(tau, sigma, rho, beta, ||K||^2) satisfying the convergence condition of the primal-dual method.

    Condition: 1/tau - sigma ||K||^2 > beta / 2 and 0 < rho < delta with
    delta = 2 - (beta / 2) / (1/tau - sigma ||K||^2).  If tau <= 0 it is set to
    0.99 / (beta / 2 + sigma ||K||^2).
    """
    beta = _vis.vis_lipschitz(p.vis) if p.vis is not None else lipschitz(p.psf, p.w)
    k2 = op_norm_sq(p)
    tau = p.tau if p.tau > 0 else 0.99 / (beta / 2.0 + p.sigma * k2)
    margin = 1.0 / tau - p.sigma * k2
    if not margin > beta / 2.0:
        raise ValueError("step sizes violate 1/tau - sigma ||K||^2 > beta/2")
    delta = 2.0 - (beta / 2.0) / margin
    if not (0.0 < p.rho < delta):
        raise ValueError("relaxation rho outside (0, delta)")
    return tau, p.sigma, p.rho, beta, k2


# --------------------------------------------------------------------------
# The primal-dual method (Sec. 3)
#
# The problem of eq. (reg) + eq. (RegAll) has the form
#     min_X  f(X) + g(X) + h(K X)
# with f the smooth data term (gradient eq. (grad)), g the indicator of the
# positive orthant, h = ||.||_1 and K the stacked analysis operator of the
# prior.  The method Sec. 3 uses for it (the one it cites for its step sizes)
# alternates a forward-backward step on X with a proximal step on the dual
# variable of K, then relaxes both.  Below, that step is written once for any
# (f, g, h, K), and the MUFFIN iteration is that step with MUFFIN's operators.
# --------------------------------------------------------------------------
def primal_dual_step(x, duals, grad_f, K, K_adj, prox_g, prox_h_conj, tau, sigma, rho):
    """One step of the primal-dual method for min f(x) + g(x) + h(K x).

    ``duals`` is a tuple of dual blocks, one per block of K's output; ``K`` maps a
    primal point to a tuple of such blocks and ``K_adj`` a tuple back to the primal
    space.  With p = prox_g(x - tau (grad_f(x) + K^dagger y)) and
    q = prox_{sigma h*}(y + sigma K (2p - x)), the new point is rho (p, q) + (1 - rho) (x, y).
    """
    p = prox_g(x - tau * (grad_f(x) + K_adj(*duals)))
    ext = K(2.0 * p - x)
    q = tuple(prox_h_conj(y + sigma * k) for y, k in zip(duals, ext))
    x_new = rho * p + (1.0 - rho) * x
    duals_new = tuple(rho * qi + (1.0 - rho) * yi for qi, yi in zip(q, duals))
    return x_new, duals_new


def l1_conj_prox(z):
    """prox of sigma h* for h = ||.||_1: h* is the indicator of the unit l-infinity ball, whose prox
    (for any sigma) is the projection onto that ball, entry by entry: ``sat`` (Sec. 3)."""
    return sat(z)


@dataclass
class AnalysisOperator:
    """K of the prior in eq. (RegAll): K X = (mu_s omega W_s x_l for every channel l,
    mu_lambda X W_lambda), so that mu_s sum_l ||omega W_s x_l||_1 + mu_lambda sum_n ||W_lambda x^n||_1
    = ||K X||_1.  Its dual variable is the pair (U, V) of Sec. 3."""
    J: int
    gen: int
    mu_s: float
    mu_l: float
    omega: np.ndarray  # (J+1,)
    prior: str = "iuwt"

    def spatial(self, x):
        """mu_s omega W_s x for one channel image (N, N) -> (J+1, N, N) (union of bases: (8, N, N))."""
        if self.prior == "uob":
            return self.mu_s * _uob.uob(x, self.J)
        return self.mu_s * self.omega[:, None, None] * iuwt(x, self.J, self.gen)

    def spatial_adjoint(self, u):
        """mu_s W_s^dagger (omega u) for one channel's decomposition -> (N, N)."""
        if self.prior == "uob":
            return self.mu_s * _uob.uob_adjoint(u, self.J)
        return self.mu_s * iuwt_adjoint(self.omega[:, None, None] * u, self.J, self.gen)

    def apply(self, X):
        return np.stack([self.spatial(x) for x in X]), self.mu_l * spectral(X)

    def adjoint(self, U, V):
        return np.stack([self.spatial_adjoint(u) for u in U]) + self.mu_l * spectral_adjoint(V)


def analysis_operator(p: Problem) -> AnalysisOperator:
    return AnalysisOperator(J=p.J, gen=p.gen, mu_s=p.mu_s, mu_l=p.mu_l, omega=plane_weights(p.J, p.omega),
                            prior=p.prior)


@dataclass
class State:
    X: np.ndarray  # (L, N, N)
    U: np.ndarray  # (L, J+1, N, N)
    V: np.ndarray  # (L, N, N)
    k: int = 0


def init_state(p: Problem, X0=None) -> State:
    """Initial point (Algorithm 1, "Initialize"): X = max(X0, 0) or 0, U = V = 0."""
    L, N = p.L, p.N
    X = np.zeros((L, N, N)) if X0 is None else positive(np.asarray(X0, dtype=np.float64))
    planes = _uob.N_BASES if p.prior == "uob" else p.J + 1
    return State(X=X, U=np.zeros((L, planes, N, N)), V=np.zeros((L, N, N)))


def iterate(p: Problem, st: State, tau: float) -> State:
    """One MUFFIN iteration (Algorithm 1): the primal-dual step with f the data term, g the
    positivity indicator, h = ||.||_1 and K the stacked analysis operator."""
    K = analysis_operator(p)
    X, (U, V) = primal_dual_step(st.X, (st.U, st.V), lambda x: problem_gradient(p, x),
                                 K.apply, K.adjoint, positive, l1_conj_prox, tau, p.sigma, p.rho)
    return State(X=X, U=U, V=V, k=st.k + 1)


def solve(p: Problem, n_iter: int, X0=None, tau: float | None = None, record_every: int = 0, state=None):
    """Run n_iter iterations of Algorithm 1 from init_state (or from ``state``); returns
    (state, objective history every record_every iterations)."""
    if tau is None:
        tau = step_sizes(p)[0]
    st = init_state(p, X0) if state is None else state
    hist = []
    for it in range(n_iter):
        st = iterate(p, st, tau)
        if record_every and (it + 1) % record_every == 0:
            hist.append(objective(p, st.X)[0])
    return st, np.array(hist)


def two_step_calibration(p: Problem, n1: int, n2: int, tau1: float | None = None, tau2: float | None = None):
    """The calibration strategy of Sec. 4: step 1 runs the method with mu_lambda = 0 (the problem
    separates over the channels), step 2 keeps mu_s and starts the full method (mu_lambda of p)
    from step 1's X; U and V start at 0 in both steps (Algorithm 1's initialisation with step 1's
    X as the initial condition).  Returns (state after step 1, state after step 2)."""
    p1 = Problem(**{**p.__dict__, "mu_l": 0.0})
    st1, _ = solve(p1, n1, tau=tau1)
    st2, _ = solve(p, n2, X0=st1.X, tau=tau2)
    return st1, st2


def snr_db(X, X_true) -> float:
    """SNR(X, X*) = 10 log10(||X*||^2 / ||X - X*||^2) (Sec. 4)."""
    return float(10.0 * np.log10(np.sum(X_true ** 2) / np.sum((X - X_true) ** 2)))
