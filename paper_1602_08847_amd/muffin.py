"""Python binding of libmuffin (C ABI in include/muffin.h): argument marshalling only.

Every computation runs in the HIP library.  Device arrays are torch tensors on the GPU (float32,
contiguous); their ``data_ptr()`` and torch's current stream are handed to the library.  If the
library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MUFFIN_LIBRARY selects another build of the same library (the checked build of the tests)
LIB_PATH = os.environ.get("MUFFIN_LIBRARY") or os.path.join(_HERE, "libmuffin.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmuffin not built at {LIB_PATH}; run __graft_entry__.build()")
# torch is loaded first so that libmuffin binds to the HIP runtime torch already uses (both carry
# the same soname): device pointers and streams are shared with torch.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ESTEP, ESTATE = 0, -1, -2, -3, -4, -5, -6
OP_H, OP_HT, OP_GRAD, OP_IUWT, OP_IUWT_ADJ, OP_DCT, OP_IDCT, OP_IUWT_SCHED = 1, 2, 3, 4, 5, 6, 7, 8
OP_PHI, OP_PHI_ADJ = 9, 10  # visibility contexts: image -> visibilities, visibilities -> image

EXPORTS = [
    "muffin_init", "muffin_step", "muffin_solve", "muffin_objective", "muffin_info",
    "muffin_set_x", "muffin_get_x", "muffin_get_u", "muffin_get_v", "muffin_state_size",
    "muffin_get_state", "muffin_set_state", "muffin_apply_op", "muffin_profile",
    "muffin_step_timed", "muffin_free", "muffin_strerror", "muffin_last_error",
    "muffin_cnn_create", "muffin_cnn_param_count", "muffin_cnn_get_params", "muffin_cnn_set_params",
    "muffin_cnn_predict", "muffin_cnn_predict_noalloc", "muffin_cnn_loss_grad", "muffin_cnn_train_step", "muffin_cnn_layer",
    "muffin_cnn_free", "muffin_warm_start", "muffin_autotune", "muffin_batch_init", "muffin_batch_step",
    "muffin_batch_step_timed", "muffin_batch_objective", "muffin_batch_get_x", "muffin_batch_info",
    "muffin_batch_autotune", "muffin_batch_free", "muffin_step_monitored", "muffin_snr", "muffin_batch_snr",
    "muffin_warm_input", "muffin_batch_set_x", "muffin_batch_warm_input", "muffin_uob_filter",
    "muffin_debug_oob", "muffin_init_vis", "muffin_vis_residual", "muffin_set_band_tiles",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("L", ctypes.c_int32), ("J", ctypes.c_int32),
        ("iuwt_gen", ctypes.c_int32), ("penalize_coarse", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("prior", ctypes.c_int32),
        ("mu_s", ctypes.c_double), ("mu_lambda", ctypes.c_double),
        ("tau", ctypes.c_double), ("sigma", ctypes.c_double), ("rho", ctypes.c_double),
        ("chan_weight", ctypes.POINTER(ctypes.c_float)),
    ]


_vp, _i32, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double


class VisDesc(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("cell", ctypes.c_double),
        ("uvw", ctypes.POINTER(ctypes.c_double)), ("lam", ctypes.POINTER(ctypes.c_double)),
        ("power_iters", ctypes.c_int32),
    ]
_lib.muffin_init.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(Params), _vp, _vp, ctypes.c_int, _vp]
_lib.muffin_init_vis.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(Params), ctypes.POINTER(VisDesc), _vp,
                                 ctypes.c_int, _vp]
_lib.muffin_vis_residual.argtypes = [_vp, _vp, ctypes.c_int]
_lib.muffin_step.argtypes = [_vp, _i32]
_lib.muffin_solve.argtypes = [_vp, _i32, _i32, _i32, _dbl, _dbl, ctypes.POINTER(_i32), ctypes.POINTER(_dbl)]
_lib.muffin_step_monitored.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_snr.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(_dbl)]
_lib.muffin_batch_snr.argtypes = [_vp, _i32, _vp, ctypes.c_int, ctypes.POINTER(_dbl)]
_lib.muffin_warm_input.argtypes = [_vp, _vp, ctypes.c_int]
_lib.muffin_batch_set_x.argtypes = [_vp, _i32, _vp, ctypes.c_int]
_lib.muffin_batch_warm_input.argtypes = [_vp, _i32, _vp, ctypes.c_int]
_lib.muffin_uob_filter.argtypes = [_i32, ctypes.POINTER(_dbl), _i32]
_lib.muffin_debug_oob.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
_lib.muffin_set_band_tiles.argtypes = [_i32, _i32, _i32, _i32, _i32]
_lib.muffin_objective.argtypes = [_vp, ctypes.POINTER(_dbl)]
_lib.muffin_info.argtypes = [_vp, ctypes.POINTER(_dbl)]
for _n in ("muffin_set_x", "muffin_get_x", "muffin_get_u", "muffin_get_v"):
    getattr(_lib, _n).argtypes = [_vp, _vp, ctypes.c_int]
_lib.muffin_state_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.muffin_get_state.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.muffin_set_state.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.muffin_apply_op.argtypes = [_vp, ctypes.c_int, _vp, _vp]
_lib.muffin_profile.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_step_timed.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_free.argtypes = [_vp]
_lib.muffin_free.restype = None
_lib.muffin_strerror.argtypes = [ctypes.c_int]
_lib.muffin_strerror.restype = ctypes.c_char_p
_lib.muffin_last_error.argtypes = []
_lib.muffin_last_error.restype = ctypes.c_char_p
_lib.muffin_cnn_create.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.c_uint64, _vp]
_lib.muffin_cnn_param_count.argtypes = [_vp, ctypes.POINTER(_i32)]
_lib.muffin_cnn_get_params.argtypes = [_vp, _vp, _i32]
_lib.muffin_cnn_set_params.argtypes = [_vp, _vp, _i32]
_lib.muffin_cnn_predict.argtypes = [_vp, _vp, _vp, _i32, _i32]
_lib.muffin_cnn_predict_noalloc.argtypes = [_vp, _vp, _vp, _i32, _i32]
_lib.muffin_cnn_loss_grad.argtypes = [_vp, _vp, _vp, _i32, _i32, ctypes.POINTER(_dbl), _vp]
_lib.muffin_cnn_train_step.argtypes = [_vp, _vp, _vp, _i32, _i32, ctypes.c_float, ctypes.POINTER(_dbl)]
_lib.muffin_cnn_layer.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _i32]
_lib.muffin_cnn_free.argtypes = [_vp]
_lib.muffin_cnn_free.restype = None
_lib.muffin_warm_start.argtypes = [_vp, _vp]
_lib.muffin_autotune.argtypes = [_vp, _i32, ctypes.c_char_p, ctypes.c_size_t]
_lib.muffin_batch_init.argtypes = [ctypes.POINTER(_vp), _i32, ctypes.POINTER(Params), ctypes.POINTER(_vp),
                                   ctypes.POINTER(_vp), ctypes.c_int, _vp]
_lib.muffin_batch_step.argtypes = [_vp, _i32]
_lib.muffin_batch_step_timed.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_batch_objective.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_batch_get_x.argtypes = [_vp, _i32, _vp, ctypes.c_int]
_lib.muffin_batch_info.argtypes = [_vp, _i32, ctypes.POINTER(_dbl)]
_lib.muffin_batch_autotune.argtypes = [_vp, _i32, ctypes.c_char_p, ctypes.c_size_t]
_lib.muffin_batch_free.argtypes = [_vp]
_lib.muffin_batch_free.restype = None


FLAG_SINGLE_SCALE = 1  # one IUWT launch per scale (same results as the fused pairs of scales)
FLAG_NO_FUSED_TAIL = 2  # last analysis pair and the next first adjoint pair as two launches (same results)
FLAG_FUSED_TAIL = 4  # always fuse them (by default: when the cube is large enough, or as autotuned)
FLAG_UOB_ALL_BASES = 8  # union of bases: one workgroup runs all bases of a tile on every level (same results)
FLAG_UOB_PER_BASIS = 16  # union of bases: one workgroup per basis after the first level (same results)
FLAG_SPECTRAL_DENSE = 32  # L without an FFT plan: cosine-table products for the spectral step
FLAG_SPECTRAL_BLUESTEIN = 64  # L without an FFT plan: Bluestein DFTs for the spectral step
# kernel families of the IUWT launches (the autotuner report's "family")
FAMILY_ANALYSIS, FAMILY_ADJOINT, FAMILY_ANALYSIS_G1, FAMILY_ADJOINT_G1 = 0, 1, 2, 3
FAMILY_PAIR_ANALYSIS, FAMILY_PAIR_ADJOINT, FAMILY_TRIPLE_ANALYSIS, FAMILY_TRIPLE_ADJOINT = 5, 6, 7, 8
FAMILY_FUSED_PAIR, FAMILY_PAIR_ANALYSIS_G1, FAMILY_PAIR_ADJOINT_G1 = 9, 10, 11
STOP_OBJECTIVE, STOP_CHANGE = 0, 1  # stopping rules of muffin_solve
PRIOR_IUWT, PRIOR_UOB = 0, 1  # spatial prior: the IUWT, or the union of the first 8 Daubechies bases
UOB_BASES = 8


class MuffinError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.muffin_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.muffin_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc: int, where: str):
    if rc != OK:
        raise MuffinError(rc, where)


def _torch():
    import torch
    return torch


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, shape, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Muffin:
    """One reconstruction context (one cube) on the current GPU."""

    def __init__(self, dirty, psf, J: int, mu_s: float, mu_lambda: float, iuwt_gen: int = 2,
                 penalize_coarse: bool = True, tau: float = 0.0, sigma: float = 1.0,
                 rho: float = 1.0, chan_weight=None, flags: int = 0, prior: int = PRIOR_IUWT):
        torch = _torch()
        dirty = torch.as_tensor(dirty, dtype=torch.float32).cuda().contiguous()
        psf = torch.as_tensor(psf, dtype=torch.float32).cuda().contiguous()
        L, N, N2 = dirty.shape
        if N != N2 or tuple(psf.shape) != (L, N, N):
            raise ValueError("dirty and psf must both be [L][N][N]")
        self.N, self.L, self.J, self.K = N, L, J, 0
        self.planes = UOB_BASES if prior == PRIOR_UOB else J + 1  # dual planes per channel
        self._cw = None
        p = Params(N=N, L=L, J=J, iuwt_gen=iuwt_gen, penalize_coarse=int(bool(penalize_coarse)),
                   flags=flags, prior=prior, mu_s=mu_s, mu_lambda=mu_lambda, tau=tau, sigma=sigma, rho=rho)
        if chan_weight is not None:
            self._cw = np.ascontiguousarray(chan_weight, dtype=np.float32)
            if self._cw.shape != (L,):
                raise ValueError("chan_weight must have shape (L,)")
            p.chan_weight = self._cw.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        h = ctypes.c_void_p()
        _check(_lib.muffin_init(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(dirty.data_ptr()),
                                ctypes.c_void_p(psf.data_ptr()), 1, _stream_handle()), "muffin_init")
        self._h = h

    @classmethod
    def from_visibilities(cls, vis, uvw, lam, cell: float, N: int, J: int, mu_s: float, mu_lambda: float,
                          iuwt_gen: int = 2, penalize_coarse: bool = True, tau: float = 0.0, sigma: float = 1.0,
                          rho: float = 1.0, flags: int = 0, prior: int = PRIOR_IUWT, power_iters: int = 0,
                          chan_weight=None):
        """A context with the visibility-domain data term: vis (L, K) complex (or (L, K, 2) float),
        uvw (K, 3) baselines in metres, lam (L,) wavelengths in metres, cell the pixel size, optional
        channel weights (L,)."""
        torch = _torch()
        v = np.asarray(vis)
        if np.iscomplexobj(v):
            v = np.stack([v.real, v.imag], axis=-1)
        vt = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float32)).cuda().contiguous()
        if vt.dim() != 3 or vt.shape[2] != 2:
            raise ValueError("vis must be (L, K) complex or (L, K, 2) float")
        L, K = int(vt.shape[0]), int(vt.shape[1])
        self = cls.__new__(cls)
        self.N, self.L, self.J, self.K = N, L, J, K
        self.planes = UOB_BASES if prior == PRIOR_UOB else J + 1
        self._cw = None
        self._uvw = np.ascontiguousarray(uvw, dtype=np.float64)
        self._lam = np.ascontiguousarray(lam, dtype=np.float64)
        if self._uvw.shape != (K, 3) or self._lam.shape != (L,):
            raise ValueError("uvw must be (K, 3) and lam (L,)")
        d = VisDesc(K=K, cell=cell, uvw=self._uvw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    lam=self._lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), power_iters=power_iters)
        p = Params(N=N, L=L, J=J, iuwt_gen=iuwt_gen, penalize_coarse=int(bool(penalize_coarse)),
                   flags=flags, prior=prior, mu_s=mu_s, mu_lambda=mu_lambda, tau=tau, sigma=sigma, rho=rho)
        if chan_weight is not None:
            self._cw = np.ascontiguousarray(chan_weight, dtype=np.float32)
            if self._cw.shape != (L,):
                raise ValueError("chan_weight must have shape (L,)")
            p.chan_weight = self._cw.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        h = ctypes.c_void_p()
        _check(_lib.muffin_init_vis(ctypes.byref(h), ctypes.byref(p), ctypes.byref(d),
                                    ctypes.c_void_p(vt.data_ptr()), 1, _stream_handle()), "muffin_init_vis")
        self._h = h
        return self

    def vis_residual(self):
        """Phi x - v of the current X, (L, K, 2) float32 on the GPU."""
        return self._get(_lib.muffin_vis_residual, (self.L, self.K, 2))

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.muffin_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ iteration
    def step(self, n: int = 1):
        _check(_lib.muffin_step(self._h, n), "muffin_step")

    def step_timed(self, n: int) -> float:
        ms = ctypes.c_double()
        _check(_lib.muffin_step_timed(self._h, n, ctypes.byref(ms)), "muffin_step_timed")
        return ms.value

    def profile(self, n: int) -> np.ndarray:
        out = (ctypes.c_double * 32)()
        _check(_lib.muffin_profile(self._h, n, out), "muffin_profile")
        return np.array(out[:])

    def solve(self, max_iter: int, check_every: int = 10, tol: float = 1e-4, f_ref: float = math.nan,
              rule: int = STOP_OBJECTIVE):
        it, f = _i32(), _dbl()
        _check(_lib.muffin_solve(self._h, max_iter, check_every, rule, tol, f_ref, ctypes.byref(it),
                                 ctypes.byref(f)), "muffin_solve")
        return it.value, f.value

    def step_monitored(self, n: int = 1) -> dict:
        out = (_dbl * 6)()
        _check(_lib.muffin_step_monitored(self._h, n, out), "muffin_step_monitored")
        keys = ["dX", "X", "dU", "U", "dV", "V"]
        return dict(zip(keys, out[:]))

    def snr(self, truth) -> float:
        torch = _torch()
        t = torch.as_tensor(truth, dtype=torch.float32).cuda().contiguous()
        out = _dbl()
        _check(_lib.muffin_snr(self._h, _dev_ptr(t, (self.L, self.N, self.N), "truth"), 1, ctypes.byref(out)),
               "muffin_snr")
        return out.value

    def warm_input(self):
        return self._get(_lib.muffin_warm_input, (self.L, self.N, self.N))

    def objective(self) -> np.ndarray:
        out = (ctypes.c_double * 4)()
        _check(_lib.muffin_objective(self._h, out), "muffin_objective")
        return np.array(out[:])

    def info(self) -> dict:
        out = (ctypes.c_double * 8)()
        _check(_lib.muffin_info(self._h, out), "muffin_info")
        keys = ["tau", "sigma", "rho", "beta", "K2", "Ws2", "delta", "iter"]
        return dict(zip(keys, out[:]))

    # ------------------------------------------------------------------ state
    def set_x(self, x0):
        torch = _torch()
        x0 = torch.as_tensor(x0, dtype=torch.float32).cuda().contiguous()
        _check(_lib.muffin_set_x(self._h, _dev_ptr(x0, (self.L, self.N, self.N), "x0"), 1), "muffin_set_x")
        torch.cuda.current_stream().synchronize()

    def _get(self, fn, shape):
        torch = _torch()
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
        _check(fn(self._h, ctypes.c_void_p(out.data_ptr()), 1), fn.__name__)
        return out

    def get_x(self):
        return self._get(_lib.muffin_get_x, (self.L, self.N, self.N))

    def get_u(self):
        return self._get(_lib.muffin_get_u, (self.L, self.planes, self.N, self.N))

    def get_v(self):
        return self._get(_lib.muffin_get_v, (self.L, self.N, self.N))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(_lib.muffin_state_size(self._h, ctypes.byref(n)), "muffin_state_size")
        buf = ctypes.create_string_buffer(n.value)
        _check(_lib.muffin_get_state(self._h, buf, n.value), "muffin_get_state")
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(_lib.muffin_set_state(self._h, buf, len(blob)), "muffin_set_state")

    def autotune(self, reps: int = 3) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(_lib.muffin_autotune(self._h, reps, buf, len(buf)), "muffin_autotune")
        return buf.value.decode()

    def warm_start(self, net: "Cnn"):
        _check(_lib.muffin_warm_start(self._h, net._h), "muffin_warm_start")
        _torch().cuda.current_stream().synchronize()

    # ------------------------------------------------------------------ single operators
    def apply_op(self, op: int, x):
        torch = _torch()
        L, N = self.L, self.N
        cube, ucube, vshape = (L, N, N), (L, self.planes, N, N), (L, self.K, 2)
        in_shape = ucube if op == OP_IUWT_ADJ else vshape if op == OP_PHI_ADJ else cube
        out_shape = ucube if op in (OP_IUWT, OP_IUWT_SCHED) else vshape if op == OP_PHI else cube
        x = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        out = torch.empty(out_shape, dtype=torch.float32, device="cuda")
        _check(_lib.muffin_apply_op(self._h, op, _dev_ptr(x, in_shape, "in"),
                                    _dev_ptr(out, out_shape, "out")), "muffin_apply_op")
        return out


class Cnn:
    """The warm-start network (four 3x3 convolutions, BF16 MFMA kernels) on the current GPU."""

    def __init__(self, seed: int = 0, features: int = 32):
        h = ctypes.c_void_p()
        _check(_lib.muffin_cnn_create(ctypes.byref(h), features, seed, _stream_handle()), "muffin_cnn_create")
        self._h = h
        n = _i32()
        _check(_lib.muffin_cnn_param_count(self._h, ctypes.byref(n)), "muffin_cnn_param_count")
        self.n_params = n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.muffin_cnn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(_lib.muffin_cnn_get_params(self._h, out.ctypes.data, self.n_params), "muffin_cnn_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.shape != (self.n_params,):
            raise ValueError("parameter vector has the wrong size")
        _check(_lib.muffin_cnn_set_params(self._h, p.ctypes.data, self.n_params), "muffin_cnn_set_params")

    @staticmethod
    def _planes(x):
        torch = _torch()
        x = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        if x.dim() != 3 or x.shape[1] != x.shape[2]:
            raise ValueError("expected [B][N][N]")
        return x

    def predict(self, x):
        torch = _torch()
        x = self._planes(x)
        out = torch.empty_like(x)
        B, N = x.shape[0], x.shape[1]
        _check(_lib.muffin_cnn_predict(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       B, N), "muffin_cnn_predict")
        torch.cuda.current_stream().synchronize()
        return out

    def predict_noalloc(self, x, out=None):
        """predict() through the allocation-free entry point (library-held workspace); out, if
        given, is a preallocated contiguous float32 device tensor of x's shape."""
        torch = _torch()
        x = self._planes(x)
        if out is None:
            out = torch.empty_like(x)
        B, N = x.shape[0], x.shape[1]
        _check(_lib.muffin_cnn_predict_noalloc(self._h, ctypes.c_void_p(x.data_ptr()),
                                               _dev_ptr(out, tuple(x.shape), "out"), B, N),
               "muffin_cnn_predict_noalloc")
        torch.cuda.current_stream().synchronize()
        return out

    def loss_grad(self, x, target):
        x, t = self._planes(x), self._planes(target)
        loss = _dbl()
        g = np.empty(self.n_params, dtype=np.float32)
        _check(_lib.muffin_cnn_loss_grad(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         x.shape[0], x.shape[1], ctypes.byref(loss), g.ctypes.data),
               "muffin_cnn_loss_grad")
        return loss.value, g

    def train_step(self, x, target, lr: float) -> float:
        x, t = self._planes(x), self._planes(target)
        loss = _dbl()
        _check(_lib.muffin_cnn_train_step(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                          x.shape[0], x.shape[1], lr, ctypes.byref(loss)), "muffin_cnn_train_step")
        return loss.value

    def layer(self, layer: int, op: int, x, dz=None):
        """Single-layer forward (op 0) or backward (op 1) on FP32 [B][C][N][N] device tensors."""
        torch = _torch()
        x = torch.as_tensor(x, dtype=torch.float32).cuda().contiguous()
        B, N = x.shape[0], x.shape[2]
        cin, cout = (1 if layer == 1 else 32), (1 if layer == 4 else 32)
        if op == 0:
            out = torch.empty((B, cout, N, N), dtype=torch.float32, device="cuda")
            _check(_lib.muffin_cnn_layer(self._h, layer, 0, ctypes.c_void_p(x.data_ptr()), None,
                                         ctypes.c_void_p(out.data_ptr()), None, B, N), "muffin_cnn_layer")
            return out
        dz = torch.as_tensor(dz, dtype=torch.float32).cuda().contiguous()
        out = torch.empty((B, cin, N, N), dtype=torch.float32, device="cuda")
        dp = np.empty(cout * cin * 9 + cout, dtype=np.float32)
        _check(_lib.muffin_cnn_layer(self._h, layer, 1, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(dz.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), dp.ctypes.data, B, N), "muffin_cnn_layer")
        return out, dp


class Batch:
    """Independent cubes of uneven sizes advanced together (muffin_batch_*)."""

    def __init__(self, cubes, J: int, mu_s: float, mu_lambda, iuwt_gen: int = 2, sigma: float = 1.0,
                 rho: float = 1.0, tau=0.0, flags: int = 0, prior: int = PRIOR_IUWT):
        """cubes: list of (dirty, psf) pairs of [L_i][N_i][N_i] arrays; mu_s, mu_lambda and tau may be
        scalars or per-cube sequences (cubes of different mu_s fall into different groups)."""
        torch = _torch()
        n = len(cubes)
        mss = list(mu_s) if np.ndim(mu_s) else [mu_s] * n
        mls = list(mu_lambda) if np.ndim(mu_lambda) else [mu_lambda] * n
        taus = list(tau) if np.ndim(tau) else [tau] * n
        self._keep = []
        ps = (Params * n)()
        dptr = (_vp * n)()
        fptr = (_vp * n)()
        self.shapes = []
        for i, (d, f) in enumerate(cubes):
            d = torch.as_tensor(d, dtype=torch.float32).cuda().contiguous()
            f = torch.as_tensor(f, dtype=torch.float32).cuda().contiguous()
            L, N, _ = d.shape
            self.shapes.append((L, N))
            self._keep += [d, f]
            ps[i] = Params(N=N, L=L, J=J, iuwt_gen=iuwt_gen, penalize_coarse=1, flags=flags, prior=prior, mu_s=mss[i],
                           mu_lambda=mls[i], tau=taus[i], sigma=sigma, rho=rho)
            dptr[i] = d.data_ptr()
            fptr[i] = f.data_ptr()
        h = ctypes.c_void_p()
        _check(_lib.muffin_batch_init(ctypes.byref(h), n, ps, dptr, fptr, 1, _stream_handle()), "muffin_batch_init")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.muffin_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(_lib.muffin_batch_step(self._h, n), "muffin_batch_step")

    def step_timed(self, n: int) -> float:
        ms = _dbl()
        _check(_lib.muffin_batch_step_timed(self._h, n, ctypes.byref(ms)), "muffin_batch_step_timed")
        return ms.value

    def objective(self, cube: int) -> np.ndarray:
        out = (_dbl * 4)()
        _check(_lib.muffin_batch_objective(self._h, cube, out), "muffin_batch_objective")
        return np.array(out[:])

    def info(self, cube: int) -> dict:
        out = (_dbl * 8)()
        _check(_lib.muffin_batch_info(self._h, cube, out), "muffin_batch_info")
        return dict(zip(["tau", "sigma", "rho", "beta", "K2", "Ws2", "delta", "iter"], out[:]))

    def get_x(self, cube: int):
        torch = _torch()
        L, N = self.shapes[cube]
        out = torch.empty((L, N, N), dtype=torch.float32, device="cuda")
        _check(_lib.muffin_batch_get_x(self._h, cube, ctypes.c_void_p(out.data_ptr()), 1), "muffin_batch_get_x")
        torch.cuda.current_stream().synchronize()
        return out

    def set_x(self, cube: int, x0):
        torch = _torch()
        L, N = self.shapes[cube]
        x0 = torch.as_tensor(x0, dtype=torch.float32).cuda().contiguous()
        _check(_lib.muffin_batch_set_x(self._h, cube, _dev_ptr(x0, (L, N, N), "x0"), 1), "muffin_batch_set_x")
        torch.cuda.current_stream().synchronize()

    def warm_input(self, cube: int):
        torch = _torch()
        L, N = self.shapes[cube]
        out = torch.empty((L, N, N), dtype=torch.float32, device="cuda")
        _check(_lib.muffin_batch_warm_input(self._h, cube, ctypes.c_void_p(out.data_ptr()), 1),
               "muffin_batch_warm_input")
        return out

    def snr(self, cube: int, truth) -> float:
        torch = _torch()
        L, N = self.shapes[cube]
        t = torch.as_tensor(truth, dtype=torch.float32).cuda().contiguous()
        out = _dbl()
        _check(_lib.muffin_batch_snr(self._h, cube, _dev_ptr(t, (L, N, N), "truth"), 1, ctypes.byref(out)),
               "muffin_batch_snr")
        return out.value

    def autotune(self, reps: int = 3) -> str:
        buf = ctypes.create_string_buffer(1 << 20)
        _check(_lib.muffin_batch_autotune(self._h, reps, buf, len(buf)), "muffin_batch_autotune")
        return buf.value.decode()


def cnn_params_to_oracle(p: np.ndarray):
    """Split the flat parameter vector into the [(w, b)] list of the network's four layers."""
    p = np.asarray(p, dtype=np.float64)
    shapes = [(32, 1), (32, 32), (32, 32), (1, 32)]
    out, off = [], 0
    for o, c in shapes:
        w = p[off:off + o * c * 9].reshape(o, c, 3, 3)
        off += o * c * 9
        b = p[off:off + o]
        off += o
        out.append((w, b))
    return out


def cnn_params_from_oracle(params) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def uob_filter(n: int) -> np.ndarray:
    """The library's Daubechies scaling filter with n vanishing moments (host computation)."""
    out = (_dbl * (2 * n))()
    _check(_lib.muffin_uob_filter(n, out, 2 * n), "muffin_uob_filter")
    return np.array(out[:])


def set_band_tiles(N: int, j: int, family: int, rows: int, class_groups: int = 1):
    """Record band rows (0: default) and class groups of one IUWT kernel family, process-wide."""
    _check(_lib.muffin_set_band_tiles(N, j, family, rows, class_groups), "muffin_set_band_tiles")


def last_error() -> str:
    return _lib.muffin_last_error().decode(errors="replace")


def debug_oob() -> int:
    """Kernel indices caught out of bounds since the last call (checked builds only)."""
    n = ctypes.c_uint64()
    _check(_lib.muffin_debug_oob(ctypes.byref(n)), "muffin_debug_oob")
    return int(n.value)
