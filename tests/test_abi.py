"""The C-ABI library loads and exports every entry point include/muffin.h declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muffin.h")
LIB = os.path.join(ROOT, "paper_1602_08847_amd", "libmuffin.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(muffin_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_header_entry_points():
    from paper_1602_08847_amd import muffin
    assert sorted(muffin.EXPORTS) == declared()


def test_strerror_codes():
    from paper_1602_08847_amd import muffin
    lib = muffin._lib
    assert lib.muffin_strerror(0) == b"ok"
    for code in (-1, -2, -3, -4, -5, -6):
        assert lib.muffin_strerror(code) not in (b"ok", b"unknown error")
    assert lib.muffin_strerror(-99) == b"unknown error"


def test_null_arguments_are_rejected_without_a_gpu():
    """Argument checks run before any device call."""
    from paper_1602_08847_amd import muffin
    lib = muffin._lib
    assert lib.muffin_init(None, None, None, None, 0, None) == muffin.EINVAL
    h = ctypes.c_void_p()
    assert lib.muffin_init(ctypes.byref(h), None, None, None, 0, None) == muffin.EINVAL
    p = muffin.Params(N=100, L=4, J=2, iuwt_gen=2, penalize_coarse=1, mu_s=0.1, mu_lambda=0.1,
                      tau=0.0, sigma=1.0, rho=1.0)
    assert lib.muffin_init(ctypes.byref(h), ctypes.byref(p), None, None, 0, None) == muffin.EINVAL
    assert b"N must be" in lib.muffin_last_error()
    for bad in (dict(N=64, L=0), dict(N=64, L=4, J=0), dict(N=64, L=4, J=2, iuwt_gen=3),
                dict(N=64, L=4, J=2, iuwt_gen=2, sigma=-1.0), dict(N=64, L=4, J=2, iuwt_gen=2, mu_s=-1)):
        q = muffin.Params(**{**dict(N=64, L=4, J=2, iuwt_gen=2, penalize_coarse=1, mu_s=0.1,
                                    mu_lambda=0.1, tau=0.0, sigma=1.0, rho=1.0), **bad})
        assert lib.muffin_init(ctypes.byref(h), ctypes.byref(q), None, None, 0, None) == muffin.EINVAL
    out = (ctypes.c_double * 8)()
    assert lib.muffin_step(None, 1) == muffin.EINVAL
    assert lib.muffin_objective(None, out) == muffin.EINVAL
    assert lib.muffin_info(None, out) == muffin.EINVAL
    assert lib.muffin_get_x(None, None, 0) == muffin.EINVAL
    assert lib.muffin_apply_op(None, 1, None, None) == muffin.EINVAL
    lib.muffin_free(None)


def test_library_daubechies_filters_match_the_oracle_and_closed_forms():
    """The library builds its union-of-bases filters on the host (Durand-Kerner roots in long double),
    independently of the oracle (numpy companion-matrix roots): both agree, and with the published
    Haar and db2 filters."""
    import numpy as np
    from oracle import uob
    from paper_1602_08847_amd import muffin
    for n in range(1, 9):
        np.testing.assert_allclose(muffin.uob_filter(n), uob.daubechies_lowpass(n), atol=1e-12)
    s3 = np.sqrt(3.0)
    np.testing.assert_allclose(muffin.uob_filter(2), np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0)),
                               atol=1e-15)
    np.testing.assert_allclose(muffin.uob_filter(1), [2 ** -0.5, 2 ** -0.5], atol=1e-16)
    h = (ctypes.c_double * 4)()
    assert muffin._lib.muffin_uob_filter(9, h, 4) == muffin.EINVAL
    assert muffin._lib.muffin_uob_filter(3, h, 4) == muffin.EINVAL  # buffer shorter than 6 taps


def test_band_tiles_setter_validates_without_a_gpu():
    """muffin_set_band_tiles only records launch choices: it is checked on the host."""
    from paper_1602_08847_amd import muffin
    bad = [(64, 2, muffin.FAMILY_PAIR_ANALYSIS, 24, 1),   # rows must divide N
           (64, 2, muffin.FAMILY_PAIR_ANALYSIS, 16, 8),   # more groups than classes (2^2)
           (64, 3, muffin.FAMILY_PAIR_ADJOINT, 16, 3),    # not a power of two
           (64, 4, muffin.FAMILY_TRIPLE_ANALYSIS, 16, 16),  # more than 8 groups
           (64, 3, 4, 16, 1),                             # no such family
           (2048, 3, muffin.FAMILY_PAIR_ANALYSIS, 16, 1)]  # N beyond the kernels' limit
    for args in bad:
        assert muffin._lib.muffin_set_band_tiles(*args) == -1, args
    # accepted, then back to the defaults
    muffin.set_band_tiles(64, 3, muffin.FAMILY_PAIR_ADJOINT, 32, 8)
    muffin.set_band_tiles(64, 3, muffin.FAMILY_FUSED_PAIR, 64, 4)
    for f in (muffin.FAMILY_PAIR_ADJOINT, muffin.FAMILY_FUSED_PAIR):
        muffin.set_band_tiles(64, 3, f, 0, 0)
