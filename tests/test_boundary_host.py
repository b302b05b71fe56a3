"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function declared in include/sgks.h, and validates arguments without touching
the device."""
import ctypes

import pytest

from paper_2606_18073_amd import sgks as G


@pytest.fixture(scope="module")
def lib():
    return G.load_library()


def test_exports_every_declared_symbol(lib):
    names = G.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_default_options(lib):
    o = G.default_options()
    assert (o.ell, o.max_iters, o.zeta, o.qr_passes, o.value_dtype) == (3, 200, 8, 2, G.F64)
    assert o.sketch_mode == G.SKETCH_SPARSE_SIGN and o.refine_steps == 0


def _csr(rows, cols, nnz):
    # non-null fake pointers: validation never dereferences them
    return G.CsrStruct(rows, cols, nnz, 0x1000, 0x2000, 0x3000)


def _v(lib, A, L, b=0x4000, mu=1e-2, s=400, **kw):
    o = G.default_options()
    o.max_iters = kw.pop("max_iters", 100)
    for k, v in kw.items():
        setattr(o, k, v)
    return lib.sgks_validate(ctypes.byref(A), ctypes.byref(L), ctypes.c_void_p(b), mu, s,
                             ctypes.byref(o))


def test_validation_codes(lib):
    A, L = _csr(100, 80, 500), _csr(160, 80, 320)
    assert _v(lib, A, L) == 0
    assert _v(lib, A, _csr(160, 81, 320)) == -2                 # A.cols != L.cols
    assert _v(lib, A, L, mu=0.0) == -3
    assert _v(lib, A, L, mu=-1.0) == -3
    assert _v(lib, A, L, mu=float("nan")) == -3
    assert _v(lib, A, L, mu=float("inf")) == -3
    assert _v(lib, A, L, s=50) == -4                            # s < ell + max_iters
    assert _v(lib, A, L, s=4096) == -4                          # above the LDS bin limit
    assert _v(lib, A, L, s=6, max_iters=0, zeta=8) == -4        # zeta > s
    assert _v(lib, A, L, zeta=3) == -1
    assert _v(lib, A, L, qr_passes=3) == -1
    assert _v(lib, A, L, value_dtype=7) == -1
    assert _v(lib, A, L, lanes_A=3) == -1
    assert _v(lib, A, L, max_iters=600, s=2000) == -5           # capacity above 512 columns
    assert _v(lib, A, L, b=0) == -1                             # null b
    assert _v(lib, _csr(0, 80, 0), L) == -2                     # empty A
    bad = G.CsrStruct(100, 80, 500, 0, 0x2000, 0x3000)
    assert _v(lib, bad, L) == -1                                # null rowptr
    # identity sketch needs s >= max(m, p)
    assert _v(lib, A, L, s=150, sketch_mode=G.SKETCH_IDENTITY) == -4
    assert _v(lib, A, L, s=160, sketch_mode=G.SKETCH_IDENTITY) == 0


def test_strerror(lib):
    for code in [0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10]:
        assert lib.sgks_strerror(code)
    assert lib.sgks_strerror(-1234) == b"unknown error"


def test_null_handles_are_rejected(lib):
    assert lib.sgks_iterate(None, 1) == -1
    assert lib.sgks_solution(None, None) == -1
    assert lib.sgks_dim(None) == 0
    lib.sgks_destroy(None)
