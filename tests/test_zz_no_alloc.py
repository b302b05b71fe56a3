"""The allocation-free variant of sgks_copy_state (through the C ABI): the basis W
staged through the library's static device array gives the same bits as
sgks_copy_state, on two calls in a row (the second with a smaller problem, so
stale staging contents from the first would show), and a basis whose single
column exceeds the array is refused with SGKS_ERR_CAPACITY."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_common import problem, say  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402

SCRATCH = 16 << 20   # SGKS_NOALLOC_SCRATCH_BYTES


def _copy(S, fn):
    rc, it = S.status()
    d = S.ell + it
    buf = np.full(S.n * d, np.nan)
    got = fn(S._h, 0, buf.ctypes.data_as(ctypes.c_void_p), buf.size)
    return int(got), buf


def test_noalloc_copy_matches_copy_state_on_two_calls():
    lib = G.load_library()
    big = problem("deblur2d", "full")      # W: 65,536 x 33 doubles = 17.3 MB, two chunks
    small = problem("deblur2d", "small")   # W: 1,600 x 15 doubles
    for P, k in ((big, 30), (small, 12)):
        say("case noalloc copy", P.name, P.n, "k", k)
        S, _ = G.solve_problem(P, k=k)
        assert 8 * P.n * (P.ell + k) > SCRATCH or P is small
        n1, ref = _copy(S, lib.sgks_copy_state)
        n2, got = _copy(S, lib.sgks_copy_state_noalloc)
        assert n1 == n2 == P.n * (P.ell + k)
        assert np.array_equal(ref, got)
        # the other pieces go through sgks_copy_state unchanged
        y1 = np.zeros(P.ell + k)
        y2 = np.zeros(P.ell + k)
        assert lib.sgks_copy_state(S._h, 1, y1.ctypes.data_as(ctypes.c_void_p), y1.size) == y1.size
        assert lib.sgks_copy_state_noalloc(S._h, 1, y2.ctypes.data_as(ctypes.c_void_p),
                                           y2.size) == y2.size
        assert np.array_equal(y1, y2)
        # too small a destination is refused before any copy
        buf = np.zeros(P.n)
        assert lib.sgks_copy_state_noalloc(S._h, 0, buf.ctypes.data_as(ctypes.c_void_p),
                                           buf.size) == -1
        S.close()


def test_noalloc_copy_refuses_a_column_larger_than_the_array():
    import scipy.sparse as sp
    lib = G.load_library()
    n = SCRATCH // 8 + 1024                # one column of W exceeds the staging array
    I = sp.identity(n, format="csr")
    I.indices = I.indices.astype(np.int32)
    I.indptr = I.indptr.astype(np.int32)
    A = G.DeviceCsr.from_scipy(I, "f32")
    b = torch.linspace(1.0, 2.0, n, device="cuda", dtype=torch.float32)
    say("case noalloc capacity", n)
    S = G.SGKS(A, A, b, 0.5, 8, 0, ell=1, max_iters=0)
    buf = np.zeros(n)
    assert lib.sgks_copy_state_noalloc(S._h, 0, buf.ctypes.data_as(ctypes.c_void_p),
                                       buf.size) == -5
    assert lib.sgks_copy_state(S._h, 0, buf.ctypes.data_as(ctypes.c_void_p), buf.size) == n
    assert np.allclose(buf, torch.linspace(1.0, 2.0, n, dtype=torch.float64).numpy() /
                       np.linalg.norm(torch.linspace(1.0, 2.0, n, dtype=torch.float64).numpy()),
                       rtol=1e-6)
    S.close()
