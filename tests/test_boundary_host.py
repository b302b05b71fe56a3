"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function declared in include/sgks.h, and validates arguments without touching
the device."""
import ctypes
import os
import subprocess

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
    assert (o.graph, o.autotune, o.lanes_A, o.lanes_At, o.append_groups) == (0, 0, 0, 0, 0)
    assert o.gradient_form == G.GRADIENT_MAINTAINED


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
    assert _v(lib, A, L, s=16385) == -4                         # above the largest sketch
    assert _v(lib, A, L, s=16384) == 0
    assert _v(lib, A, L, s=1025) == 0                           # the multi-workgroup append
    assert _v(lib, A, L, method=2) == -1
    assert _v(lib, A, L, method=G.METHOD_GKS) == 0               # no sketch: s not used
    assert _v(lib, A, L, method=G.METHOD_GKS, refine_steps=1) == -1
    assert _v(lib, A, L, s=6, max_iters=0, zeta=8) == -4        # zeta > s
    assert _v(lib, A, L, zeta=3) == -1
    assert _v(lib, A, L, qr_passes=3) == -1
    assert _v(lib, A, L, value_dtype=7) == -1
    assert _v(lib, A, L, lanes_A=3) == -1
    assert _v(lib, A, L, graph=2) == -1
    assert _v(lib, A, L, autotune=-1) == -1
    assert _v(lib, A, L, gradient_form=2) == -1
    assert _v(lib, A, L, max_iters=600, s=2000) == -5           # capacity above 512 columns
    assert _v(lib, A, L, b=0) == -1                             # null b
    assert _v(lib, _csr(0, 80, 0), L) == -2                     # empty A
    bad = G.CsrStruct(100, 80, 500, 0, 0x2000, 0x3000)
    assert _v(lib, bad, L) == -1                                # null rowptr
    # identity sketch needs s >= max(m, p)
    assert _v(lib, A, L, s=150, sketch_mode=G.SKETCH_IDENTITY) == -4
    assert _v(lib, A, L, s=160, sketch_mode=G.SKETCH_IDENTITY) == 0
    # the total-derivative adjoint's history: sGKS, maintained form, no refinement
    assert _v(lib, A, L, keep_history=1) == 0
    assert _v(lib, A, L, keep_history=2) == -1
    assert _v(lib, A, L, keep_history=1, refine_steps=1) == -1
    assert _v(lib, A, L, keep_history=1, gradient_form=G.GRADIENT_DIRECT) == -1
    assert _v(lib, A, L, keep_history=1, method=G.METHOD_GKS) == -1


def test_strerror(lib):
    for code in [0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10]:
        assert lib.sgks_strerror(code)
    assert lib.sgks_strerror(-1234) == b"unknown error"


def test_null_handles_are_rejected(lib):
    assert lib.sgks_iterate(None, 1) == -1
    assert lib.sgks_solution(None, None) == -1
    assert lib.sgks_dim(None) == 0
    lib.sgks_destroy(None)


def test_null_batch_handles_are_rejected(lib):
    assert lib.sgks_batch_iterate(None, 1) == -1
    assert lib.sgks_batch_get(None, 0) is None
    assert lib.sgks_batch_count(None) == 0
    assert lib.sgks_batch_profile_enable(None, 1) == -1
    assert lib.sgks_batch_profile_read(None, None, None) == -1
    assert lib.sgks_get_tuning(None, None) == -1
    lib.sgks_batch_destroy(None)


def test_batch_argument_checks_before_device_work(lib):
    out = ctypes.c_void_p()
    probs = (G.ProblemStruct * 2)()
    for p in probs:
        p.A, p.L = _csr(100, 80, 500), _csr(160, 80, 320)
        p.b, p.mu, p.sketch_rows, p.seed = 0x4000, 1e-2, 400, 0
    o = G.default_options()
    o.max_iters = 100
    assert lib.sgks_batch_create(0, probs, ctypes.byref(o), ctypes.byref(out)) == -1
    assert lib.sgks_batch_create(G.MAX_BATCH + 1, probs, ctypes.byref(o),
                                 ctypes.byref(out)) == -1
    assert lib.sgks_batch_create(2, None, ctypes.byref(o), ctypes.byref(out)) == -1
    o.lanes_A = 4          # per-problem choices are not shared options
    assert lib.sgks_batch_create(2, probs, ctypes.byref(o), ctypes.byref(out)) == -1
    o.lanes_A = 0
    probs[1].mu = -1.0     # each problem is validated before any set-up
    assert lib.sgks_batch_create(2, probs, ctypes.byref(o), ctypes.byref(out)) == -3
    probs[1].mu = 1e-2
    probs[1].sketch_rows = 50
    assert lib.sgks_batch_create(2, probs, ctypes.byref(o), ctypes.byref(out)) == -4
    assert out.value is None


LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "sgks.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu\n", sizeof(sgks_options), offsetof(sgks_options, graph),
           offsetof(sgks_options, stream), sizeof(sgks_problem), offsetof(sgks_problem, b),
           offsetof(sgks_problem, seed));
    printf("%zu %zu\n", sizeof(sgks_csr), offsetof(sgks_problem, sketch_rows));
    printf("%zu %zu\n", offsetof(sgks_options, workspace), offsetof(sgks_options, workspace_bytes));
    printf("%zu %zu\n", offsetof(sgks_options, method), offsetof(sgks_options, order));
    printf("%zu\n", offsetof(sgks_problem, order));
    printf("%zu\n", offsetof(sgks_options, keep_history));
    return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of sgks_options, sgks_csr and sgks_problem have the C layout."""
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = [int(v) for v in out]
    O, P = G.Options, G.ProblemStruct
    assert got == [ctypes.sizeof(O), O.graph.offset, O.stream.offset, ctypes.sizeof(P),
                   P.b.offset, P.seed.offset, ctypes.sizeof(G.CsrStruct), P.sketch_rows.offset,
                   O.workspace.offset, O.workspace_bytes.offset, O.method.offset,
                   O.order.offset, P.order.offset, O.keep_history.offset]


def test_workspace_bytes_host_only(lib):
    """Size of a context's device memory without touching the device."""
    A, L = _csr(100, 80, 500), _csr(160, 80, 320)

    def ws(s=400, **kw):
        o = G.default_options()
        o.max_iters = kw.pop("max_iters", 100)
        for k, v in kw.items():
            setattr(o, k, v)
        return lib.sgks_workspace_bytes(ctypes.byref(A), ctypes.byref(L), s, ctypes.byref(o))

    base = ws()
    assert base > 0
    # W (and HW) grow with the capacity: 8 bytes per unknown per column each
    assert ws(max_iters=150) - base >= 2 * 8 * 80 * 50
    assert ws(gradient_form=G.GRADIENT_DIRECT) < base       # no HW
    assert ws(s=50) == 0                                     # invalid: s < ell + max_iters
    assert ws(zeta=3) == 0
    # keep_history: at least E (n x max_iters) and the y and u histories
    assert ws(keep_history=1) - base >= 8 * 80 * 100 + 2 * 8 * 103 * 104


def test_batch_workspace_bytes_and_checks_before_device_work(lib):
    """The batch workspace holds each context's arena (256-byte aligned) and the States
    array; too small or misaligned workspaces are refused before any device work."""
    probs = (G.ProblemStruct * 2)()
    sizes = []
    o = G.default_options()
    o.max_iters = 100
    for i, p in enumerate(probs):
        p.A, p.L = _csr(100 + 20 * i, 80, 500), _csr(160, 80, 320)
        p.b, p.mu, p.sketch_rows, p.seed = 0x4000, 1e-2, 400, i
        sizes.append(lib.sgks_workspace_bytes(ctypes.byref(p.A), ctypes.byref(p.L), 400,
                                              ctypes.byref(o)))
    total = lib.sgks_batch_workspace_bytes(2, probs, ctypes.byref(o))
    up = lambda v: (v + 255) // 256 * 256
    assert all(v > 0 for v in sizes)
    assert total > sum(up(v) for v in sizes)
    assert total - sum(up(v) for v in sizes) <= up(2 * 4096)     # the States array
    assert lib.sgks_batch_workspace_bytes(0, probs, ctypes.byref(o)) == 0
    probs[1].sketch_rows = 50
    assert lib.sgks_batch_workspace_bytes(2, probs, ctypes.byref(o)) == 0
    probs[1].sketch_rows = 400
    out = ctypes.c_void_p()
    o.workspace, o.workspace_bytes = 0x10000, total - 1      # too small
    assert lib.sgks_batch_create(2, probs, ctypes.byref(o), ctypes.byref(out)) == -1
    o.workspace, o.workspace_bytes = 0x10008, total + 256    # misaligned
    assert lib.sgks_batch_create(2, probs, ctypes.byref(o), ctypes.byref(out)) == -1
    assert out.value is None
