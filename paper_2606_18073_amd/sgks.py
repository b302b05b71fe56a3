"""Python binding of libsgks.so (ctypes).  Argument marshalling only.

PyTorch supplies device memory and the stream; every step of the solver runs in
the library's HIP kernels.  The library must be built (``python -m
paper_2606_18073_amd.build``); a missing library raises at import of the
binding's first use -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libsgks.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sgks.h")

OK = 0
BREAKDOWN = 1
ERRORS = {
    -1: "INVALID_ARG", -2: "SHAPE", -3: "BAD_MU", -4: "SKETCH_SIZE", -5: "CAPACITY",
    -6: "ZERO_RHS", -7: "NONFINITE", -8: "HIP", -9: "DEVICE", -10: "INITIAL_SPACE",
}
F32, F64 = 0, 1
GRADIENT_MAINTAINED, GRADIENT_DIRECT = 0, 1
METHOD_SGKS, METHOD_GKS = 0, 1
SKETCH_SPARSE_SIGN, SKETCH_IDENTITY, SKETCH_SRTT = 0, 1, 2
PHASES = 8
# phase 0: x = W y (direct gradient form) or r = (H W) y - A^T b (maintained);
# phase 2: r = A^T u + mu L^T t (direct) or the new column of H W (maintained)
PHASE_NAMES = ["gemv", "forward_Ax_Lx", "adjoint", "spmv_new_column",
               "qr_append_solve", "gemvt_WTr", "refine_step", "sketch_scatter"]
STATE = {"W": 0, "y": 1, "Q_A": 2, "R_A": 3, "Q_L": 4, "R_L": 5, "d_A": 6, "G": 7, "c_b": 8}


class SgksError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: sgks error {code} ({ERRORS.get(code, 'unknown')})")


class CsrStruct(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("ell", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("zeta", ctypes.c_int32), ("value_dtype", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("qr_passes", ctypes.c_int32),
                ("sketch_mode", ctypes.c_int32), ("lanes_A", ctypes.c_int32),
                ("lanes_At", ctypes.c_int32), ("append_groups", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("gradient_form", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("method", ctypes.c_int32),
                ("keep_history", ctypes.c_int32),
                ("order", ctypes.c_void_p),
                ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class ProblemStruct(ctypes.Structure):
    _fields_ = [("A", CsrStruct), ("L", CsrStruct), ("b", ctypes.c_void_p),
                ("mu", ctypes.c_double), ("sketch_rows", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("order", ctypes.c_void_p)]


MAX_BATCH = 64


_lib = None


def load_library(path=LIB_PATH):
    """Load libsgks.so and declare the prototypes (fails loudly if it is missing)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2606_18073_amd.build`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.sgks_default_options.argtypes = [P(Options)]
    L.sgks_default_options.restype = None
    L.sgks_validate.argtypes = [P(CsrStruct), P(CsrStruct), ctypes.c_void_p, ctypes.c_double,
                                ctypes.c_int32, P(Options)]
    L.sgks_validate.restype = ctypes.c_int
    L.sgks_workspace_bytes.argtypes = [P(CsrStruct), P(CsrStruct), ctypes.c_int32, P(Options)]
    L.sgks_workspace_bytes.restype = ctypes.c_size_t
    L.sgks_create.argtypes = [P(CsrStruct), P(CsrStruct), ctypes.c_void_p, ctypes.c_double,
                              ctypes.c_int32, ctypes.c_uint64, P(Options), P(ctypes.c_void_p)]
    L.sgks_create.restype = ctypes.c_int
    L.sgks_iterate.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.sgks_iterate.restype = ctypes.c_int
    L.sgks_solution.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.sgks_solution.restype = ctypes.c_int
    L.sgks_residual_norm.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_double)]
    L.sgks_residual_norm.restype = ctypes.c_int
    L.sgks_status.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
    L.sgks_status.restype = ctypes.c_int
    L.sgks_backward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                P(ctypes.c_double)]
    L.sgks_backward.restype = ctypes.c_int
    L.sgks_backward_total.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      P(ctypes.c_double), P(ctypes.c_double)]
    L.sgks_backward_total.restype = ctypes.c_int
    L.sgks_copy_state.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_int64]
    L.sgks_copy_state.restype = ctypes.c_int64
    L.sgks_copy_state_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_int64]
    L.sgks_copy_state_noalloc.restype = ctypes.c_int64
    L.sgks_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.sgks_profile_enable.restype = ctypes.c_int
    L.sgks_profile_read.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int64)]
    L.sgks_profile_read.restype = ctypes.c_int
    L.sgks_dim.argtypes = [ctypes.c_void_p]
    L.sgks_dim.restype = ctypes.c_int32
    L.sgks_get_tuning.argtypes = [ctypes.c_void_p, P(ctypes.c_int32)]
    L.sgks_get_tuning.restype = ctypes.c_int
    L.sgks_batch_workspace_bytes.argtypes = [ctypes.c_int32, P(ProblemStruct), P(Options)]
    L.sgks_batch_workspace_bytes.restype = ctypes.c_size_t
    L.sgks_batch_create.argtypes = [ctypes.c_int32, P(ProblemStruct), P(Options),
                                    P(ctypes.c_void_p)]
    L.sgks_batch_create.restype = ctypes.c_int
    L.sgks_batch_iterate.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.sgks_batch_iterate.restype = ctypes.c_int
    L.sgks_batch_get.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.sgks_batch_get.restype = ctypes.c_void_p
    L.sgks_batch_count.argtypes = [ctypes.c_void_p]
    L.sgks_batch_count.restype = ctypes.c_int32
    L.sgks_batch_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.sgks_batch_profile_enable.restype = ctypes.c_int
    L.sgks_batch_profile_read.argtypes = [ctypes.c_void_p, P(ctypes.c_double),
                                          P(ctypes.c_int64)]
    L.sgks_batch_profile_read.restype = ctypes.c_int
    L.sgks_batch_destroy.argtypes = [ctypes.c_void_p]
    L.sgks_batch_destroy.restype = None
    L.sgks_destroy.argtypes = [ctypes.c_void_p]
    L.sgks_destroy.restype = None
    L.sgks_strerror.argtypes = [ctypes.c_int]
    L.sgks_strerror.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = L
    return L


def header_functions(header=HEADER):
    """Names of the functions declared in include/sgks.h."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgks_[a-z_]+)\s*\(", text)))


def default_options():
    o = Options()
    load_library().sgks_default_options(ctypes.byref(o))
    return o


class DeviceCsr:
    """A CSR matrix resident on the GPU (int32 rowptr / colind, f32 or f64 values)."""

    def __init__(self, rowptr, colind, val, shape):
        self.rowptr, self.colind, self.val = rowptr, colind, val
        self.shape = tuple(int(v) for v in shape)

    @classmethod
    def from_scipy(cls, M, dtype="f64", device="cuda"):
        import torch
        vt = torch.float32 if dtype == "f32" else torch.float64
        rp = torch.as_tensor(np.ascontiguousarray(M.indptr, dtype=np.int32), device=device)
        ci = torch.as_tensor(np.ascontiguousarray(M.indices, dtype=np.int32), device=device)
        va = torch.as_tensor(np.ascontiguousarray(M.data), device=device).to(vt)
        return cls(rp, ci, va, M.shape)

    @property
    def nnz(self):
        return int(self.colind.numel())

    def struct(self):
        return CsrStruct(self.shape[0], self.shape[1], self.nnz, self.rowptr.data_ptr(),
                         self.colind.data_ptr(), self.val.data_ptr())


def _check(code, where):
    if code < 0:
        raise SgksError(code, where)
    return code


def make_options(lib, vdt, stream, *, ell=3, max_iters=200, zeta=8, refine_steps=0, qr_passes=2,
                 sketch="sparse_sign", lanes_A=0, lanes_At=0, append_groups=0, graph=False,
                 autotune=False, gradient="maintained", method="sgks", keep_history=False):
    o = Options()
    lib.sgks_default_options(ctypes.byref(o))
    o.ell, o.max_iters, o.zeta, o.value_dtype = ell, max_iters, zeta, vdt
    o.refine_steps, o.qr_passes = refine_steps, qr_passes
    o.sketch_mode = {"sparse_sign": SKETCH_SPARSE_SIGN, "identity": SKETCH_IDENTITY,
                     "srtt": SKETCH_SRTT}[sketch]
    o.lanes_A, o.lanes_At, o.append_groups = lanes_A, lanes_At, append_groups
    o.graph, o.autotune = int(bool(graph)), int(bool(autotune))
    o.gradient_form = GRADIENT_DIRECT if gradient == "direct" else GRADIENT_MAINTAINED
    if method not in ("sgks", "gks"):
        raise ValueError(method)
    o.method = METHOD_GKS if method == "gks" else METHOD_SGKS
    o.keep_history = int(bool(keep_history))
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    return o


class SGKS:
    """One sGKS solve on the GPU: sgks_create / sgks_iterate / sgks_solution / ..."""

    def __init__(self, A: DeviceCsr, L: DeviceCsr, b, mu, s, seed=0, *, ell=3, stream=None,
                 workspace=None, order=None, **opts):
        import torch
        self._lib = load_library()
        self.A, self.L, self.b = A, L, b
        vdt = F32 if A.val.dtype == torch.float32 else F64
        if L.val.dtype != A.val.dtype or b.dtype != A.val.dtype:
            raise TypeError("A, L and b must share one value dtype")
        if stream is None:
            stream = torch.cuda.current_stream(b.device)
        self.stream = stream
        o = make_options(self._lib, vdt, stream, ell=ell, **opts)
        if workspace is not None:
            # caller-owned device memory (e.g. a torch uint8 tensor): no allocation inside
            self._workspace = workspace
            o.workspace = ctypes.c_void_p(workspace.data_ptr())
            o.workspace_bytes = workspace.numel() * workspace.element_size()
        if order is not None:
            # the internal order of the unknowns (device int32, kept alive with the context)
            self._order = order.to(device=b.device, dtype=torch.int32).contiguous()
            o.order = ctypes.c_void_p(self._order.data_ptr())
        self.options = o
        self._owner = None
        self.mu, self.s, self.seed, self.ell = float(mu), int(s), int(seed), int(ell)
        self.n = A.shape[1]
        self.m = A.shape[0]
        self._As, self._Ls = A.struct(), L.struct()
        h = ctypes.c_void_p()
        rc = self._lib.sgks_create(ctypes.byref(self._As), ctypes.byref(self._Ls),
                                   ctypes.c_void_p(b.data_ptr()), float(mu), int(s),
                                   ctypes.c_uint64(seed), ctypes.byref(o), ctypes.byref(h))
        _check(rc, "sgks_create")
        self._h = h

    def iterate(self, k):
        _check(self._lib.sgks_iterate(self._h, int(k)), "sgks_iterate")
        return self

    def solution(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.b.device)
        _check(self._lib.sgks_solution(self._h, ctypes.c_void_p(out.data_ptr())), "sgks_solution")
        return out

    def residual_norm(self):
        t, s = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sgks_residual_norm(self._h, ctypes.byref(t), ctypes.byref(s)),
               "sgks_residual_norm")
        return t.value, s.value

    def status(self):
        it = ctypes.c_int32()
        rc = self._lib.sgks_status(self._h, ctypes.byref(it))
        return rc, it.value

    def backward(self, grad_x):
        import torch
        grad_x = grad_x.to(torch.float64).contiguous()
        gb = torch.empty(self.m, dtype=torch.float64, device=self.b.device)
        gm = ctypes.c_double()
        _check(self._lib.sgks_backward(self._h, ctypes.c_void_p(grad_x.data_ptr()),
                                       ctypes.c_void_p(gb.data_ptr()), ctypes.byref(gm)),
               "sgks_backward")
        return gb, gm.value

    def backward_total(self, grad_x, with_error=False):
        """(d loss/d b, d loss/d mu) through every expansion (sgks_backward_total);
        the solver must be created with keep_history=True.  with_error: also the
        rounding-error estimate d eps kappa(G)^2.  Warns when it exceeds 1e-3."""
        import torch
        grad_x = grad_x.to(torch.float64).contiguous()
        gb = torch.empty(self.m, dtype=torch.float64, device=self.b.device)
        gm, est = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sgks_backward_total(self._h, ctypes.c_void_p(grad_x.data_ptr()),
                                             ctypes.c_void_p(gb.data_ptr()), ctypes.byref(gm),
                                             ctypes.byref(est)),
               "sgks_backward_total")
        if not est.value <= 1e-3:
            import warnings
            warnings.warn(f"sgks_backward_total: estimated relative error {est.value:.1e} "
                          "(d eps kappa(G)^2); the gradient is dominated by rounding",
                          RuntimeWarning, stacklevel=2)
        return (gb, gm.value, est.value) if with_error else (gb, gm.value)

    def profile(self, on=True):
        _check(self._lib.sgks_profile_enable(self._h, 1 if on else 0), "sgks_profile_enable")
        return self

    def profile_read(self):
        """(ms, launches) per phase since the last read (synchronising)."""
        ms = (ctypes.c_double * PHASES)()
        cnt = (ctypes.c_int64 * PHASES)()
        _check(self._lib.sgks_profile_read(self._h, ms, cnt), "sgks_profile_read")
        return list(ms), list(cnt)

    def dim(self):
        return int(self._lib.sgks_dim(self._h))

    def tuning(self):
        """Launch shapes in use: lanes per row of A, L, A^T/L^T; scatter workgroups over
        S_A's and S_L's columns; append groups (1 = compact)."""
        v = (ctypes.c_int32 * 6)()
        _check(self._lib.sgks_get_tuning(self._h, v), "sgks_get_tuning")
        keys = ("lanes_A", "lanes_L", "lanes_At", "scatter_blocks_A", "scatter_blocks_L",
                "append_groups")
        return dict(zip(keys, v))

    def lanes(self):
        """Lanes per CSR row in use: (rows of A, rows of L, rows of A^T / L^T)."""
        t = self.tuning()
        return t["lanes_A"], t["lanes_L"], t["lanes_At"]

    @classmethod
    def _borrowed(cls, owner, handle, A, L, b, mu, s, seed, ell, stream):
        S = cls.__new__(cls)
        S._lib = owner._lib
        S.A, S.L, S.b = A, L, b
        S.stream = stream
        S.options = owner.options
        S.mu, S.s, S.seed, S.ell = float(mu), int(s), int(seed), int(ell)
        S.n, S.m = A.shape[1], A.shape[0]
        S._h = ctypes.c_void_p(handle)
        S._owner = owner   # keeps the batch (which owns the context) alive
        return S

    def state(self, which):
        """Copy one state array to host (numpy, column-major shapes as in sgks.h)."""
        rc, it = self.status()
        d = self.ell + it
        gks = self.options.method == METHOD_GKS
        qa = (self.m if gks else self.s, d)
        ql = (self.L.shape[0] if gks else self.s, d)
        shapes = {"W": (self.n, d), "y": (d,), "Q_A": qa, "R_A": (d, d),
                  "Q_L": ql, "R_L": (d, d), "d_A": (d,), "G": (d, d), "c_b": (self.s,)}
        shp = shapes[which]
        buf = np.zeros(int(np.prod(shp)), dtype=np.float64)
        got = self._lib.sgks_copy_state(self._h, STATE[which],
                                        buf.ctypes.data_as(ctypes.c_void_p), buf.size)
        _check(int(got), "sgks_copy_state")
        return buf.reshape(shp[::-1]).T if len(shp) == 2 else buf

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owner", None) is None:
                self._lib.sgks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SGKSBatch:
    """Batched sGKS (sgks_batch_*): many problems of uneven sizes, one launch per step.

    problems: sequence of (A: DeviceCsr, L: DeviceCsr, b, mu, s, seed); the options
    (ell, max_iters, zeta, refine_steps, qr_passes, sketch, graph, autotune) are
    shared.  problem(i) gives problem i as an SGKS view (solution, residual_norm,
    status, state, backward)."""

    def __init__(self, problems, *, ell=3, stream=None, workspace=None, **opts):
        import torch
        self._lib = load_library()
        problems = list(problems)
        if not 1 <= len(problems) <= MAX_BATCH:
            raise ValueError(f"a batch holds 1..{MAX_BATCH} problems")
        b0 = problems[0][2]
        vdt = F32 if b0.dtype == torch.float32 else F64
        for A, L, b, *_ in problems:
            if A.val.dtype != b0.dtype or L.val.dtype != b0.dtype or b.dtype != b0.dtype:
                raise TypeError("all operators and right-hand sides must share one value dtype")
        if stream is None:
            stream = torch.cuda.current_stream(b0.device)
        self.stream = stream
        self.options = make_options(self._lib, vdt, stream, ell=ell, **opts)
        if workspace is not None:
            # caller-owned device memory for every context and the States array
            self._workspace = workspace
            self.options.workspace = ctypes.c_void_p(workspace.data_ptr())
            self.options.workspace_bytes = workspace.numel() * workspace.element_size()
        self.problems = problems
        self.ell = int(ell)
        arr = _problem_array(problems)
        h = ctypes.c_void_p()
        _check(self._lib.sgks_batch_create(len(problems), arr, ctypes.byref(self.options),
                                           ctypes.byref(h)), "sgks_batch_create")
        self._h = h
        self._views = [None] * len(problems)

    def __len__(self):
        return int(self._lib.sgks_batch_count(self._h))

    def iterate(self, k):
        _check(self._lib.sgks_batch_iterate(self._h, int(k)), "sgks_batch_iterate")
        return self

    def problem(self, i):
        if self._views[i] is None:
            hdl = self._lib.sgks_batch_get(self._h, int(i))
            if not hdl:
                raise IndexError(i)
            A, L, b, mu, s, seed = self.problems[i][:6]
            self._views[i] = SGKS._borrowed(self, hdl, A, L, b, mu, s, seed, self.ell,
                                            self.stream)
        return self._views[i]

    def solutions(self):
        return [self.problem(i).solution() for i in range(len(self.problems))]

    def profile(self, on=True):
        _check(self._lib.sgks_batch_profile_enable(self._h, 1 if on else 0),
               "sgks_batch_profile_enable")
        return self

    def profile_read(self):
        ms = (ctypes.c_double * PHASES)()
        cnt = (ctypes.c_int64 * PHASES)()
        _check(self._lib.sgks_batch_profile_read(self._h, ms, cnt), "sgks_batch_profile_read")
        return list(ms), list(cnt)

    def close(self):
        if getattr(self, "_h", None):
            for v in self._views:
                if v is not None:
                    v._h = None
            self._lib.sgks_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_array(problems):
    """problems: (A, L, b, mu, s, seed[, order]) tuples; order a device int32 tensor."""
    arr = (ProblemStruct * len(problems))()
    for i, pr in enumerate(problems):
        A, L, b, mu, s, seed = pr[:6]
        arr[i].A, arr[i].L = A.struct(), L.struct()
        arr[i].b = b.data_ptr()
        arr[i].mu, arr[i].sketch_rows, arr[i].seed = float(mu), int(s), int(seed)
        if len(pr) > 6 and pr[6] is not None:
            arr[i].order = pr[6].data_ptr()
    return arr


def batch_workspace_bytes(problems, *, ell=3, value_dtype="f32", **opts):
    """Device bytes of a batch of (A, L, b, mu, s, seed) problems (sgks_batch_workspace_bytes)."""
    lib = load_library()

    class _S:
        cuda_stream = 0
    o = make_options(lib, F32 if value_dtype == "f32" else F64, _S(), ell=ell, **opts)
    problems = list(problems)
    return int(lib.sgks_batch_workspace_bytes(len(problems), _problem_array(problems),
                                              ctypes.byref(o)))


def workspace_bytes(A: DeviceCsr, L: DeviceCsr, s, *, ell=3, value_dtype="f32", **opts):
    """Device bytes a context of these shapes and options uses (sgks_workspace_bytes)."""
    lib = load_library()

    class _S:   # the stream is not needed for the size
        cuda_stream = 0
    o = make_options(lib, F32 if value_dtype == "f32" else F64, _S(), ell=ell, **opts)
    As, Ls = A.struct(), L.struct()
    return int(lib.sgks_workspace_bytes(ctypes.byref(As), ctypes.byref(Ls), int(s),
                                        ctypes.byref(o)))


def upload_problem(P, device="cuda"):
    """DeviceCsr A, L and the device b of a workloads.Problem in its storage dtype."""
    import torch
    A = DeviceCsr.from_scipy(P.A, P.dtype, device)
    L = DeviceCsr.from_scipy(P.L, P.dtype, device)
    vt = torch.float32 if P.dtype == "f32" else torch.float64
    b = torch.as_tensor(P.b, device=device).to(vt)
    return A, L, b


def upload_batch(Ps, device="cuda", orders=None):
    """(A, L, b, mu, s, seed[, order]) tuples of device data for a list of
    workloads.Problem; orders: host int32 arrays (or None) of the unknowns' order."""
    import torch
    out = []
    for i, P in enumerate(Ps):
        A, L, b = upload_problem(P, device)
        o = orders[i] if orders is not None else None
        if o is None:
            out.append((A, L, b, P.mu, P.s, P.seed))
        else:
            out.append((A, L, b, P.mu, P.s, P.seed,
                        torch.as_tensor(o, dtype=torch.int32, device=device)))
    return out


def solve_batch(Ps, k=None, device="cuda", **kw):
    """Batched create + k iterations of a list of problems sharing ell, zeta, refinement."""
    k = Ps[0].k if k is None else k
    opts = dict(ell=Ps[0].ell, max_iters=max(k, 1), zeta=Ps[0].zeta,
                refine_steps=Ps[0].refine_steps)
    opts.update(kw)
    B = SGKSBatch(upload_batch(Ps, device), **opts)
    B.iterate(k)
    return B, B.solutions()


def solve_problem(P, k=None, device="cuda", **kw):
    """Create, iterate k (default P.k) times; returns (solver, x as float64 tensor)."""
    A, L, b = upload_problem(P, device)
    k = P.k if k is None else k
    opts = dict(ell=P.ell, max_iters=max(k, 1), zeta=P.zeta, refine_steps=P.refine_steps)
    opts.update(kw)
    S = SGKS(A, L, b, P.mu, P.s, P.seed, **opts)
    S.iterate(k)
    return S, S.solution()


_FUNCTION = None


def _function_class():
    """torch.autograd.Function whose backward is the library's frozen-basis adjoint
    (sgks_backward) or, with adjoint="total", the total derivative through every
    expansion (sgks_backward_total)."""
    global _FUNCTION
    if _FUNCTION is not None:
        return _FUNCTION
    import torch

    class SGKSFunction(torch.autograd.Function):
        """x_k = sGKS(b, mu).  backward: d loss/d b = S_A^T Q_A R_A z and
        d loss/d mu = -(R_L z).(R_L y), z = H^{-1} W^T grad_x, with the basis W and
        the factors Q_A, R_A, R_L of the forward solve held fixed (sgks_backward);
        with adjoint="total" the derivative of the whole map (sgks_backward_total).
        W stays on the device between the two calls."""

        @staticmethod
        def forward(ctx, b, mu, A, L, s, seed, k, opts):
            if opts.get("refine_steps", 0) and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
                raise ValueError("sgks_solve: no backward with refine_steps > 0 (the adjoint "
                                 "is that of the unrefined projected solve)")
            opts = dict(opts)
            adjoint = opts.pop("adjoint", "frozen")
            if adjoint not in ("frozen", "total"):
                raise ValueError(adjoint)
            if adjoint == "total":
                opts["keep_history"] = True
            S = SGKS(A, L, b.detach().contiguous(), float(mu), s, seed, **opts)
            S.iterate(k)
            ctx.solver = S
            ctx.total = adjoint == "total"
            ctx.b_dtype = b.dtype
            ctx.mu_meta = (mu.dtype, mu.device, mu.shape) if torch.is_tensor(mu) else None
            return S.solution()

        @staticmethod
        def backward(ctx, grad_x):
            gb, gmu = (ctx.solver.backward_total(grad_x) if ctx.total
                       else ctx.solver.backward(grad_x))
            gmu_t = None
            if ctx.mu_meta is not None:
                dt, dev, shp = ctx.mu_meta
                gmu_t = torch.full(shp, gmu, dtype=dt, device=dev)
            return gb.to(ctx.b_dtype), gmu_t, None, None, None, None, None, None

    _FUNCTION = SGKSFunction
    return _FUNCTION


def sgks_solve(A: DeviceCsr, L: DeviceCsr, b, mu, s, k, seed=0, **opts):
    """Differentiable x_k (float64 tensor) of k sGKS expansions; b and mu may require grad.
    adjoint="frozen" (default) or "total" selects the backward (see _function_class)."""
    opts.setdefault("max_iters", max(int(k), 1))
    return _function_class().apply(b, mu, A, L, int(s), int(seed), int(k), opts)
