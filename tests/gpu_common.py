"""Helpers shared by the GPU test modules (imported only after the GPU check)."""
import math
import sys

import numpy as np

from oracle import sgks_oracle as O
from workloads import make


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


_cache = {}


def problem(name, scale, seed=0):
    key = (name, scale, seed)
    if key not in _cache:
        _cache[key] = make(name, seed, scale)
    return _cache[key]


def oracle_run(P, k=None, **kw):
    k = P.k if k is None else k
    return O.sgks(P.A, P.L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell,
                  refine_steps=P.refine_steps, **kw)


def backward_error(RA, RL, dA, mu, y):
    """Normwise backward error of y as a least-squares solution of the projected problem
    min || [R_A; sqrt(mu) R_L] y - [d_A; 0] || (eq:projected_sketched_bis):
    ||M^T (M y - f)|| / (||M|| (||M|| ||y|| + 2 ||f||)).  A backward-stable solver keeps it
    at a modest multiple of d * eps whatever the condition number of M."""
    M = np.vstack([RA, math.sqrt(mu) * RL])
    f = np.concatenate([dA, np.zeros(RL.shape[0])])
    nM = np.linalg.norm(M, 2)
    return float(np.linalg.norm(M.T @ (M @ y - f)) /
                 (nM * (nM * np.linalg.norm(y) + 2 * np.linalg.norm(f))))


# backward error allowed for the GPU's projected solve, in units of d * eps
BACKWARD_ERROR_UNITS = 50.0


def check_state_consistency(S, P, tol=1e-9, sketch="sparse_sign"):
    """Relations that hold at any k: the GPU's factors are factors of the GPU's basis."""
    W = S.state("W")
    y = S.state("y")
    QA, RA, QL, RL = S.state("Q_A"), S.state("R_A"), S.state("Q_L"), S.state("R_L")
    dA, cb = S.state("d_A"), S.state("c_b")
    S_A, S_L = O.make_sketches(P.m, P.p, P.s, P.seed, P.zeta, kind=sketch)
    d = W.shape[1]
    # unit columns (normalised basis)
    assert np.allclose(np.linalg.norm(W, axis=0), 1.0, atol=1e-12)
    # c_b = S_A b (integer-exact pattern or selection, FP64 sums)
    cb_ref = S_A @ P.b
    assert rel(cb, cb_ref) < (1e-13 if sketch != "srtt" else 1e-12)
    AW = P.A @ W
    LW = P.L @ W
    SAW = S_A @ AW
    SLW = S_L @ LW
    assert np.linalg.norm(QA @ RA - SAW) <= tol * np.linalg.norm(SAW)
    assert np.linalg.norm(QL @ RL - SLW) <= tol * np.linalg.norm(SLW)
    assert np.linalg.norm(QA.T @ QA - np.eye(d)) < 1e-8
    assert np.linalg.norm(QL.T @ QL - np.eye(d)) < 1e-8
    assert np.allclose(np.triu(RA), RA) and np.allclose(np.triu(RL), RL)
    assert rel(dA, QA.T @ cb_ref) < 1e-10
    # y solves the projected problem built from the GPU factors (before refinement)
    y_ref, Gf = O.projected_solve(RA, RL, dA, P.mu)
    kap = np.linalg.cond(np.vstack([RA, math.sqrt(P.mu) * RL]))
    if P.refine_steps == 0:
        # for any kappa: y is a backward-stable solution of the GPU's own projected problem
        eta = backward_error(RA, RL, dA, P.mu, y)
        eta_ref = backward_error(RA, RL, dA, P.mu, y_ref)
        say(f"  projected solve: kappa {kap:.2e}, backward error {eta:.2e} "
            f"(Householder on the same factors {eta_ref:.2e}, bound "
            f"{BACKWARD_ERROR_UNITS * d * 2.2e-16:.2e})")
        assert eta <= BACKWARD_ERROR_UNITS * d * 2.2e-16, (eta, kap)
        if kap <= KAPPA_TRUSTED:
            assert rel(y, y_ref) <= max(1e-10, 1e-15 * kap * 10), (rel(y, y_ref), kap)
    else:
        # refined y: the oracle's heavy-ball steps from y_ref on the GPU basis.  The
        # library evaluates W^T r(y) as (W^T H W) y - W^T A^T b (the same vector); the
        # spread between those two FP64 evaluations, taken here on the same basis, scales
        # the bound (as the permuted oracle does for the trajectories)
        y_ir = O.refine(P.A, P.L, P.b, P.mu, W, y_ref, Gf, P.s, P.refine_steps)
        y_m = _refine_from_projected_normal_matrix(P, W, AW, LW, y_ref, Gf)
        spread = rel(y_m, y_ir)
        e = rel(y, y_ir)
        say(f"  refined y: kappa {kap:.2e}, vs oracle refinement {e:.2e} (two FP64 forms of "
            f"W^T r differ by {spread:.2e})")
        assert e <= max(1e-9, 1e-15 * kap * 100, 10 * spread), (e, kap, spread)
    return W, y


def _refine_from_projected_normal_matrix(P, W, AW, LW, y0, Gf):
    """The oracle's refinement steps with W^T r(y) evaluated as M y - c, M = W^T H W,
    c = W^T A^T b (FP64, numpy): a second summation order of the same gradient."""
    import scipy.linalg as sla
    M = AW.T @ AW + P.mu * (LW.T @ LW)
    c = W.T @ (P.A.T @ P.b)
    al, be = O.refinement_weights(W.shape[1], P.s)
    y, yp = y0.copy(), y0.copy()
    for _ in range(P.refine_steps):
        dl = sla.solve_triangular(Gf, sla.solve_triangular(Gf, M @ y - c, trans="T"))
        y, yp = y - al * dl + be * (y - yp), y
    return y


def cond_at(ref, P, k):
    """kappa of the stacked projected matrix [R_A; sqrt(mu) R_L] of the oracle after k
    expansions (the factors only grow by appended columns, so the leading block is it)."""
    d = P.ell + k
    Gs = np.vstack([ref.R_A[:d, :d], math.sqrt(P.mu) * ref.R_L[:d, :d]])
    return float(np.linalg.cond(Gs))


# Trajectory parity is asserted while kappa(G_k) <= KAPPA_TRUSTED: two FP64
# evaluations of the same iteration then agree to about kappa * 1e-16 times a
# modest growth factor, below the 1e-5 bound of the FP32-operator path.  Beyond
# it the projected problem is numerically singular in FP64 and only the
# relations that hold for any rounding are checked.
KAPPA_TRUSTED = 1e10


# ----------------------------------------------------------------------------
# oracle runs in worker processes (started before the GPU is touched, see
# conftest.py), so that the long full-size references run beside the GPU tests
# ----------------------------------------------------------------------------

_pool = None


def start_oracle_pool(workers=6):
    global _pool
    if _pool is None:
        import multiprocessing as mp
        _pool = mp.get_context("spawn").Pool(processes=workers)
    return _pool


def _build(spec):
    kind = spec[0]
    if kind == "batch_problem":
        from workloads import generators as gen
        return gen.batch_problem(spec[1])
    return make(kind, spec[2], spec[1])


def _oracle_history(spec, k, checkpoints, permute=None):
    """x after each checkpoint expansion count and kappa(G_k) there.  With permute (a
    seed), the oracle runs on the problem with its unknowns permuted (the columns of A
    and L): the same iteration in exact arithmetic, another rounding order of its sparse
    products; x is mapped back to the original order."""
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits
    P = _build(spec)
    A, L, Pm = P.A, P.L, None
    if permute is not None:
        perm = np.random.default_rng(permute).permutation(P.n)
        Pm = sp.identity(P.n, format="csr")[:, perm]          # x = Pm x'
        A = (P.A @ Pm).tocsr()
        L = (P.L @ Pm).tocsr()
        A.sort_indices()
        L.sort_indices()
    with threadpool_limits(1):
        ref = O.sgks(A, L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell,
                     refine_steps=P.refine_steps, keep_history=True)
    back = (lambda v: Pm @ v) if Pm is not None else (lambda v: v)
    hist = {kk: back(ref.x_hist[kk]) for kk in checkpoints if kk <= ref.iters}
    kap = {kk: cond_at(ref, P, kk) for kk in checkpoints if kk <= ref.iters}
    return hist, kap, ref.iters, ref.status


def wait_ref(res, what=""):
    """The result of an oracle run, printing a line every 20 s while it is still running."""
    import time
    t0 = time.time()
    if hasattr(res, "ready"):
        while not res.ready():
            res.wait(20)
            if not res.ready():
                say(f"  waiting for the oracle {what} ({time.time() - t0:.0f} s)")
    return res.get()


class _Now:
    def __init__(self, fn, args):
        self.fn, self.args, self.val = fn, args, None

    def get(self, timeout=None):
        if self.val is None:
            self.val = self.fn(*self.args)
        return self.val


def oracle_history_async(spec, k, checkpoints, permute=None):
    """Oracle trajectory of a workload ((name, scale, seed) or ("batch_problem", i)) at the
    checkpoints: computed in a worker process when the pool runs, else on .get()."""
    args = (spec, k, tuple(checkpoints), permute)
    if _pool is not None:
        return _pool.apply_async(_oracle_history, args)
    return _Now(_oracle_history, args)
