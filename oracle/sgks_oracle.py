"""FP64 CPU oracle of GKS and sketched GKS (sGKS).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the HIP
path (no kernels, headers, helpers or constants); both sides take their inputs
from the seeded generators in ``workloads`` only.

Everything here is plain numpy / scipy in float64, written to be read against
the paper (Palitta & Pasha, "A Sketched Generalized Krylov Subspace Method for
Large-Scale Regularization"):

  * general-form Tikhonov problem, eq:tik
  * GKS, Alg. 1 (Sec. 2.1), with the rank-one QR update eq:updqr, the
    right-hand-side update eq:dA_update, the projector eq:single_mgs and the
    loss ratio eq:loss_criterion
  * sGKS, Alg. 2 (Sec. 3): no reorthogonalisation, sketch-and-solve projected
    problem eq:projected_sketched_bis with two independent sketches S_A, S_L
  * iterative refinement of the projected solve (end of Sec. 3.1; Sec. 4.3)
  * a frozen-basis adjoint of the final projected solve, and the total
    derivative of x_k through every expansion and the initial basis (reverse
    sweep); neither is in the paper
  * the sparse-sign embedding (the paper uses an SRTT, eq:sketching_trig, and
    states the method is independent of the embedding, Sec. 2.2)

Library primitives used as single steps: scipy CSR products, numpy.linalg.qr
(Householder), scipy.linalg.solve_triangular, numpy.linalg.solve/svd.

Readings where the paper is silent (each also listed in the design notes):
  * S_A is s x m and S_L is s x p (the text's "s_A x n" is a dimension slip),
    s_A = s_L = s.
  * W_0 = V_0 = CGS2-orthonormal basis of K_ell(A^T A, A^T b), ell = 3.
  * Appended sGKS columns are r / ||r|| (a column scaling; x_k unchanged in
    exact arithmetic, cf. the change of variables in the proof of Prop. 1).
  * The QR column append projects twice (CGS2) unless qr_passes = 1, which is
    the single projection written in eq:updqr.
  * "k iterations" = k expansions; the last projected problem has ell + k columns.
  * Breakdown: stop when ||r|| <= 1e-14 ||A^T b||, or when the new column of
    [R_A; sqrt(mu) R_L] keeps at most 1e-14 of its norm after projection on
    the previous columns (the expansion adds nothing to the projected problem);
    the column is then not appended.
  * Iterative refinement (the paper defers to FOSSILS): sketch-preconditioned
    heavy-ball steps on the unsketched projected normal equations,
        delta_i = (G^T G)^{-1} W^T r(y_i),
        y_{i+1} = y_i - alpha delta_i + beta (y_i - y_{i-1}),  y_{-1} = y_0,
    with G the R factor of [R_A; sqrt(mu) R_L], eta = sqrt(d/s),
    alpha = (1 - eta^2)^2, beta = eta^2.  Fixed point: the unsketched projected
    solution y_sGKS0 of eq:sGKS_noSASL.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

STATUS_OK = 0
STATUS_BREAKDOWN = 1

# ----------------------------------------------------------------------------
# Sparse-sign embedding.
#
# The paper never defines it (it uses an SRTT).  Definition used here:
# column j of S (h columns, s rows) has zeta nonzeros +-1/sqrt(zeta) in
# distinct rows.  Rows and signs come from SplitMix64 (Steele, Lea & Flood,
# "Fast splittable pseudorandom number generators", OOPSLA 2014):
#   gamma = 0x9E3779B97F4A7C15
#   mix64(z): z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
#             z *= 0x94D049BB133111EB; z ^= z>>31            (mod 2^64)
#   key(stream, j) = mix64(seed + gamma * (2 j + stream + 1))
#   draw c of column j: z_c = mix64(key + gamma * (c + 1)), c = 0, 1, ...
#   row = ((z >> 32) * s) >> 32, sign = -1 if (z & 1) else +1
# Slot t takes the next draws until the row is new for the column.
# Stream 0 builds S_A, stream 1 builds S_L.
# ----------------------------------------------------------------------------

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    """SplitMix64 finaliser on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * _M1
        z = z ^ (z >> np.uint64(27))
        z = z * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def sparse_sign_pattern(h, s, zeta, seed, stream):
    """(rows, signs), each h x zeta: the nonzero rows and signs of every column."""
    if zeta > s:
        raise ValueError("zeta must not exceed s")
    j = np.arange(h, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = mix64(np.uint64(seed) + GAMMA * (np.uint64(2) * j + np.uint64(stream + 1)))
    rows = np.full((h, zeta), -1, dtype=np.int64)
    signs = np.zeros((h, zeta), dtype=np.int64)
    counter = np.zeros(h, dtype=np.uint64)
    for t in range(zeta):
        pending = np.arange(h)
        while pending.size:
            with np.errstate(over="ignore"):
                z = mix64(key[pending] + GAMMA * (counter[pending] + np.uint64(1)))
            counter[pending] += np.uint64(1)
            row = ((z >> np.uint64(32)) * np.uint64(s)) >> np.uint64(32)
            row = row.astype(np.int64)
            dup = (rows[pending, :t] == row[:, None]).any(axis=1)
            acc = pending[~dup]
            rows[acc, t] = row[~dup]
            signs[acc, t] = np.where((z[~dup] & np.uint64(1)) == 1, -1, 1)
            pending = pending[dup]
    return rows, signs


def sparse_sign_matrix(h, s, zeta, seed, stream):
    """The s x h sparse-sign embedding as a CSR matrix with entries +-1/sqrt(zeta)."""
    rows, signs = sparse_sign_pattern(h, s, zeta, seed, stream)
    cols = np.repeat(np.arange(h), zeta)
    vals = signs.ravel() / math.sqrt(zeta)
    return sp.csr_matrix((vals, (rows.ravel(), cols)), shape=(s, h))


# ----------------------------------------------------------------------------
# Subsampled randomised trigonometric transform (SRTT, eq:sketching_trig):
#   S = sqrt(h / s) D F E  (s x h)
# E: diagonal of Rademacher signs, F: the orthonormal DCT-II of length h,
#   F[k, i] = c_k cos(pi k (2 i + 1) / (2 h)),  c_0 = sqrt(1/h), c_k = sqrt(2/h),
# D: s distinct rows of the identity.  The paper does not fix how E and D are
# drawn; here both come from SplitMix64 (same finaliser and gamma as above):
#   sign key  ks = mix64(seed + gamma (stream + 3)),  E_i = -1 if mix64(ks + gamma (i + 1)) is odd
#   row key   kr = mix64(seed + gamma (stream + 1)),  draw c: z_c = mix64(kr + gamma (c + 1)),
#             row = ((z_c >> 32) h) >> 32, a row already drawn is skipped, until s rows;
#   output j of S is frequency rows[j] (draw order).
# ----------------------------------------------------------------------------

def srtt_signs(h, seed, stream):
    """The h Rademacher signs of E (+1 / -1)."""
    with np.errstate(over="ignore"):
        ks = mix64(np.uint64(seed) + GAMMA * np.uint64(stream + 3))
        z = mix64(ks + GAMMA * (np.arange(h, dtype=np.uint64) + np.uint64(1)))
    return np.where((z & np.uint64(1)) == 1, -1.0, 1.0)


def srtt_rows(h, s, seed, stream):
    """The s distinct frequencies D selects, in draw order."""
    if s > h:
        raise ValueError("an SRTT selects at most h rows")
    with np.errstate(over="ignore"):
        kr = mix64(np.uint64(seed) + GAMMA * np.uint64(stream + 1))
    rows, seen, c = [], set(), 0
    while len(rows) < s:
        with np.errstate(over="ignore"):
            z = int(mix64(kr + GAMMA * np.uint64(c + 1)))
        c += 1
        r = ((z >> 32) * h) >> 32
        if r not in seen:
            seen.add(r)
            rows.append(r)
    return np.array(rows, dtype=np.int64)


class SRTT:
    """S = sqrt(h/s) D F E applied with the fast DCT-II (scipy.fft, orthonormal) as one
    step; S @ v for a vector or the columns of a matrix, S.T @ w for its transpose."""

    def __init__(self, h, s, seed, stream):
        self.h, self.s = h, s
        self.E = srtt_signs(h, seed, stream)
        self.rows = srtt_rows(h, s, seed, stream)
        self.scale = math.sqrt(h / s)
        self.shape = (s, h)

    def __matmul__(self, v):
        import scipy.fft as fft
        v = np.asarray(v, dtype=np.float64)
        ev = self.E[:, None] * v if v.ndim == 2 else self.E * v
        return self.scale * fft.dct(ev, type=2, norm="ortho", axis=0)[self.rows]

    @property
    def T(self):
        return _SRTTTranspose(self)


class _SRTTTranspose:
    def __init__(self, S):
        self.S = S
        self.shape = (S.h, S.s)

    def __matmul__(self, w):
        import scipy.fft as fft
        S = self.S
        w = np.asarray(w, dtype=np.float64)
        full = np.zeros((S.h,) + w.shape[1:])
        full[S.rows] = w
        out = fft.idct(full, type=2, norm="ortho", axis=0)     # F^T, F orthonormal
        return S.scale * (S.E[:, None] * out if w.ndim == 2 else S.E * out)


# ----------------------------------------------------------------------------
# Building blocks
# ----------------------------------------------------------------------------

def gradient(A, L, b, mu, x):
    """r = A^T (A x - b) + mu L^T (L x)   (eq: gradient, with x = W_k y_k)."""
    return A.T @ (A @ x - b) + mu * (L.T @ (L @ x))


def qr_append(Q, R, a, passes=2):
    """Append column a to the thin QR factorisation Q R (eq:updqr).

    p = Q^T a, a_perp = a - Q p (repeated `passes` times, the projections
    accumulating into p), rho = ||a_perp||, q = a_perp / rho,
    R <- [[R, p], [0, rho]], Q <- [Q, q].
    If rho <= 1e-14 ||a|| the new direction is numerically absent: q = 0,
    rho = 0 and the returned flag is True."""
    d = R.shape[0]
    p = np.zeros(d)
    v = a.astype(np.float64).copy()
    for _ in range(passes):
        c = Q.T @ v
        v = v - Q @ c
        p = p + c
    rho = float(np.linalg.norm(v))
    degenerate = rho <= 1e-14 * float(np.linalg.norm(a))
    if degenerate:
        q = np.zeros_like(v)
        rho = 0.0
    else:
        q = v / rho
    R2 = np.zeros((d + 1, d + 1))
    R2[:d, :d] = R
    R2[:d, d] = p
    R2[d, d] = rho
    Q2 = np.concatenate([Q, q[:, None]], axis=1)
    return Q2, R2, degenerate


def projected_solve(R_A, R_L, d_A, mu):
    """y = argmin || [R_A; sqrt(mu) R_L] y - [d_A; 0] ||  (eq:projected_sketched_bis).

    Householder QR of the stacked 2d x d matrix.  Returns (y, G) with G the
    triangular factor (used by the refinement and the adjoint)."""
    d = R_A.shape[0]
    M = np.vstack([R_A, math.sqrt(mu) * R_L])
    f = np.concatenate([d_A, np.zeros(d)])
    U, G = np.linalg.qr(M, mode="reduced")
    y = sla.solve_triangular(G, U.T @ f, lower=False)
    return y, G


def gram_solve(G, g):
    """delta = (G^T G)^{-1} g by two triangular solves."""
    t = sla.solve_triangular(G, g, trans="T", lower=False)
    return sla.solve_triangular(G, t, lower=False)


class DegenerateInitialSpace(ValueError):
    """K_ell(A^T A, A^T b) has dimension below ell."""


def initial_basis(A, b, ell):
    """Orthonormal basis of the Krylov space K_ell(A^T A, A^T b) (Sec. 2.1, Sec. 4).

    Raises DegenerateInitialSpace when a new Krylov vector keeps less than
    1e-12 of its norm after the two projections (the space stopped growing)."""
    v = A.T @ b
    V = (v / np.linalg.norm(v))[:, None]
    for _ in range(1, ell):
        w = A.T @ (A @ V[:, -1])
        p = w
        for _ in range(2):
            p = p - V @ (V.T @ p)
        if not np.linalg.norm(p) > 1e-12 * np.linalg.norm(w):
            raise DegenerateInitialSpace("K_ell(A^T A, A^T b) has dimension < ell")
        V = np.concatenate([V, (p / np.linalg.norm(p))[:, None]], axis=1)
    return V


def mgs_project(V, r):
    """One modified Gram-Schmidt sweep of r against the columns of V (eq:single_mgs)."""
    v = r.copy()
    for j in range(V.shape[1]):
        v = v - (V[:, j] @ v) * V[:, j]
    return v


# ----------------------------------------------------------------------------
# Result container
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    x: np.ndarray                  # x_k = W_k y_k
    y: np.ndarray
    W: np.ndarray                  # basis (n x d)
    Q_A: np.ndarray
    R_A: np.ndarray
    Q_L: np.ndarray
    R_L: np.ndarray
    d_A: np.ndarray
    G: np.ndarray                  # R factor of [R_A; sqrt(mu) R_L]
    c_b: np.ndarray                # S_A b
    iters: int
    status: int
    x_hist: list                   # x after each expansion (index 0 = initial space)
    y_hist: list
    degenerate: int = 0            # number of numerically absent QR columns


# ----------------------------------------------------------------------------
# sGKS (Alg. 2) and its unsketched / identity-sketch variant
# ----------------------------------------------------------------------------

def make_sketches(m, p, s, seed, zeta=8, kind="sparse_sign"):
    """(S_A, S_L): s x m and s x p sparse-sign embeddings, SRTTs for kind="srtt"
    (eq:sketching_trig), or identities for kind="identity"."""
    if kind == "identity":
        return sp.identity(m, format="csr"), sp.identity(p, format="csr")
    if kind == "srtt":
        return SRTT(m, s, seed, 0), SRTT(p, s, seed, 1)
    if kind != "sparse_sign":
        raise ValueError(kind)
    return (sparse_sign_matrix(m, s, zeta, seed, 0), sparse_sign_matrix(p, s, zeta, seed, 1))


def sgks(A, L, b, mu, k, s, seed, zeta=8, ell=3, refine_steps=0, qr_passes=2,
         sketch="sparse_sign", keep_history=False):
    """k expansions of sGKS (Alg. 2) on min ||Ax-b||^2 + mu ||Lx||^2 (eq:tik).

    Per expansion: x = W y; r = A^T(Ax-b) + mu L^T L x (eq: gradient); append
    r / ||r|| to W without reorthogonalisation; update the thin QR factors of
    S_A A W and S_L L W by one column (eq:updqr) and d_A by one entry
    (eq:dA_update, with S_A b in place of b); solve the projected sketched
    problem (eq:projected_sketched_bis); optionally refine y.
    sketch="identity" gives sGKS_0 of Prop. 1."""
    A = sp.csr_matrix(A, dtype=np.float64)
    L = sp.csr_matrix(L, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    S_A, S_L = make_sketches(m, L.shape[0], s, seed, zeta, sketch)
    c_b = S_A @ b
    sA = S_A.shape[0]
    sL = S_L.shape[0]

    W = np.zeros((n, 0))
    Q_A, R_A = np.zeros((sA, 0)), np.zeros((0, 0))
    Q_L, R_L = np.zeros((sL, 0)), np.zeros((0, 0))
    d_A = np.zeros(0)
    degenerate = 0

    def append(w):
        """Append w; returns False (and changes nothing) when the new column of
        [R_A; sqrt(mu) R_L] is numerically dependent on the previous ones."""
        nonlocal W, Q_A, R_A, Q_L, R_L, d_A, degenerate
        QA2, RA2, da = qr_append(Q_A, R_A, S_A @ (A @ w), qr_passes)
        QL2, RL2, dl = qr_append(Q_L, R_L, S_L @ (L @ w), qr_passes)
        col = np.concatenate([RA2[:, -1], math.sqrt(mu) * RL2[:, -1]])
        _, Gt = np.linalg.qr(np.vstack([RA2, math.sqrt(mu) * RL2]), mode="reduced")
        if not abs(Gt[-1, -1]) > 1e-14 * np.linalg.norm(col):
            return False
        W = np.concatenate([W, w[:, None]], axis=1)
        Q_A, R_A, Q_L, R_L = QA2, RA2, QL2, RL2
        d_A = np.concatenate([d_A, [Q_A[:, -1] @ c_b]])
        degenerate += int(da) + int(dl)
        return True

    def solve():
        y, G = projected_solve(R_A, R_L, d_A, mu)
        return refine(A, L, b, mu, W, y, G, sA, refine_steps), G

    V0 = initial_basis(A, b, ell)
    for j in range(ell):
        if not append(V0[:, j]):
            raise DegenerateInitialSpace("sketched initial columns are dependent")
    y, G = solve()
    x_hist = [W @ y] if keep_history else []
    y_hist = [y] if keep_history else []
    r0 = float(np.linalg.norm(A.T @ b))
    status = STATUS_OK
    it = 0
    for it in range(1, k + 1):
        r = gradient(A, L, b, mu, W @ y)
        nr = float(np.linalg.norm(r))
        if not nr > 1e-14 * r0 or not append(r / nr):
            status = STATUS_BREAKDOWN
            it -= 1
            break
        y, G = solve()
        if keep_history:
            x_hist.append(W @ y)
            y_hist.append(y)
    return Result(W @ y, y, W, Q_A, R_A, Q_L, R_L, d_A, G, c_b, it, status, x_hist, y_hist,
                  degenerate)


def refinement_weights(d, s):
    """Heavy-ball weights (alpha, beta) for a d-column problem and s sketch rows."""
    eta2 = min(d / float(s), 0.999)
    return (1.0 - eta2) ** 2, eta2


def refine(A, L, b, mu, W, y, G, s, steps):
    """`steps` sketch-preconditioned heavy-ball refinement steps of the projected solve.

    Each step needs the gradient r(y) = A^T(A W y - b) + mu L^T L W y, whose
    projection W^T r(y) is the residual of the unsketched projected normal
    equations (eq:sGKS_noSASL)."""
    alpha, beta = refinement_weights(W.shape[1], s)
    y_prev = y
    for _ in range(steps):
        r = gradient(A, L, b, mu, W @ y)
        y_next = y - alpha * gram_solve(G, W.T @ r) + beta * (y - y_prev)
        y_prev, y = y, y_next
    return y


def unsketched_projected_solution(A, L, b, mu, W):
    """y_sGKS0 of eq:sGKS_noSASL on a given basis W: min ||A W y - b||^2 + mu ||L W y||^2."""
    M = np.vstack([A @ W, math.sqrt(mu) * (L @ W)])
    f = np.concatenate([b, np.zeros(L.shape[0])])
    y, *_ = np.linalg.lstsq(M, f, rcond=None)
    return y


# ----------------------------------------------------------------------------
# GKS (Alg. 1)
# ----------------------------------------------------------------------------

def gks(A, L, b, mu, k, ell=3, tau=1e-10, qr_passes=2, keep_history=False):
    """k iterations of GKS (Alg. 1): orthonormal V, reorthogonalised expansion.

    The new direction is r projected by one MGS sweep (eq:single_mgs); when
    the loss ratio ||V^T v|| / ||v|| (eq:loss_criterion) is >= tau a second
    sweep follows.  QR factors of A V and L V are updated by eq:updqr and
    d_A = Q_A^T b by eq:dA_update."""
    A = sp.csr_matrix(A, dtype=np.float64)
    L = sp.csr_matrix(L, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    V = np.zeros((n, 0))
    Q_A, R_A = np.zeros((m, 0)), np.zeros((0, 0))
    Q_L, R_L = np.zeros((L.shape[0], 0)), np.zeros((0, 0))
    d_A = np.zeros(0)

    def append(v):
        nonlocal V, Q_A, R_A, Q_L, R_L, d_A
        V = np.concatenate([V, v[:, None]], axis=1)
        Q_A, R_A, _ = qr_append(Q_A, R_A, A @ v, qr_passes)
        Q_L, R_L, _ = qr_append(Q_L, R_L, L @ v, qr_passes)
        d_A = np.concatenate([d_A, [Q_A[:, -1] @ b]])

    V0 = initial_basis(A, b, ell)
    for j in range(ell):
        append(V0[:, j])
    y, G = projected_solve(R_A, R_L, d_A, mu)
    x_hist = [V @ y] if keep_history else []
    y_hist = [y] if keep_history else []
    r0 = float(np.linalg.norm(A.T @ b))
    status = STATUS_OK
    it = 0
    for it in range(1, k + 1):
        r = gradient(A, L, b, mu, V @ y)
        v = mgs_project(V, r)
        nv = float(np.linalg.norm(v))
        if not nv > 1e-14 * r0:
            status = STATUS_BREAKDOWN
            it -= 1
            break
        loss = float(np.linalg.norm(V.T @ v)) / nv
        if loss >= tau:
            v = mgs_project(V, v)
        append(v / np.linalg.norm(v))
        y, G = projected_solve(R_A, R_L, d_A, mu)
        if keep_history:
            x_hist.append(V @ y)
            y_hist.append(y)
    return Result(V @ y, y, V, Q_A, R_A, Q_L, R_L, d_A, G, b, it, status, x_hist, y_hist)


# ----------------------------------------------------------------------------
# Residual norms, adjoint, dense references
# ----------------------------------------------------------------------------

def tikhonov_residual(A, L, b, mu, x):
    """sqrt(||A x - b||^2 + mu ||L x||^2)."""
    return math.sqrt(float(np.linalg.norm(A @ x - b) ** 2 + mu * np.linalg.norm(L @ x) ** 2))


def sketched_residual(A, L, b, mu, x, s, seed, zeta=8, kind="sparse_sign"):
    """sqrt(||S_A(A x - b)||^2 + mu ||S_L L x||^2) (the functional of eq:tik_new_sketched)."""
    S_A, S_L = make_sketches(A.shape[0], L.shape[0], s, seed, zeta, kind)
    return math.sqrt(float(np.linalg.norm(S_A @ (A @ x - b)) ** 2
                           + mu * np.linalg.norm(S_L @ (L @ x)) ** 2))


def _stacked_r(res: Result, mu):
    """G, the R factor (Householder) of [R_A; sqrt(mu) R_L], so that
    H = R_A^T R_A + mu R_L^T R_L = G^T G."""
    _, G = np.linalg.qr(np.vstack([res.R_A, math.sqrt(mu) * res.R_L]), mode="reduced")
    return G


def frozen_adjoint(res: Result, mu, g_x):
    """Gradients of loss(x_k) w.r.t. b and mu with W, Q_A, R_A, R_L held fixed.

    x = W y, y = H^{-1} R_A^T Q_A^T S_A b with H = R_A^T R_A + mu R_L^T R_L, so
    for g_x = d loss / d x:  z = H^{-1} W^T g_x,
    d loss / d b  = S_A^T Q_A R_A z   (returned as the s-vector v = Q_A R_A z,
                                        and applied to S_A^T by the caller),
    d loss / d mu = -(R_L z) . (R_L y).
    H^{-1} is applied as G^{-1} G^{-T} with G the R factor of the stacked matrix
    (H = G^T G), which does not square the condition number as forming H would."""
    z = gram_solve(_stacked_r(res, mu), res.W.T @ g_x)
    v = res.Q_A @ (res.R_A @ z)
    gmu = -float((res.R_L @ z) @ (res.R_L @ res.y))
    return v, gmu


def frozen_adjoint_b(res: Result, mu, g_x, A, L, s, seed, zeta=8, sketch="sparse_sign"):
    """(d loss / d b as an m-vector, d loss / d mu) of the frozen map."""
    v, gmu = frozen_adjoint(res, mu, g_x)
    S_A, _ = make_sketches(A.shape[0], L.shape[0], s, seed, zeta, sketch)
    return S_A.T @ v, gmu


def frozen_map(res: Result, b, mu, S_A):
    """x(b, mu) = W H(mu)^{-1} R_A^T Q_A^T S_A b with the basis and factors held fixed."""
    return res.W @ gram_solve(_stacked_r(res, mu), res.R_A.T @ (res.Q_A.T @ (S_A @ b)))


def total_adjoint(A, L, b, mu, k, s, seed, g_x, zeta=8, ell=3, sketch="sparse_sign"):
    """(d loss / d b, d loss / d mu) of the whole sGKS map b, mu -> x_k (Alg. 2, k
    expansions, no refinement), given g_x = d loss / d x_k.  Not in the paper.

    Differentiated map (the exact-arithmetic form of every step of Alg. 2):
      * W_0 = Gram-Schmidt of the Krylov chain v_1 = A^T b / ||A^T b||,
        p_i = (I - V_i V_i^T) A^T A v_i, v_{i+1} = p_i / ||p_i|| (Sec. 2.1);
      * with B_A = S_A A W_j, B_L = S_L L W_j and c_b = S_A b, the projected
        solve eq:projected_sketched_bis is y_j = N_j^{-1} B_A^T c_b with
        N_j = B_A^T B_A + mu B_L^T B_L (Q_A R_A = B_A, Q_L R_L = B_L by
        eq:updqr, d_A = Q_A^T c_b by eq:dA_update);
      * x_j = W_j y_j; r_j = A^T (A x_j - b) + mu L^T L x_j (eq: gradient);
        the next column is r_j / ||r_j||.
    The reverse sweep runs j = k, ..., 0 and keeps the adjoint of every basis
    column as an explicit n x d matrix; N_j^{-1} is applied through the R factor
    of [B_A; sqrt(mu) B_L] (no squared condition number)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    L = sp.csr_matrix(L, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    res = sgks(A, L, b, mu, k, s, seed, zeta, ell, sketch=sketch, keep_history=True)
    if res.status != STATUS_OK or res.iters != k:
        raise ValueError("the total adjoint needs k expansions without breakdown")
    S_A, S_L = make_sketches(A.shape[0], L.shape[0], s, seed, zeta, sketch)
    W = res.W
    n, d = W.shape
    c_b = S_A @ b
    BA = S_A @ (A @ W)
    BL = S_L @ (L @ W)

    def hess(v):
        return A.T @ (A @ v) + mu * (L.T @ (L @ v))

    Wbar = np.zeros((n, d))
    gb = np.zeros(A.shape[0])
    gmu = 0.0
    cbar = np.zeros(c_b.shape[0])
    for j in range(k, -1, -1):
        dj = ell + j
        y = res.y_hist[j]
        if j == k:
            xbar = np.asarray(g_x, dtype=np.float64)
        else:
            # column dj was r_j / ||r_j||
            x_j = res.x_hist[j]
            r = gradient(A, L, b, mu, x_j)
            w = W[:, dj]
            wbar = Wbar[:, dj]
            rbar = (wbar - w * (w @ wbar)) / np.linalg.norm(r)
            xbar = hess(rbar)
            gb -= A @ rbar
            gmu += float((L @ rbar) @ (L @ x_j))
        # x_j = W_j y_j
        Wbar[:, :dj] += np.outer(xbar, y)
        ybar = W[:, :dj].T @ xbar
        # y_j = N_j^{-1} B_A^T c_b
        Bj, Lj = BA[:, :dj], BL[:, :dj]
        _, G = np.linalg.qr(np.vstack([Bj, math.sqrt(mu) * Lj]), mode="reduced")
        u = gram_solve(G, ybar)
        cbar += Bj @ u
        sym = np.outer(y, u) + np.outer(u, y)
        BAbar = np.outer(c_b, u) - Bj @ sym
        BLbar = -mu * (Lj @ sym)
        gmu -= float((Lj @ u) @ (Lj @ y))
        Wbar[:, :dj] += A.T @ (S_A.T @ BAbar) + L.T @ (S_L.T @ BLbar)
    # W_0: reverse of the Krylov Gram-Schmidt chain
    V = W[:, :ell]
    Vbar = Wbar[:, :ell].copy()
    for i in range(ell - 1, 0, -1):
        z = A.T @ (A @ V[:, i - 1])
        Vi = V[:, :i]
        p = z - Vi @ (Vi.T @ z)
        pbar = (Vbar[:, i] - V[:, i] * (V[:, i] @ Vbar[:, i])) / np.linalg.norm(p)
        zbar = pbar - Vi @ (Vi.T @ pbar)
        Vbar[:, :i] -= np.outer(pbar, Vi.T @ z) + np.outer(z, Vi.T @ pbar)
        Vbar[:, i - 1] += A.T @ (A @ zbar)
    g = A.T @ b
    v1 = V[:, 0]
    gb += A @ ((Vbar[:, 0] - v1 * (v1 @ Vbar[:, 0])) / np.linalg.norm(g))
    gb += S_A.T @ cbar
    return gb, gmu


def dense_tikhonov(A, L, b, mu):
    """Solution of (A^T A + mu L^T L) x = A^T b (normal equations of eq:tik)."""
    A = np.asarray(sp.csr_matrix(A).todense())
    L = np.asarray(sp.csr_matrix(L).todense())
    return np.linalg.solve(A.T @ A + mu * L.T @ L, A.T @ b)


def dense_sketched_tikhonov(A, L, b, mu, S_A, S_L):
    """Solution of min ||S_A(Ax-b)||^2 + mu ||S_L L x||^2 over all of R^n."""
    A = np.asarray(sp.csr_matrix(A).todense())
    L = np.asarray(sp.csr_matrix(L).todense())
    SA = np.asarray(sp.csr_matrix(S_A).todense())
    SL = np.asarray(sp.csr_matrix(S_L).todense())
    H = A.T @ SA.T @ SA @ A + mu * L.T @ SL.T @ SL @ L
    return np.linalg.solve(H, A.T @ SA.T @ (SA @ b))


def embedding_epsilon(S, Q):
    """max_i |sigma_i(S Q)^2 - 1| for orthonormal Q: the smallest eps with eq:norm_equiv on range(Q)."""
    sv = np.linalg.svd(np.asarray(S @ Q), compute_uv=False)
    return float(np.max(np.abs(sv ** 2 - 1.0)))
