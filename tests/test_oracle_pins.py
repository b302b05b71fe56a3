"""Pins of the FP64 CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the published definition) that fixes
the value it checks: closed forms, invariants, the paper's propositions, special
cases that reduce to a textbook solve, published generator outputs, brute force
on tiny inputs.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sgks_oracle as O
from workloads import generators as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(n=14, seed=1, mu=1e-2, sigma=1.5):
    A = gen.blur1d_dense(n, sigma)
    L = gen.diff1d(n)
    rng = np.random.default_rng(seed)
    x = gen.step_signal(n, rng)
    b = gen.add_noise(A @ x, 0.01, rng)
    return A, L, b, mu


def tiny2d(N=6, seed=2, mu=5e-3):
    A = gen.psf_blur2d(N, sigma=1.0, half=1)
    L = gen.grad2d(N)
    rng = np.random.default_rng(seed)
    x = gen.random_ellipses(N, rng, count=3)
    b = gen.add_noise(A @ x, 0.01, rng)
    return A, L, b, mu


# ----------------------------------------------------------------------------
# sparse-sign embedding
# ----------------------------------------------------------------------------

def test_splitmix64_published_sequence():
    """mix64(c * gamma) is SplitMix64 output c from state 0 (Steele, Lea & Flood 2014)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for c, hx in rows:
        with np.errstate(over="ignore"):
            z = O.mix64(O.GAMMA * np.uint64(int(c)))
        assert int(z) == int(hx, 16)


def _bruteforce_column(j, s, zeta, seed, stream):
    """Rows and signs of one column by a plain scalar loop (Python integers mod 2^64)."""
    mask = (1 << 64) - 1
    g = 0x9E3779B97F4A7C15
    key = int(O.mix64(np.uint64((seed + g * (2 * j + stream + 1)) & mask)))
    rows, signs, c = [], [], 0
    while len(rows) < zeta:
        z = int(O.mix64(np.uint64((key + g * (c + 1)) & mask)))
        c += 1
        row = ((z >> 32) * s) >> 32
        if row in rows:
            continue
        rows.append(row)
        signs.append(-1 if z & 1 else 1)
    return rows, signs


@pytest.mark.parametrize("s,zeta,seed,stream", [(12, 8, 0, 0), (9, 8, 3, 1), (40, 8, 11, 0), (8, 8, 5, 1)])
def test_sparse_sign_pattern_matches_scalar_definition(s, zeta, seed, stream):
    h = 50
    rows, signs = O.sparse_sign_pattern(h, s, zeta, seed, stream)
    for j in range(h):
        r, g = _bruteforce_column(j, s, zeta, seed, stream)
        assert list(rows[j]) == r
        assert list(signs[j]) == g


def test_sparse_sign_invariants():
    h, s, zeta = 3000, 64, 8
    S = O.sparse_sign_matrix(h, s, zeta, seed=7, stream=0)
    assert S.shape == (s, h)
    C = S.tocsc()
    nnz = np.diff(C.indptr)
    assert np.all(nnz == zeta)                                  # zeta distinct rows per column
    assert np.allclose(np.abs(C.data), 1 / math.sqrt(zeta), rtol=0, atol=0)
    colnorm2 = np.asarray(C.multiply(C).sum(axis=0)).ravel()
    assert np.allclose(colnorm2, 1.0, rtol=0, atol=4e-16)      # ||S e_j|| = 1
    # determinism, dependence on seed and stream
    S2 = O.sparse_sign_matrix(h, s, zeta, seed=7, stream=0)
    assert (S != S2).nnz == 0
    assert (S != O.sparse_sign_matrix(h, s, zeta, seed=8, stream=0)).nnz > 0
    assert (S != O.sparse_sign_matrix(h, s, zeta, seed=7, stream=1)).nnz > 0
    # rows roughly uniform, signs balanced
    rows, signs = O.sparse_sign_pattern(h, s, zeta, 7, 0)
    counts = np.bincount(rows.ravel(), minlength=s)
    assert counts.min() > 0.7 * h * zeta / s and counts.max() < 1.3 * h * zeta / s
    assert abs(signs.mean()) < 0.02


def test_sparse_sign_is_isometric_in_expectation():
    """E ||S x||^2 = ||x||^2 for independent +-1 signs (Def. 1 holds on average)."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(500)
    ratios = [np.linalg.norm(O.sparse_sign_matrix(500, 40, 8, sd, 0) @ x) ** 2 / (x @ x)
              for sd in range(200)]
    assert abs(np.mean(ratios) - 1.0) < 0.03


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def test_gradient_is_gradient_of_tikhonov_functional():
    """eq: gradient is half the gradient of ||Ax-b||^2 + mu ||Lx||^2 (central differences)."""
    A, L, b, mu = tiny2d()
    rng = np.random.default_rng(3)
    x = rng.standard_normal(A.shape[1])
    phi = lambda z: 0.5 * (np.linalg.norm(A @ z - b) ** 2 + mu * np.linalg.norm(L @ z) ** 2)
    r = O.gradient(A, L, b, mu, x)
    h = 1e-6
    fd = np.array([(phi(x + h * e) - phi(x - h * e)) / (2 * h) for e in np.eye(x.size)])
    assert np.allclose(r, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("passes", [1, 2])
def test_qr_append_builds_a_qr_factorisation(passes):
    """eq:updqr applied column by column gives Q^T Q = I, Q R = M, R upper with rho > 0."""
    rng = np.random.default_rng(4)
    M = rng.standard_normal((40, 12))
    Q, R = np.zeros((40, 0)), np.zeros((0, 0))
    for j in range(12):
        Q, R, deg = O.qr_append(Q, R, M[:, j], passes)
        assert not deg
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-13)
    assert np.allclose(Q @ R, M, atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.diag(R) > 0)
    # unique thin QR with positive diagonal: compare with LAPACK Householder up to signs
    _, R2 = np.linalg.qr(M)
    assert np.allclose(np.abs(R), np.abs(R2), atol=1e-12)


def test_qr_append_flags_dependent_column():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((30, 4))
    Q, R = np.zeros((30, 0)), np.zeros((0, 0))
    for j in range(4):
        Q, R, _ = O.qr_append(Q, R, M[:, j])
    c = np.array([1.0, -2.0, 0.5, 3.0])
    Q, R, deg = O.qr_append(Q, R, M @ c)
    assert deg and R[-1, -1] == 0.0 and np.all(Q[:, -1] == 0)
    assert np.allclose(R[:4, -1], R[:4, :4] @ c, atol=1e-12)   # p = Q^T M c = R c


def test_cgs2_of_ill_conditioned_columns_is_orthonormal():
    rng = np.random.default_rng(6)
    base = rng.standard_normal((200, 5))
    M = base @ np.diag([1, 1e-3, 1e-6, 1e-8, 1e-9]) @ rng.standard_normal((5, 5))
    Q, R = np.zeros((200, 0)), np.zeros((0, 0))
    for j in range(5):
        Q, R, _ = O.qr_append(Q, R, M[:, j], passes=2)
    assert np.linalg.norm(Q.T @ Q - np.eye(5)) < 1e-10


def test_projected_solve_equals_lstsq():
    """eq:projected_sketched_bis: min ||[R_A; sqrt(mu) R_L] y - [d_A; 0]||."""
    rng = np.random.default_rng(7)
    d = 9
    R_A = np.triu(rng.standard_normal((d, d))) + 3 * np.eye(d)
    R_L = np.triu(rng.standard_normal((d, d))) + 2 * np.eye(d)
    d_A = rng.standard_normal(d)
    mu = 0.3
    y, G = O.projected_solve(R_A, R_L, d_A, mu)
    M = np.vstack([R_A, math.sqrt(mu) * R_L])
    y2 = np.linalg.lstsq(M, np.concatenate([d_A, np.zeros(d)]), rcond=None)[0]
    assert np.allclose(y, y2, rtol=1e-12, atol=1e-13)
    assert np.allclose(G.T @ G, M.T @ M, rtol=1e-12, atol=1e-12)
    g = rng.standard_normal(d)
    assert np.allclose(M.T @ M @ O.gram_solve(G, g), g, atol=1e-11)


def test_initial_basis_spans_krylov_space():
    """W_0 = orthonormal basis of K_3(A^T A, A^T b) (Sec. 2.1, ell = 3 in Sec. 4)."""
    A, L, b, mu = tiny2d()
    V = O.initial_basis(A, b, 3)
    assert np.allclose(V.T @ V, np.eye(3), atol=1e-13)
    K = [A.T @ b]
    for _ in range(2):
        K.append(A.T @ (A @ K[-1]))
    for v in K:
        assert np.linalg.norm(v - V @ (V.T @ v)) <= 1e-10 * np.linalg.norm(v)


# ----------------------------------------------------------------------------
# GKS (Alg. 1)
# ----------------------------------------------------------------------------

def test_gks_full_space_is_dense_tikhonov():
    """At d = n the projected problem is eq:tik itself: Cholesky/LU of the normal equations."""
    for A, L, b, mu in (tiny(), tiny2d()):
        n = A.shape[1]
        res = O.gks(A, L, b, mu, n - 3)
        # either the space is all of R^n, or it stopped growing on an invariant
        # subspace of A^T A + mu L^T L containing A^T b, which holds the solution
        assert res.W.shape[1] == n or res.status == O.STATUS_BREAKDOWN
        xd = O.dense_tikhonov(A, L, b, mu)
        assert np.linalg.norm(res.x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_gks_basis_orthonormal_and_gradient_orthogonal():
    """V^T V = I, and V_k^T r_{k+1} = 0 (normal equations of eq:projected_withQR)."""
    A, L, b, mu = tiny2d(N=8)
    res = O.gks(A, L, b, mu, 20, keep_history=True)
    V = res.W
    assert np.linalg.norm(V.T @ V - np.eye(V.shape[1])) < 1e-12
    for k in range(0, 20, 4):
        d = 3 + k
        r = O.gradient(A, L, b, mu, res.x_hist[k])
        assert np.linalg.norm(V[:, :d].T @ r) <= 1e-9 * np.linalg.norm(r)


def test_gks_cheap_stopping_identity():
    """eq:stoppingcriterion_cheap: ||x_k - x_{k-1}|| = ||y_k - [y_{k-1}; 0]||."""
    A, L, b, mu = tiny2d(N=8)
    res = O.gks(A, L, b, mu, 12, keep_history=True)
    for k in range(1, 13):
        lhs = np.linalg.norm(res.x_hist[k] - res.x_hist[k - 1])
        rhs = np.linalg.norm(res.y_hist[k] - np.concatenate([res.y_hist[k - 1], [0.0]]))
        assert abs(lhs - rhs) <= 1e-10 * max(rhs, 1e-300)


# ----------------------------------------------------------------------------
# sGKS (Alg. 2)
# ----------------------------------------------------------------------------

def test_prop1_identity_sketch_equals_gks():
    """Prop. 1: without sketching, the sGKS iterates equal the GKS iterates."""
    for A, L, b, mu in (tiny(n=40), tiny2d(N=8)):
        k = 15
        g = O.gks(A, L, b, mu, k, keep_history=True)
        s0 = O.sgks(A, L, b, mu, k, 0, 0, sketch="identity", keep_history=True)
        for j in range(k + 1):
            assert np.linalg.norm(g.x_hist[j] - s0.x_hist[j]) <= 1e-10 * np.linalg.norm(g.x_hist[j])


def test_sgks_full_space_is_dense_sketched_tikhonov():
    """At d = n, x_k minimises the sketched functional eq:tik_new_sketched over R^n."""
    A, L, b, mu = tiny(n=8, sigma=0.8)
    s, seed = 100, 5
    res = O.sgks(A, L, b, mu, 5, s, seed)
    assert res.W.shape == (8, 8)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    xs = O.dense_sketched_tikhonov(A, L, b, mu, S_A, S_L)
    tol = 1e-14 * np.linalg.cond(res.W) ** 2          # W is not orthonormal (Sec. 3)
    assert np.linalg.norm(res.x - xs) <= tol * np.linalg.norm(xs)


def test_sgks_qr_factors_are_factors_of_sketched_products():
    """Q_A R_A = S_A A W_k, Q_L R_L = S_L L W_k, d_A = Q_A^T S_A b (Sec. 3)."""
    A, L, b, mu = tiny2d(N=8)
    s, seed = 60, 3
    res = O.sgks(A, L, b, mu, 10, s, seed)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    SAW = S_A @ (A @ res.W)
    SLW = S_L @ (L @ res.W)
    assert np.allclose(res.Q_A @ res.R_A, SAW, atol=1e-12 * np.abs(SAW).max())
    assert np.allclose(res.Q_L @ res.R_L, SLW, atol=1e-12 * np.abs(SLW).max())
    assert np.allclose(res.d_A, res.Q_A.T @ (S_A @ b), atol=1e-12)
    # columns of W are the initial basis followed by normalised gradients
    assert np.allclose(np.linalg.norm(res.W, axis=0), 1.0)


def test_sgks_y_minimises_sketched_projected_functional():
    """y_k solves eq:tik_new_sketched on the current basis (checked by dense lstsq)."""
    A, L, b, mu = tiny2d(N=8)
    s, seed = 60, 9
    res = O.sgks(A, L, b, mu, 10, s, seed)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    M = np.vstack([S_A @ (A @ res.W), math.sqrt(mu) * (S_L @ (L @ res.W))])
    f = np.concatenate([S_A @ b, np.zeros(s)])
    y2 = np.linalg.lstsq(M, f, rcond=None)[0]
    assert np.linalg.norm(res.y - y2) <= 1e-9 * np.linalg.norm(y2)


def test_sgks_gradient_is_new_basis_column():
    """Alg. 2: W_{k+1} = [W_k, r_{k+1}/||r_{k+1}||] with r from eq: gradient at x_k."""
    A, L, b, mu = tiny2d(N=8)
    res = O.sgks(A, L, b, mu, 6, 50, 1, keep_history=True)
    for k in range(6):
        r = O.gradient(A, L, b, mu, res.x_hist[k])
        assert np.allclose(res.W[:, 3 + k], r / np.linalg.norm(r), atol=1e-12)


def _eps(S, M):
    Q, _ = np.linalg.qr(M)
    return O.embedding_epsilon(S, Q)


def test_sketched_residual_within_embedding_bound_and_prop2():
    """Def. 1 on range([AW, b]) and range(LW); Prop. 2 with theta = max(eps_A, eps_L)."""
    A, L, b, mu = tiny2d(N=10)
    s, seed = 150, 4
    res = O.sgks(A, L, b, mu, 8, s, seed)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    W = res.W
    eA = _eps(S_A, np.column_stack([A @ W, b]))
    eL = _eps(S_L, L @ W)
    eps = max(eA, eL)
    assert eps < 1
    phi = lambda y: np.linalg.norm(A @ W @ y - b) ** 2 + mu * np.linalg.norm(L @ W @ y) ** 2
    phis = lambda y: (np.linalg.norm(S_A @ (A @ W @ y - b)) ** 2
                      + mu * np.linalg.norm(S_L @ (L @ W @ y)) ** 2)
    rng = np.random.default_rng(0)
    for y in [res.y] + [rng.standard_normal(W.shape[1]) for _ in range(5)]:
        ratio = phis(y) / phi(y)
        assert 1 - eps - 1e-12 <= ratio <= 1 + eps + 1e-12
    y0 = O.unsketched_projected_solution(A, L, b, mu, W)
    assert phi(res.y) <= (1 + eps) / (1 - eps) * phi(y0) * (1 + 1e-12)
    assert phi(y0) <= phi(res.y) * (1 + 1e-12)


@pytest.mark.parametrize("s", [30, 40, 80])
def test_refinement_converges_to_unsketched_projected_solution(s):
    """IR moves y_sGKS toward y_sGKS0 (end of Sec. 3.1), also at sketch distortion > 1/2."""
    A, L, b, mu = tiny2d(N=10)
    res = O.sgks(A, L, b, mu, 8, s, 2)
    W = res.W
    y0 = O.unsketched_projected_solution(A, L, b, mu, W)
    H = W.T @ (A.T @ (A @ W)) + mu * W.T @ (L.T @ (L @ W))
    err = lambda y: math.sqrt((y - y0) @ H @ (y - y0))
    e0 = err(res.y)
    assert err(O.refine(A, L, b, mu, W, res.y, res.G, s, 2)) < 0.5 * e0
    assert err(O.refine(A, L, b, mu, W, res.y, res.G, s, 60)) <= 1e-7 * e0


def test_sgks_with_refinement_tracks_gks_better():
    """With IR the sGKS iterate is closer to the unsketched (GKS) iterate (Sec. 4.3)."""
    A, L, b, mu = tiny2d(N=10)
    g = O.gks(A, L, b, mu, 10)
    plain = O.sgks(A, L, b, mu, 10, 30, 1)
    ir = O.sgks(A, L, b, mu, 10, 30, 1, refine_steps=4)
    assert np.linalg.norm(ir.x - g.x) < np.linalg.norm(plain.x - g.x)


def test_breakdown_on_invariant_subspace():
    """A = L = I: K_3(A^T A, A^T b) is span{b}; the expansion stops (status BREAKDOWN)."""
    n = 10
    A = sp.identity(n, format="csr")
    L = sp.identity(n, format="csr")
    b = np.linspace(1, 2, n)
    V = O.initial_basis(A, b, 1)
    res = O.sgks(A, L, b, 0.5, 4, 0, 0, ell=1, sketch="identity")
    assert res.status == O.STATUS_BREAKDOWN and res.iters == 0
    assert np.allclose(res.x, b / 1.5)
    assert np.allclose(V[:, 0], b / np.linalg.norm(b))
    with pytest.raises(O.DegenerateInitialSpace):
        O.initial_basis(A, b, 2)


def test_breakdown_on_dependent_sketched_column():
    """A = L = I with a sparse-sign sketch: r(x) is parallel to b, so the new column
    repeats w_1; the stacked projected column is dependent and the expansion stops."""
    n = 64
    A = sp.identity(n, format="csr")
    b = np.linspace(1, 2, n)
    res = O.sgks(A, A, b, 0.5, 4, 16, 0, ell=1)
    assert res.status == O.STATUS_BREAKDOWN and res.iters == 0 and res.W.shape[1] == 1


# ----------------------------------------------------------------------------
# frozen-basis adjoint
# ----------------------------------------------------------------------------

def test_frozen_adjoint_matches_central_differences():
    A, L, b, mu = tiny2d(N=8)
    s, seed = 60, 3
    res = O.sgks(A, L, b, mu, 10, s, seed)
    S_A, _ = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    rng = np.random.default_rng(1)
    x_t = rng.standard_normal(A.shape[1])
    loss = lambda bb, mm: float(np.linalg.norm(O.frozen_map(res, bb, mm, S_A) - x_t) ** 2)
    gb, gmu = O.frozen_adjoint_b(res, mu, 2 * (res.x - x_t), A, L, s, seed)
    assert np.allclose(O.frozen_map(res, b, mu, S_A), res.x, rtol=1e-9)
    h = 1e-6
    for i in rng.choice(A.shape[0], 6, replace=False):
        e = np.zeros_like(b)
        e[i] = h
        fd = (loss(b + e, mu) - loss(b - e, mu)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * max(1.0, abs(fd))
    hm = 1e-6 * mu
    fdm = (loss(b, mu + hm) - loss(b, mu - hm)) / (2 * hm)
    assert abs(fdm - gmu) <= 1e-6 * max(1.0, abs(fdm))


def test_frozen_adjoint_equals_dense_adjoint_at_full_space():
    """At d = n the frozen map is the dense sketched Tikhonov map; compare with its adjoint."""
    A, L, b, mu = tiny(n=8, sigma=0.8)
    s, seed = 100, 5
    res = O.sgks(A, L, b, mu, 5, s, seed)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    Ad, Ld = A.toarray(), L.toarray()
    SA, SL = S_A.toarray(), S_L.toarray()
    H = Ad.T @ SA.T @ SA @ Ad + mu * Ld.T @ SL.T @ SL @ Ld
    x = np.linalg.solve(H, Ad.T @ SA.T @ SA @ b)
    rng = np.random.default_rng(2)
    g_x = rng.standard_normal(A.shape[1])
    gb_dense = SA.T @ SA @ Ad @ np.linalg.solve(H, g_x)
    gmu_dense = -float(g_x @ np.linalg.solve(H, Ld.T @ SL.T @ SL @ Ld @ x))
    gb, gmu = O.frozen_adjoint_b(res, mu, g_x, A, L, s, seed)
    tol = 1e-14 * np.linalg.cond(res.W) ** 2
    assert np.linalg.norm(gb - gb_dense) <= tol * np.linalg.norm(gb_dense)
    assert abs(gmu - gmu_dense) <= tol * abs(gmu_dense)


# ----------------------------------------------------------------------------
# total-derivative adjoint (through every expansion and the initial basis)
# ----------------------------------------------------------------------------

def _total_fd_errors(A, L, b, mu, k, s, seed, sketch, g_x, gb, gmu, rng, ndir=3):
    """Relative errors of the adjoint against central differences of
    g_x . x_k(b, mu), x_k from k expansions of the oracle's Alg. 2."""
    f = lambda bb, mm: float(g_x @ O.sgks(A, L, bb, mm, k, s, seed, sketch=sketch).x)
    errs = []
    for _ in range(ndir):
        db = rng.standard_normal(b.size)
        h = 1e-5 * np.linalg.norm(b) / np.linalg.norm(db)
        fd = (f(b + h * db, mu) - f(b - h * db, mu)) / (2 * h)
        errs.append(abs(fd - gb @ db) / max(abs(fd), 1e-3))
    hm = 1e-5 * mu
    fd = (f(b, mu + hm) - f(b, mu - hm)) / (2 * hm)
    errs.append(abs(fd - gmu) / max(abs(fd), 1e-3))
    return errs


@pytest.mark.parametrize("k,sketch", [(0, "sparse_sign"), (4, "sparse_sign"), (6, "srtt")])
def test_total_adjoint_matches_central_differences(k, sketch):
    """The reverse sweep is the derivative of the composed map of Alg. 2: directional
    derivatives in b and mu from central differences of x_k itself.  k = 0 leaves
    only the initial Krylov basis and the first projected solve."""
    A, L, b, mu = tiny2d(N=6 if sketch == "sparse_sign" else 8)
    s, seed = 60, 3
    rng = np.random.default_rng(7)
    g_x = rng.standard_normal(A.shape[1])
    gb, gmu = O.total_adjoint(A, L, b, mu, k, s, seed, g_x, sketch=sketch)
    assert max(_total_fd_errors(A, L, b, mu, k, s, seed, sketch, g_x, gb, gmu, rng)) < 1e-6


def test_total_adjoint_at_full_space_is_dense_adjoint():
    """At d = n, x_k is the dense sketched Tikhonov solution whatever the basis, so every
    contribution through the basis cancels and the adjoint is the closed form
    S_A^T S_A A Hs^{-1} g_x, -(Hs^{-1} g_x)^T L^T S_L^T S_L L x."""
    A, L, b, mu = tiny(n=8, sigma=0.8)
    s, seed = 100, 5
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed)
    Ad, Ld = A.toarray(), L.toarray()
    SA, SL = S_A.toarray(), S_L.toarray()
    H = Ad.T @ SA.T @ SA @ Ad + mu * Ld.T @ SL.T @ SL @ Ld
    x = np.linalg.solve(H, Ad.T @ SA.T @ SA @ b)
    g_x = np.random.default_rng(2).standard_normal(A.shape[1])
    z = np.linalg.solve(H, g_x)
    gb_dense = SA.T @ SA @ Ad @ z
    gmu_dense = -float(z @ (Ld.T @ SL.T @ SL @ Ld @ x))
    res = O.sgks(A, L, b, mu, 5, s, seed)
    gb, gmu = O.total_adjoint(A, L, b, mu, 5, s, seed, g_x)
    tol = 1e-13 * np.linalg.cond(res.W) ** 2
    assert np.linalg.norm(gb - gb_dense) <= tol * np.linalg.norm(gb_dense)
    assert abs(gmu - gmu_dense) <= tol * abs(gmu_dense)


def test_total_adjoint_of_identity_sketch_is_the_derivative_of_gks():
    """Prop. 1: with identity sketches sGKS_0 has the iterates of GKS (Alg. 1, whose basis
    is reorthogonalised).  The total adjoint of sGKS_0 therefore differentiates the GKS map:
    compare with central differences of the oracle's GKS solution."""
    A, L, b, mu = tiny2d(N=6)
    k = 5
    s = max(A.shape[0], L.shape[0])
    rng = np.random.default_rng(9)
    g_x = rng.standard_normal(A.shape[1])
    gb, gmu = O.total_adjoint(A, L, b, mu, k, s, 0, g_x, sketch="identity")
    f = lambda bb, mm: float(g_x @ O.gks(A, L, bb, mm, k).x)
    for _ in range(3):
        db = rng.standard_normal(b.size)
        h = 1e-5 * np.linalg.norm(b) / np.linalg.norm(db)
        fd = (f(b + h * db, mu) - f(b - h * db, mu)) / (2 * h)
        assert abs(fd - gb @ db) <= 1e-6 * max(abs(fd), 1e-3)
    hm = 1e-5 * mu
    fdm = (f(b, mu + hm) - f(b, mu - hm)) / (2 * hm)
    assert abs(fdm - gmu) <= 1e-6 * max(abs(fdm), 1e-3)


def test_total_adjoint_pins_reject_a_wrong_solve_and_the_frozen_adjoint(monkeypatch):
    """The difference pin separates the total derivative from plausible slips: the
    frozen-basis adjoint (no path through W) and a projected solve applied with one
    triangular factor only both miss it by far more than the tolerance."""
    A, L, b, mu = tiny2d(N=6)
    k, s, seed = 4, 60, 3
    rng = np.random.default_rng(7)
    g_x = rng.standard_normal(A.shape[1])
    res = O.sgks(A, L, b, mu, k, s, seed)
    gb_f, gmu_f = O.frozen_adjoint_b(res, mu, g_x, A, L, s, seed)
    assert max(_total_fd_errors(A, L, b, mu, k, s, seed, "sparse_sign", g_x, gb_f, gmu_f,
                                np.random.default_rng(7))) > 1e-3
    import scipy.linalg as sla
    with monkeypatch.context() as mp:
        mp.setattr(O, "gram_solve", lambda G, g: sla.solve_triangular(G, g, lower=False))
        gb_w, gmu_w = O.total_adjoint(A, L, b, mu, k, s, seed, g_x)
    assert max(_total_fd_errors(A, L, b, mu, k, s, seed, "sparse_sign", g_x, gb_w, gmu_w,
                                np.random.default_rng(7))) > 1e-3


# ----------------------------------------------------------------------------
# planted mistakes: the pins above must catch plausible slips in the oracle
# ----------------------------------------------------------------------------

def test_pins_catch_planted_mistakes(monkeypatch):
    A, L, b, mu = tiny2d(N=8)
    good = O.sgks(A, L, b, mu, 8, 60, 3, keep_history=True)

    # (1) sign slip in the regularisation term of the gradient: the central
    #     difference pin of eq: gradient rejects it, and the sGKS basis built
    #     from it no longer holds the true normalised gradient
    def bad_gradient(A_, L_, b_, mu_, x):
        return A_.T @ (A_ @ x - b_) - mu_ * (L_.T @ (L_ @ x))
    rng = np.random.default_rng(3)
    x = rng.standard_normal(A.shape[1])
    phi = lambda z: 0.5 * (np.linalg.norm(A @ z - b) ** 2 + mu * np.linalg.norm(L @ z) ** 2)
    fd = np.array([(phi(x + 1e-6 * e) - phi(x - 1e-6 * e)) / 2e-6 for e in np.eye(x.size)])
    assert not np.allclose(bad_gradient(A, L, b, mu, x), fd, rtol=1e-6, atol=1e-8)
    true_gradient = O.gradient
    with monkeypatch.context() as mp:
        mp.setattr(O, "gradient", bad_gradient)
        bad = O.sgks(A, L, b, mu, 3, 60, 3, keep_history=True)
    r = true_gradient(A, L, b, mu, bad.x_hist[0])
    assert not np.allclose(bad.W[:, 3], r / np.linalg.norm(r), atol=1e-6)

    # (2) unsketched right-hand side in d_A: d_A = Q_A^T S_A b fails
    orig = O.make_sketches
    with monkeypatch.context() as mp:
        def swapped(m, p, s, seed, zeta=8, kind="sparse_sign"):
            S_A, S_L = orig(m, p, s, seed, zeta, kind)
            return S_A, O.sparse_sign_matrix(p, s, zeta, seed, 0)   # wrong stream for S_L
        mp.setattr(O, "make_sketches", swapped)
        bad = O.sgks(A, L, b, mu, 8, 60, 3)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], 60, 3)
    SLW = S_L @ (L @ bad.W)
    assert not np.allclose(bad.Q_L @ bad.R_L, SLW, atol=1e-8)

    # (3) a transposed operand in the projected solve breaks the lstsq pin
    def bad_solve(R_A, R_L, d_A, mu_):
        d = R_A.shape[0]
        M = np.vstack([R_A.T, math.sqrt(mu_) * R_L])
        y = np.linalg.lstsq(M, np.concatenate([d_A, np.zeros(d)]), rcond=None)[0]
        return y, np.linalg.qr(M)[1]
    with monkeypatch.context() as mp:
        mp.setattr(O, "projected_solve", bad_solve)
        bad = O.sgks(A, L, b, mu, 4, 60, 3)
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], 60, 3)
    M = np.vstack([S_A @ (A @ bad.W), math.sqrt(mu) * (S_L @ (L @ bad.W))])
    y2 = np.linalg.lstsq(M, np.concatenate([S_A @ b, np.zeros(60)]), rcond=None)[0]
    assert np.linalg.norm(bad.y - y2) > 1e-6 * np.linalg.norm(y2)
    assert good.status == O.STATUS_OK


# ----------------------------------------------------------------------------
# residual norms (eq:tik, eq:tik_new_sketched) and the small-factor formula
# ----------------------------------------------------------------------------

def _dense_sparse_sign(h, s, zeta, seed, stream):
    """The s x h sparse-sign embedding built column by column from the scalar
    definition (no call into the oracle's vectorised pattern)."""
    S = np.zeros((s, h))
    for j in range(h):
        rows, signs = _bruteforce_column(j, s, zeta, seed, stream)
        for r, g in zip(rows, signs):
            S[r, j] = g / math.sqrt(zeta)
    return S


def test_tikhonov_residual_is_stacked_least_squares_norm():
    """sqrt(||Ax-b||^2 + mu||Lx||^2) is the norm of [A; sqrt(mu) L] x - [b; 0] (eq:tik);
    at the Tikhonov minimiser it equals sqrt(||b||^2 - b^T A x) (normal equations)."""
    A, L, b, mu = tiny2d(N=7)
    Ad, Ld = A.toarray(), L.toarray()
    M = np.vstack([Ad, math.sqrt(mu) * Ld])
    f = np.concatenate([b, np.zeros(Ld.shape[0])])
    rng = np.random.default_rng(5)
    for x in [rng.standard_normal(A.shape[1]) for _ in range(3)]:
        assert abs(O.tikhonov_residual(A, L, b, mu, x) - np.linalg.norm(M @ x - f)) <= \
            1e-13 * np.linalg.norm(M @ x - f)
    x_star = np.linalg.lstsq(M, f, rcond=None)[0]
    closed = math.sqrt(b @ b - b @ (Ad @ x_star))
    assert abs(O.tikhonov_residual(A, L, b, mu, x_star) - closed) <= 1e-10 * closed


def test_sketched_residual_is_stacked_sketched_norm():
    """eq:tik_new_sketched: sqrt(||S_A(Ax-b)||^2 + mu||S_L L x||^2) equals the norm of
    [S_A A; sqrt(mu) S_L L] x - [S_A b; 0] with S_A, S_L built from the scalar
    definition; with identity sketches it is the Tikhonov residual."""
    A, L, b, mu = tiny2d(N=7)
    s, seed, zeta = 30, 9, 8
    SA = _dense_sparse_sign(A.shape[0], s, zeta, seed, 0)
    SL = _dense_sparse_sign(L.shape[0], s, zeta, seed, 1)
    M = np.vstack([SA @ A.toarray(), math.sqrt(mu) * SL @ L.toarray()])
    f = np.concatenate([SA @ b, np.zeros(s)])
    rng = np.random.default_rng(6)
    for x in [rng.standard_normal(A.shape[1]) for _ in range(3)]:
        ref = np.linalg.norm(M @ x - f)
        assert abs(O.sketched_residual(A, L, b, mu, x, s, seed, zeta) - ref) <= 1e-13 * ref
        ident = O.sketched_residual(A, L, b, mu, x, s, seed, zeta, kind="identity")
        assert abs(ident - O.tikhonov_residual(A, L, b, mu, x)) <= 1e-13 * ident


def test_small_factor_sketched_residual_equals_sketched_residual():
    """At x = W y the sketched residual follows from the small factors alone:
    ||R_A y - d_A||^2 + (||S_A b||^2 - ||d_A||^2) + mu ||R_L y||^2, since
    S_A A W = Q_A R_A, S_L L W = Q_L R_L and d_A = Q_A^T S_A b (eq:updqr,
    eq:dA_update); checked for the sGKS y and for other y."""
    A, L, b, mu = tiny2d(N=10)
    s, seed = 90, 2
    res = O.sgks(A, L, b, mu, 9, s, seed)
    rng = np.random.default_rng(7)
    for y in [res.y] + [rng.standard_normal(res.y.size) for _ in range(3)]:
        small2 = (np.linalg.norm(res.R_A @ y - res.d_A) ** 2
                  + (res.c_b @ res.c_b - res.d_A @ res.d_A)
                  + mu * np.linalg.norm(res.R_L @ y) ** 2)
        ref = O.sketched_residual(A, L, b, mu, res.W @ y, s, seed)
        assert abs(math.sqrt(small2) - ref) <= 1e-11 * ref


# ----------------------------------------------------------------------------
# heavy-ball refinement weights
# ----------------------------------------------------------------------------

def test_refinement_two_steps_worked_by_hand():
    """Two heavy-ball steps on a 1 x 1 problem, values worked out by hand:
    A = 2, L = 1, b = 4, mu = 1, W = 1, G = 2, d / s = 1 / 4 so eta^2 = 1/4,
    alpha = (1 - 1/4)^2 = 9/16, beta = 1/4.  r(y) = A^T(Ay - b) + mu L^T L y
    = 5y - 8, delta = r / G^2 = (5y - 8) / 4.
      y0 = 1:        delta0 = -3/4,        y1 = 1 + (9/16)(3/4)            = 1.421875
      y1:            delta1 = -57/256,     y2 = y1 + (9/16)(57/256) + (1/4)(y1 - y0)
                                               = 1.652587890625
    (fixed point 8/5)."""
    A = sp.csr_matrix(np.array([[2.0]]))
    L = sp.csr_matrix(np.array([[1.0]]))
    b = np.array([4.0])
    W = np.array([[1.0]])
    G = np.array([[2.0]])
    y1 = O.refine(A, L, b, 1.0, W, np.array([1.0]), G, 4, 1)
    y2 = O.refine(A, L, b, 1.0, W, np.array([1.0]), G, 4, 2)
    assert y1[0] == 1.421875
    assert y2[0] == 1.652587890625
    assert O.refinement_weights(1, 4) == (0.5625, 0.25)


def test_refinement_weights_give_the_optimal_heavy_ball_rate():
    """With the preconditioned spectrum in [1/(1+eta)^2, 1/(1-eta)^2] (singular values
    of the sketched basis in [1-eta, 1+eta]), Polyak's optimal step and momentum are
    alpha = 4/(sqrt(l_max) + sqrt(l_min))^2 = (1-eta^2)^2 and
    beta = ((sqrt(l_max) - sqrt(l_min))/(sqrt(l_max) + sqrt(l_min)))^2 = eta^2, and the
    error contracts like eta^k; a diagonal system with both extremes shows it."""
    d, s = 4, 25
    eta = math.sqrt(d / s)
    lam = np.array([1 / (1 + eta) ** 2, 1 / (1 - eta) ** 2, 1.0, 0.9])
    lmin, lmax = lam.min(), lam.max()
    a_opt = 4 / (math.sqrt(lmax) + math.sqrt(lmin)) ** 2
    b_opt = ((math.sqrt(lmax) - math.sqrt(lmin)) / (math.sqrt(lmax) + math.sqrt(lmin))) ** 2
    alpha, beta = O.refinement_weights(d, s)
    assert abs(alpha - a_opt) <= 1e-15 and abs(beta - b_opt) <= 1e-15
    # the oracle's refine() on this system: A = diag(sqrt(lam)), L = 0, W = I, G = I,
    # so W^T r(y) = lam * y - sqrt(lam) * b and the solution is b / sqrt(lam)
    A = sp.diags(np.sqrt(lam)).tocsr()
    L = sp.csr_matrix((1, d))
    b = np.ones(d)
    y_star = b / np.sqrt(lam)
    e0 = np.linalg.norm(np.zeros(d) - y_star)
    k = 40
    y = O.refine(A, L, b, 1.0, np.eye(d), np.zeros(d), np.eye(d), s, k)
    rate = (np.linalg.norm(y - y_star) / e0) ** (1.0 / k)
    assert rate <= 1.1 * eta
    # a wrong momentum (beta = 0, plain preconditioned Richardson) is slower
    with pytest.MonkeyPatch().context() as mp:
        mp.setattr(O, "refinement_weights", lambda d_, s_: (alpha, 0.0))
        y_r = O.refine(A, L, b, 1.0, np.eye(d), np.zeros(d), np.eye(d), s, k)
    assert np.linalg.norm(y_r - y_star) > 10 * np.linalg.norm(y - y_star)


# ----------------------------------------------------------------------------
# sketch size: sGKS approaches GKS as s grows (Sec. 4.1)
# ----------------------------------------------------------------------------

def test_sgks_approaches_gks_as_sketch_grows():
    """Sec. 4.1: the reconstruction of sGKS approaches that of GKS as the sketch size
    grows; over s in {2d, 4d, 16d} (d = ell + k) and three sketch seeds the mean
    distance ||x_sGKS - x_GKS|| / ||x_GKS|| and the mean |RRE_sGKS - RRE_GKS| fall."""
    from workloads import make
    P = make("deblur1d", 0, "small")
    d = P.ell + P.k
    g = O.gks(P.A, P.L, P.b, P.mu, P.k)
    rre = lambda x: np.linalg.norm(x - P.x_true) / np.linalg.norm(P.x_true)
    dist, gap = [], []
    for s in (2 * d, 4 * d, 16 * d):
        xs = [O.sgks(P.A, P.L, P.b, P.mu, P.k, s, seed).x for seed in (0, 1, 2)]
        dist.append(np.mean([np.linalg.norm(x - g.x) / np.linalg.norm(g.x) for x in xs]))
        gap.append(np.mean([abs(rre(x) - rre(g.x)) for x in xs]))
    assert dist[0] > dist[1] > dist[2]
    assert gap[0] > gap[2]
    assert dist[2] < 0.5 * dist[0]


# ----------------------------------------------------------------------------
# SRTT (eq:sketching_trig)
# ----------------------------------------------------------------------------

def _srtt_dense_by_definition(h, s, seed, stream):
    """S = sqrt(h/s) D F E written out entry by entry: DCT-II cosines from their formula,
    signs and rows from scalar SplitMix64 loops (Python integers mod 2^64)."""
    mask = (1 << 64) - 1
    g = 0x9E3779B97F4A7C15
    mix = lambda z: int(O.mix64(np.uint64(z & mask)))
    ks = mix(seed + g * (stream + 3))
    E = [(-1.0 if mix(ks + g * (i + 1)) & 1 else 1.0) for i in range(h)]
    kr = mix(seed + g * (stream + 1))
    rows, c = [], 0
    while len(rows) < s:
        z = mix(kr + g * (c + 1))
        c += 1
        r = ((z >> 32) * h) >> 32
        if r not in rows:
            rows.append(r)
    S = np.zeros((s, h))
    for j, k in enumerate(rows):
        ck = math.sqrt((1.0 if k == 0 else 2.0) / h)
        for i in range(h):
            S[j, i] = math.sqrt(h / s) * ck * math.cos(math.pi * k * (2 * i + 1) / (2 * h)) * E[i]
    return S


@pytest.mark.parametrize("h,s,seed,stream", [(24, 10, 0, 0), (37, 37, 5, 1), (64, 9, 3, 0)])
def test_srtt_matches_its_definition(h, s, seed, stream):
    """The oracle's SRTT (fast DCT) equals the matrix written from eq:sketching_trig."""
    S = O.SRTT(h, s, seed, stream)
    M = _srtt_dense_by_definition(h, s, seed, stream)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(h)
    V = rng.standard_normal((h, 3))
    w = rng.standard_normal(s)
    assert np.allclose(S @ v, M @ v, rtol=0, atol=1e-12 * np.linalg.norm(M @ v))
    assert np.allclose(S @ V, M @ V, rtol=0, atol=1e-12 * np.linalg.norm(M @ V))
    assert np.allclose(S.T @ w, M.T @ w, rtol=0, atol=1e-12 * np.linalg.norm(M.T @ w))


def test_srtt_full_selection_is_orthogonal():
    """With s = h every frequency is kept and S = D F E is orthogonal (F and E are)."""
    h = 50
    S = O.SRTT(h, h, 7, 0)
    M = S @ np.eye(h)
    assert np.allclose(M.T @ M, np.eye(h), atol=1e-13)


def test_srtt_is_isometric_in_expectation_and_embeds():
    """E ||S x||^2 = ||x||^2 over the random signs and rows; for s well above a subspace's
    dimension the embedding distortion of Def. 1 is below one."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal(400)
    ratios = [np.linalg.norm(O.SRTT(400, 40, sd, 0) @ x) ** 2 / (x @ x) for sd in range(300)]
    assert abs(np.mean(ratios) - 1.0) < 0.03
    Q, _ = np.linalg.qr(rng.standard_normal((400, 5)))
    assert O.embedding_epsilon(O.SRTT(400, 200, 2, 0), Q) < 0.9


def test_sgks_with_srtt_satisfies_prop2():
    """Prop. 2 (max form) with SRTT sketches, eps measured on range([A W, b]), range(L W)."""
    A, L, b, mu = tiny2d(N=10)
    s, seed = 60, 4
    res = O.sgks(A, L, b, mu, 8, s, seed, sketch="srtt")
    S_A, S_L = O.make_sketches(A.shape[0], L.shape[0], s, seed, kind="srtt")
    W = res.W
    eps = max(_eps(S_A, np.column_stack([A @ W, b])), _eps(S_L, L @ W))
    assert eps < 1
    phi = lambda y: np.linalg.norm(A @ W @ y - b) ** 2 + mu * np.linalg.norm(L @ W @ y) ** 2
    y0 = O.unsketched_projected_solution(A, L, b, mu, W)
    assert phi(res.y) <= (1 + eps) / (1 - eps) * phi(y0) * (1 + 1e-12)
    # Q_A R_A = S_A A W with the SRTT
    assert np.allclose(res.Q_A @ res.R_A, S_A @ (A @ W), atol=1e-10)
