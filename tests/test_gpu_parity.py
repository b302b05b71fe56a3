"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances.  The FP64-operator path agrees with the oracle to rounding order;
the sGKS recursion amplifies rounding differences as the basis loses rank
(kappa(R_A) grows to 1e7-1e11 by k = 100 at the deblurring workload), so
trajectory parity is asserted per workload at the tolerance stated in the
test, and every workload is also checked at full k through relations that hold
for any rounding (the factors are factors of the GPU's own basis, y solves the
projected problem built from them, the new column is the normalised gradient).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402
from workloads import generators as gen  # noqa: E402
from workloads import make  # noqa: E402


from gpu_common import (KAPPA_TRUSTED, check_state_consistency, cond_at,  # noqa: E402
                        oracle_history_async, oracle_run, problem, rel, say, wait_ref)

# full-size oracle trajectories, computed in worker processes while the other
# tests run; each also on its problem with the unknowns permuted (the same
# iteration with another rounding order), which measures how far two FP64
# evaluations of the iteration drift apart at each k
CT_CHECK = (40, 80, 120, 149, 150)
DYN_CHECK = (20, 50, 100, 150, 160, 199, 200)
_REF_CT = oracle_history_async(("ct2d", "full", 0), 150, CT_CHECK)
_REF_CT_P = oracle_history_async(("ct2d", "full", 0), 150, CT_CHECK, permute=1)
_REF_DYN = oracle_history_async(("dynamic_ct", "full", 0), 200, DYN_CHECK)
_REF_DYN_P = oracle_history_async(("dynamic_ct", "full", 0), 200, DYN_CHECK, permute=1)


# ----------------------------------------------------------------------------

def test_smoke_small_fp64_parity():
    P = problem("deblur1d", "small")
    say("case deblur1d small", P.n, P.k)
    S, x = G.solve_problem(P)
    ref = oracle_run(P)
    e = rel(x.cpu().numpy(), ref.x)
    say("rel err", e)
    assert e <= 1e-10
    rc, it = S.status()
    assert rc == 0 and it == P.k
    S.close()


def test_deblur1d_full_fp64_trajectory():
    """1D deblurring, dense 256x256 blur, FP64, k = 30: x_k within 1e-10 of the oracle."""
    P = problem("deblur1d", "full")
    say("case deblur1d full", P.n, P.k)
    ref = oracle_run(P, keep_history=True)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    for k in range(0, P.k + 1, 5):
        if k:
            S.iterate(5)
        x = S.solution().cpu().numpy()
        e = rel(x, ref.x_hist[k])
        say(f"  k={k} rel err {e:.3e}")
        assert e <= 1e-10
    check_state_consistency(S, P)
    rre_gpu = rel(x, P.x_true)
    rre_ref = rel(ref.x, P.x_true)
    assert abs(rre_gpu - rre_ref) <= 1e-8 * rre_ref
    S.close()


def test_sketch_of_b_is_bit_pattern_exact():
    """S_A b from the GPU hash equals the oracle's sparse-sign matrix product."""
    for name in ("deblur1d", "deblur2d", "ct2d"):
        P = problem(name, "small")
        say("case sketch", name)
        A, L, b = G.upload_problem(P)
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
        cb = S.state("c_b")
        S_A, _ = O.make_sketches(P.m, P.p, P.s, P.seed, P.zeta)
        ref = S_A @ P.b
        assert np.max(np.abs(cb - ref)) <= 1e-13 * np.max(np.abs(ref))
        S.close()


@pytest.mark.parametrize("zeta", [2, 4, 16])
def test_other_zeta(zeta):
    P = problem("deblur2d", "small")
    say("case zeta", zeta)
    S, x = G.solve_problem(P, k=8, zeta=zeta)
    ref = O.sgks(P.A, P.L, P.b, P.mu, 8, P.s, P.seed, zeta=zeta)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-9
    S.close()


@pytest.mark.parametrize("name", ["deblur2d", "ct2d", "dynamic_ct"])
def test_small_configs_trajectory(name):
    """Reduced-size workloads (several tiles, ragged tails), FP32 operators, full small k."""
    P = problem(name, "small")
    say("case small", name, P.n, P.m, P.p, P.k, P.refine_steps)
    ref = oracle_run(P)
    S, x = G.solve_problem(P)
    e = rel(x.cpu().numpy(), ref.x)
    say("  rel err", e)
    assert e <= 1e-8
    check_state_consistency(S, P)
    S.close()


@pytest.mark.parametrize("s", [40, 64, 65, 200, 300, 520, 1000])
def test_sketch_sizes_one_workgroup_append(s):
    """Sketch sizes around the row-chunk and register-count boundaries of the
    one-workgroup appends (s <= 256, <= 512, <= 1024; one and several 64-row
    chunks, ragged last chunk), trajectory and factor relations."""
    import dataclasses
    P = dataclasses.replace(problem("deblur2d", "small"), s=s)
    k = 12
    say("case sketch size", s, "k", k)
    ref = O.sgks(P.A, P.L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell)
    S, x = G.solve_problem(P, k=k, append_groups=1)
    assert S.tuning()["append_groups"] == 1   # the one-workgroup append ran
    e = rel(x.cpu().numpy(), ref.x)
    say("  rel err", e)
    assert e <= 1e-8
    check_state_consistency(S, P)
    S.close()


def _ragged_problem():
    """A 1003 x 997 random sparse operator (FP64) with ten empty rows and seven
    empty columns, first differences with two empty rows: every size off the
    tile grids."""
    import scipy.sparse as sp
    from workloads.generators import Problem
    rng = np.random.default_rng(11)
    m, n = 1003, 997
    A = sp.random(m, n, density=0.02, random_state=rng, format="csr", dtype=np.float64)
    keep_r = np.ones(m)
    keep_r[rng.choice(m, 10, replace=False)] = 0.0
    keep_c = np.ones(n)
    keep_c[rng.choice(n, 7, replace=False)] = 0.0
    A = (sp.diags(keep_r) @ A @ sp.diags(keep_c)).tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    D = sp.diags([-np.ones(n - 1), np.ones(n - 1)], [0, 1], shape=(n - 1, n), format="csr")
    keep_l = np.ones(n - 1)
    keep_l[[5, 500]] = 0.0
    L = (sp.diags(keep_l) @ D).tocsr()
    L.eliminate_zeros()
    L.sort_indices()
    x_true = rng.standard_normal(n)
    b = A @ x_true + 0.01 * rng.standard_normal(m)
    assert np.count_nonzero(np.diff(A.indptr) == 0) >= 10
    assert np.count_nonzero(np.diff(L.indptr) == 0) == 2
    return Problem("ragged", A, L, b, x_true, mu=1e-2, k=15, s=150, seed=5, dtype="f64")


def test_ragged_operator_with_empty_rows_and_columns():
    P = _ragged_problem()
    say("case ragged", P.m, P.n, P.p, "nnz", P.A.nnz)
    ref = oracle_run(P)
    S, x = G.solve_problem(P)
    kap = cond_at(ref, P, P.k)
    e = rel(x.cpu().numpy(), ref.x)
    say(f"  rel err {e:.3e} kappa {kap:.2e}")
    assert kap <= KAPPA_TRUSTED
    assert e <= max(1e-10, 1e-15 * kap * 10)
    check_state_consistency(S, P)
    S.close()


@pytest.mark.parametrize("s,k", [(346, 343), (512, 509)])
def test_max_basis_size(s, k):
    """The largest bases on the small 2D deblurring operators: ell + k = 346 = s,
    the largest one-workgroup append (s d_max <= 120000, s >= d_max), and
    ell + k = 512 = s, the largest basis, on the append chain.  Trajectory while
    the projected problem is trustworthy in FP64; at the end the factor
    relations Q R = S A W (which hold also once sketched columns turn
    numerically dependent)."""
    import dataclasses
    P = dataclasses.replace(problem("deblur2d", "small"), s=s, k=k)
    say("case max basis", s)
    ref = oracle_run(P, keep_history=True)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    groups = S.tuning()["append_groups"]
    assert (groups == 1) if s * (P.ell + P.k) <= 120000 else (groups > 1)
    done = 0
    checked = 0
    for kk in (20, 60, 150, 300, k):
        if kk > k:
            break
        S.iterate(kk - done)
        done = kk
        rc, it = S.status()
        if rc != 0:
            say("  stopped", rc, it)
            assert rc == G.BREAKDOWN
            break
        kap = cond_at(ref, P, kk)
        if kap <= KAPPA_TRUSTED:
            e = rel(S.solution().cpu().numpy(), ref.x_hist[kk])
            say(f"  k={kk} rel err {e:.3e} kappa {kap:.2e}")
            assert e <= 1e-5
            checked += 1
    assert checked >= 1
    W = S.state("W")
    d = W.shape[1]
    say("  basis size", d, "oracle", P.ell + ref.iters)
    assert P.ell + 60 <= d <= P.ell + P.k
    QA, RA, QL, RL = S.state("Q_A"), S.state("R_A"), S.state("Q_L"), S.state("R_L")
    S_A, S_L = O.make_sketches(P.m, P.p, P.s, P.seed, P.zeta)
    SAW, SLW = S_A @ (P.A @ W), S_L @ (P.L @ W)
    assert np.linalg.norm(QA @ RA - SAW) <= 1e-9 * np.linalg.norm(SAW)
    assert np.linalg.norm(QL @ RL - SLW) <= 1e-9 * np.linalg.norm(SLW)
    assert np.allclose(np.triu(RA), RA) and np.allclose(np.triu(RL), RL)
    S.close()


@pytest.mark.parametrize("groups,refine,form", [(1, 0, "maintained"), (4, 1, "maintained"),
                                                (1, 1, "direct")])
def test_profiling_times_kernels_and_keeps_results(groups, refine, form):
    """Profiled iterations run kernel by kernel, each launch carrying events bound
    to the kernel: the same bits as graph replays, one count per kernel launched."""
    P = problem("deblur2d", "small")
    k = 12
    say("case profiling, append groups", groups, "refine", refine, form)
    A, L, b = G.upload_problem(P)
    kw = dict(max_iters=k, append_groups=groups, refine_steps=refine, gradient=form)
    S1 = G.SGKS(A, L, b, P.mu, P.s, P.seed, **kw)
    S1.profile(True).iterate(k)
    x1 = S1.solution().cpu().numpy()
    ms, cnt = S1.profile_read()
    S2 = G.SGKS(A, L, b, P.mu, P.s, P.seed, graph=True, **kw)
    S2.iterate(k)
    x2 = S2.solution().cpu().numpy()
    assert np.array_equal(x1, x2)
    n = {name: cnt[i] for i, name in enumerate(G.PHASE_NAMES)}
    say("  launches", n)
    assert n["spmv_new_column"] == k and n["sketch_scatter"] == k
    if form == "maintained":
        # one gradient launch per expansion, plus x = W y; the H W column inside the
        # compact append's launch, else in an adjoint launch of its own; with
        # refinement one launch for the new column of W^T H W and one for all the
        # steps of an expansion
        assert n["gemv"] == k + 1
        assert n["gemvt_WTr"] == k * min(refine, 1) and n["refine_step"] == k * min(refine, 1)
        assert n["forward_Ax_Lx"] == 0
        assert n["adjoint"] == (0 if groups == 1 else k)
    else:
        assert n["gemvt_WTr"] == k * refine and n["refine_step"] == k * refine
        assert n["gemv"] == k * (1 + refine) + 1
        assert n["forward_Ax_Lx"] == k * (1 + refine) and n["adjoint"] == k * (1 + refine)
    if groups == 1 and form == "maintained":
        assert n["qr_append_solve"] == k   # the compact append is one launch
    else:
        assert n["qr_append_solve"] >= k and n["qr_append_solve"] % k == 0
    assert all(v >= 0 for v in ms) and ms[G.PHASE_NAMES.index("spmv_new_column")] > 0
    # a second read starts from zero
    ms2, cnt2 = S1.profile_read()
    assert all(c == 0 for c in cnt2)
    S1.close()
    S2.close()


@pytest.mark.parametrize("groups", [1, 4])
def test_single_projection_append(groups):
    """qr_passes = 1: one CGS projection per column append, as the rank-one QR
    update is written in Sec. 2.1, on the one-workgroup append and the chain."""
    P = problem("deblur2d", "small")
    k = 16
    say("case single projection, append groups", groups)
    ref = O.sgks(P.A, P.L, P.b, P.mu, k, P.s, P.seed, zeta=P.zeta, ell=P.ell, qr_passes=1)
    S, x = G.solve_problem(P, k=k, qr_passes=1, append_groups=groups)
    assert S.tuning()["append_groups"] == groups
    e = rel(x.cpu().numpy(), ref.x)
    say("  rel err", e)
    assert e <= 1e-8
    S.close()


def test_identity_sketch_is_gks_prop1():
    """Prop. 1 on the GPU: with identity sketches the iterates are the GKS iterates."""
    P = problem("deblur1d", "small")
    s = max(P.m, P.p)
    say("case identity sketch", s)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, s, 0, max_iters=12, sketch="identity")
    g = O.gks(P.A, P.L, P.b, P.mu, 12, keep_history=True)
    for k in range(0, 13, 4):
        if k:
            S.iterate(4)
        assert rel(S.solution().cpu().numpy(), g.x_hist[k]) <= 1e-10
    S.close()


def test_resume_and_determinism():
    P = problem("deblur2d", "small")
    say("case resume/determinism")
    A, L, b = G.upload_problem(P)
    S1 = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    S1.iterate(7).iterate(P.k - 7)
    S2 = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    S2.iterate(P.k)
    x1 = S1.solution().cpu().numpy()
    x2 = S2.solution().cpu().numpy()
    assert np.array_equal(x1, x2)           # bitwise: fixed reduction orders
    S1.close()
    S2.close()


def test_residual_norms():
    P = problem("deblur2d", "small")
    say("case residual norms")
    S, x = G.solve_problem(P)
    tn, sn = S.residual_norm()
    xh = x.cpu().numpy()
    assert abs(tn - O.tikhonov_residual(P.A, P.L, P.b, P.mu, xh)) <= 1e-10 * tn
    ref_s = O.sketched_residual(P.A, P.L, P.b, P.mu, xh, P.s, P.seed, P.zeta)
    assert abs(sn - ref_s) <= 1e-8 * ref_s
    S.close()


def test_capacity_and_errors():
    P = problem("deblur1d", "small")
    say("case errors")
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=5)
    with pytest.raises(G.SgksError) as e:
        S.iterate(6)
    assert e.value.code == -5
    S.iterate(5)
    S.close()
    with pytest.raises(G.SgksError) as e:
        G.SGKS(A, L, torch.zeros_like(b), P.mu, P.s, P.seed, max_iters=5)
    assert e.value.code == -6
    bn = b.clone()
    bn[3] = float("nan")
    with pytest.raises(G.SgksError) as e:
        G.SGKS(A, L, bn, P.mu, P.s, P.seed, max_iters=5)
    assert e.value.code == -7


def _identity_problem(n=64):
    import scipy.sparse as sp
    I = sp.identity(n, format="csr")
    I.indices = I.indices.astype(np.int32)
    I.indptr = I.indptr.astype(np.int32)
    bh = np.linspace(1.0, 2.0, n)
    return G.DeviceCsr.from_scipy(I), torch.as_tensor(bh, device="cuda"), bh


def test_breakdown_invariant_subspace():
    """A = L = I, identity sketch: K_1(A^T A, A^T b) = span{b} holds the solution, r = 0."""
    A, b, bh = _identity_problem()
    say("case breakdown (invariant subspace)")
    S = G.SGKS(A, A, b, 0.5, 64, 0, ell=1, max_iters=4, sketch="identity")
    S.iterate(4)
    rc, it = S.status()
    assert rc == G.BREAKDOWN and it == 0
    assert np.allclose(S.solution().cpu().numpy(), bh / 1.5)
    S.close()


def test_breakdown_dependent_column_matches_oracle():
    """A = L = I, sparse sign: the new column repeats w_1; both sides stop at once."""
    A, b, bh = _identity_problem()
    say("case breakdown (dependent column)")
    S = G.SGKS(A, A, b, 0.5, 16, 0, ell=1, max_iters=4)
    S.iterate(4)
    rc, it = S.status()
    import scipy.sparse as sp
    ref = O.sgks(sp.identity(64, format="csr"), sp.identity(64, format="csr"), bh, 0.5, 4, 16, 0,
                 ell=1)
    assert ref.status == O.STATUS_BREAKDOWN and ref.iters == 0
    assert rc == G.BREAKDOWN and it == 0
    assert rel(S.solution().cpu().numpy(), ref.x) <= 1e-12
    S.close()


def test_degenerate_initial_space_is_rejected():
    A, b, bh = _identity_problem()
    say("case degenerate initial space")
    with pytest.raises(G.SgksError) as e:
        G.SGKS(A, A, b, 0.5, 16, 0, ell=3, max_iters=4)
    assert e.value.code == -10


def test_refinement_small():
    """Heavy-ball iterative refinement of every projected solve (CT, 2 steps)."""
    P = problem("ct2d", "small")
    assert P.refine_steps == 2
    say("case refinement")
    ref = oracle_run(P)
    S, x = G.solve_problem(P)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    S.close()


def test_backward_with_refinement_is_refused():
    """The adjoint is that of the unrefined projected solve: a context with refinement
    steps refuses sgks_backward, and the autograd function refuses to record."""
    P = problem("ct2d", "small")
    assert P.refine_steps > 0
    say("case backward with refinement")
    S, x = G.solve_problem(P, k=3)
    with pytest.raises(G.SgksError) as e:
        S.backward(torch.zeros_like(x))
    assert e.value.code == -1
    S.close()
    A, L, b = G.upload_problem(P)
    bg = b.clone().requires_grad_(True)
    with pytest.raises(ValueError):
        G.sgks_solve(A, L, bg, P.mu, P.s, 3, P.seed, refine_steps=P.refine_steps)


def test_backward_small_matches_oracle_adjoint():
    P = problem("dynamic_ct", "small")
    say("case backward")
    ref = oracle_run(P)
    S, x = G.solve_problem(P)
    xh = x.cpu().numpy()
    g_x = 2 * (xh - P.x_true)
    gb, gmu = S.backward(torch.as_tensor(g_x, device="cuda"))
    W = S.state("W")
    res = O.Result(xh, S.state("y"), W, S.state("Q_A"), S.state("R_A"), S.state("Q_L"),
                   S.state("R_L"), S.state("d_A"), S.state("G"), S.state("c_b"), P.k, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(res, P.mu, g_x, P.A, P.L, P.s, P.seed, P.zeta)
    assert rel(gb.cpu().numpy(), gb_ref) <= 1e-8
    assert abs(gmu - gmu_ref) <= 1e-8 * abs(gmu_ref)
    # and against the oracle's own run (same trajectory at this size)
    gb_o, gmu_o = O.frozen_adjoint_b(ref, P.mu, 2 * (ref.x - P.x_true), P.A, P.L, P.s, P.seed,
                                     P.zeta)
    assert rel(gb.cpu().numpy(), gb_o) <= 1e-6
    S.close()


# ----------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times
# ----------------------------------------------------------------------------

def check_new_column_is_gradient(S, P, steps=1, form="maintained"):
    """After one more expansion, the new column is r(x_prev)/||r(x_prev)|| (eq: gradient).

    The direct form evaluates r from x and agrees to 1e-10.  The maintained form
    evaluates r = (H W) y - A^T b, a sum of d + 1 FP64 terms that cancel down to
    ||r||; its error bound d eps (sum_j |y_j| ||H w_j|| + ||A^T b||) / ||r|| is
    computed here from the GPU's own basis."""
    x_prev = S.solution().cpu().numpy()
    W_prev, y_prev = S.state("W"), S.state("y")
    S.iterate(steps)
    W = S.state("W")
    r = O.gradient(P.A, P.L, P.b, P.mu, x_prev)
    w = r / np.linalg.norm(r)
    tol = 1e-10
    if form == "maintained":
        HW = P.A.T @ (P.A @ W_prev) + P.mu * (P.L.T @ (P.L @ W_prev))
        terms = np.sum(np.abs(y_prev) * np.linalg.norm(HW, axis=0)) + np.linalg.norm(P.A.T @ P.b)
        d = W_prev.shape[1]
        tol = max(tol, d * 2.2e-16 * terms / np.linalg.norm(r))
    e = rel(W[:, -1], w)
    say(f"  new column vs gradient {e:.2e} (bound {tol:.2e})")
    assert e <= tol


def test_deblur2d_full_trajectory_and_consistency():
    """2D deblurring n = 65536, FP32 operators, k = 100: x_k within 1e-5 of the oracle."""
    P = problem("deblur2d", "full")
    say("case deblur2d full", P.n, P.k)
    ref = oracle_run(P, keep_history=True)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    done = 0
    for k in (10, 40, 99):
        S.iterate(k - done)
        done = k
        e = rel(S.solution().cpu().numpy(), ref.x_hist[k])
        say(f"  k={k} rel err {e:.3e}")
        assert e <= (1e-9 if k <= 10 else 1e-5)
    check_new_column_is_gradient(S, P)
    x = S.solution().cpu().numpy()
    e = rel(x, ref.x)
    say(f"  k={P.k} rel err {e:.3e}  RRE gpu {rel(x, P.x_true):.6f} oracle {rel(ref.x, P.x_true):.6f}")
    assert e <= 1e-5
    check_state_consistency(S, P)
    S.close()


def _trajectory_against(S, P, ref_async, perm_async, checkpoints, tol):
    """Iterate S to each checkpoint and compare x_k with the oracle's x_k; the last
    expansion goes through check_new_column_is_gradient.  At the configured k the
    bound is tol.  Along the way it is max(tol, 10 e_k), e_k the distance between the
    oracle and the oracle run with permuted unknowns: where two FP64 evaluations of
    the iteration itself are e_k apart, no evaluation can be held closer to one of them."""
    hist, kap, iters, status = wait_ref(ref_async, P.name)
    hist_p, _, iters_p, _ = wait_ref(perm_async, P.name + " (permuted)")
    assert iters == iters_p == P.k and status == O.STATUS_OK
    done = 0
    for k in checkpoints:
        if k == P.k:
            check_new_column_is_gradient(S, P)
        else:
            S.iterate(k - done)
        done = k
        e = rel(S.solution().cpu().numpy(), hist[k])
        e_k = rel(hist_p[k], hist[k])
        bound = tol if k == P.k else max(tol, 10 * e_k)
        say(f"  k={k} kappa {kap[k]:.2e} rel err {e:.3e} (oracle vs permuted oracle "
            f"{e_k:.3e}, bound {bound:.1e})")
        assert e <= bound, (k, e, e_k, kap[k])
    rc, it = S.status()
    assert rc == 0 and it == P.k


@pytest.mark.timeout(900)
def test_ct2d_full_refined():
    """CT 256^2, 180 x 362 rays, FP32 operators, 2 refinement steps per solve: x_k against
    the oracle along the whole run, k = 40 ... 150; 1e-5 (the FP32-operator bound) at the
    configured output k = 150."""
    P = problem("ct2d", "full")
    say("case ct2d full", P.n, P.m, P.k)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k, refine_steps=P.refine_steps)
    _trajectory_against(S, P, _REF_CT, _REF_CT_P, CT_CHECK, 1e-5)
    check_state_consistency(S, P)
    x = S.solution().cpu().numpy()
    hist, *_ = wait_ref(_REF_CT)
    say(f"  k={P.k} RRE gpu {rel(x, P.x_true):.7f} oracle {rel(hist[P.k], P.x_true):.7f} "
        f"(grows with k on this workload: the oracle's own RRE rises from k = 20 on)")
    S.close()


@pytest.mark.timeout(900)
def test_dynamic_ct_full():
    """Dynamic CT 30 x 128^2 frames, block-diagonal A, space-time L, k = 200: x_k against
    the oracle along the whole run, k = 20 ... 200; 1e-5 at the configured output."""
    P = problem("dynamic_ct", "full")
    say("case dynamic_ct full", P.n, P.m, P.p, P.k)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k)
    _trajectory_against(S, P, _REF_DYN, _REF_DYN_P, DYN_CHECK, 1e-5)
    check_state_consistency(S, P)
    x = S.solution().cpu().numpy()
    hist, *_ = wait_ref(_REF_DYN)
    say(f"  k={P.k} RRE gpu {rel(x, P.x_true):.7f} oracle {rel(hist[P.k], P.x_true):.7f}")
    S.close()


# ----------------------------------------------------------------------------
# differentiation
# ----------------------------------------------------------------------------

def test_autograd_function_matches_backward():
    P = problem("dynamic_ct", "small")
    say("case autograd small")
    A, L, b = G.upload_problem(P)
    bg = b.clone().requires_grad_(True)
    mu = torch.tensor(P.mu, dtype=torch.float64, device="cuda", requires_grad=True)
    xt = torch.as_tensor(P.x_true, device="cuda")
    x = G.sgks_solve(A, L, bg, mu, P.s, P.k, P.seed)
    loss = ((x - xt) ** 2).sum()
    loss.backward()
    S, x2 = G.solve_problem(P)
    gb, gmu = S.backward(2 * (x2 - xt))
    assert torch.equal(x.detach(), x2)
    assert torch.allclose(bg.grad.double(), gb.to(bg.dtype).double(), rtol=0, atol=0)
    assert abs(mu.grad.item() - gmu) <= 1e-12 * abs(gmu)
    S.close()


def test_backward_is_true_derivative_at_full_space():
    """At d = n the frozen-basis adjoint is the derivative of the whole solve: compare
    with central differences of the GPU pipeline itself."""
    A_ = gen.blur1d_dense(8, 0.8)
    L_ = gen.diff1d(8)
    rng = np.random.default_rng(1)
    xt_ = gen.step_signal(8, rng)
    b_ = gen.add_noise(A_ @ xt_, 0.01, rng)
    mu_, s_, seed_ = 1e-2, 100, 5
    A, L = G.DeviceCsr.from_scipy(A_), G.DeviceCsr.from_scipy(L_)
    xt = torch.as_tensor(xt_, device="cuda")
    say("case full-space derivative")

    def loss_of(bv, mv):
        x = G.sgks_solve(A, L, bv, mv, s_, 5, seed_)
        return ((x - xt) ** 2).sum()

    bg = torch.as_tensor(b_, device="cuda").requires_grad_(True)
    mu = torch.tensor(mu_, dtype=torch.float64, device="cuda", requires_grad=True)
    loss_of(bg, mu).backward()
    h = 1e-6
    for i in range(8):
        e = torch.zeros(8, dtype=torch.float64, device="cuda")
        e[i] = h
        bb = torch.as_tensor(b_, device="cuda")
        fd = (loss_of(bb + e, mu_).item() - loss_of(bb - e, mu_).item()) / (2 * h)
        assert abs(fd - bg.grad[i].item()) <= 1e-5 * max(1.0, abs(fd)), (i, fd, bg.grad[i].item())
    hm = 1e-6 * mu_
    bb = torch.as_tensor(b_, device="cuda")
    fdm = (loss_of(bb, mu_ + hm).item() - loss_of(bb, mu_ - hm).item()) / (2 * hm)
    assert abs(fdm - mu.grad.item()) <= 1e-5 * max(1.0, abs(fdm))


def test_backward_dynamic_ct_full_size():
    """Dynamic CT 30 x 128^2 (n = 491,520): GPU adjoint vs the oracle's frozen adjoint on the
    GPU's own basis and factors (k = 30)."""
    P = problem("dynamic_ct", "full")
    k = 30
    say("case backward full", P.n, P.m, k)
    S, x = G.solve_problem(P, k=k)
    xt = torch.as_tensor(P.x_true, device="cuda")
    gb, gmu = S.backward(2 * (x - xt))
    xh = x.cpu().numpy()
    res = O.Result(xh, S.state("y"), S.state("W"), S.state("Q_A"), S.state("R_A"),
                   S.state("Q_L"), S.state("R_L"), S.state("d_A"), S.state("G"),
                   S.state("c_b"), k, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(res, P.mu, 2 * (xh - P.x_true), P.A, P.L, P.s, P.seed,
                                         P.zeta)
    e = rel(gb.cpu().numpy(), gb_ref)
    say(f"  grad_b rel err {e:.3e}, grad_mu {gmu:.6e} vs {gmu_ref:.6e}")
    assert e <= 1e-8
    assert abs(gmu - gmu_ref) <= 1e-8 * abs(gmu_ref)
    S.close()


@pytest.mark.parametrize("name", ["deblur2d", "ct2d"])
def test_gradient_forms_agree(name):
    """The maintained H W gradient and the direct A^T (A x - b) + mu L^T L x gradient
    give the same iterates (to rounding) and both match the oracle; ct2d also runs
    its two refinement steps per solve through each form."""
    P = problem(name, "small")
    say("case gradient forms", name, P.k, P.refine_steps)
    ref = oracle_run(P)
    S1, x1 = G.solve_problem(P, gradient="maintained")
    S2, x2 = G.solve_problem(P, gradient="direct")
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    e12, e1, e2 = rel(x1, x2), rel(x1, ref.x), rel(x2, ref.x)
    say(f"  maintained vs direct {e12:.2e}, vs oracle {e1:.2e} / {e2:.2e}")
    assert e12 <= 1e-9 and e1 <= 1e-8 and e2 <= 1e-8
    assert S1.status() == S2.status() == (0, P.k)
    check_state_consistency(S1, P)
    S1.close()
    S2.close()
