"""GKS (Alg. 1) on the GPU against the oracle's GKS, through the C ABI.

The GPU projects each new direction with the projector of eq:single_mgs (a
second time when the loss ratio of eq:loss_criterion reaches 1e-10); the oracle
sweeps modified Gram-Schmidt.  The two agree in exact arithmetic; the basis is
orthonormal, so the projected problem stays well conditioned and the iterates
agree to rounding."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_common import problem, rel, say  # noqa: E402
from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402


def gks_gpu(P, k, **kw):
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, 1, 0, ell=P.ell, max_iters=max(k, 1), method="gks", **kw)
    return S


def check_gks_state(S, P, tol=1e-9):
    """V orthonormal, Q_A R_A = A V, Q_L R_L = L V, Q orthonormal, d_A = Q_A^T b, y solves
    the projected problem eq:projected_withQR built from the GPU factors."""
    V = S.state("W")
    d = V.shape[1]
    QA, RA, QL, RL = S.state("Q_A"), S.state("R_A"), S.state("Q_L"), S.state("R_L")
    dA, y = S.state("d_A"), S.state("y")
    assert np.linalg.norm(V.T @ V - np.eye(d)) <= 1e-10
    AV, LV = P.A @ V, P.L @ V
    assert np.linalg.norm(QA @ RA - AV) <= tol * np.linalg.norm(AV)
    assert np.linalg.norm(QL @ RL - LV) <= tol * np.linalg.norm(LV)
    assert np.linalg.norm(QA.T @ QA - np.eye(d)) <= 1e-10
    assert np.linalg.norm(QL.T @ QL - np.eye(d)) <= 1e-10
    assert rel(dA, QA.T @ P.b) <= 1e-10
    y_ref, _ = O.projected_solve(RA, RL, dA, P.mu)
    assert rel(y, y_ref) <= 1e-10


@pytest.mark.parametrize("name", ["deblur1d", "deblur2d", "ct2d", "dynamic_ct"])
def test_gks_small_matches_oracle(name):
    P = problem(name, "small")
    say("case gks small", name, P.n, P.k)
    ref = O.gks(P.A, P.L, P.b, P.mu, P.k, ell=P.ell, keep_history=True)
    S = gks_gpu(P, P.k)
    done = 0
    for k in sorted(set(range(0, P.k + 1, 5)) | {P.k}):
        S.iterate(k - done)
        done = k
        e = rel(S.solution().cpu().numpy(), ref.x_hist[k])
        say(f"  k={k} rel err {e:.3e}")
        assert e <= 1e-10
    assert S.status() == (0, P.k)
    check_gks_state(S, P)
    S.close()


def test_gks_deblur1d_full_fp64():
    """1D deblurring, FP64, k = 30: x_k within 1e-10 of the oracle's GKS."""
    P = problem("deblur1d", "full")
    say("case gks deblur1d full")
    ref = O.gks(P.A, P.L, P.b, P.mu, P.k, ell=P.ell, keep_history=True)
    S = gks_gpu(P, P.k)
    S.iterate(P.k)
    e = rel(S.solution().cpu().numpy(), ref.x)
    say(f"  rel err {e:.3e}")
    assert e <= 1e-10
    check_gks_state(S, P)
    S.close()


def test_gks_deblur2d_full():
    """2D deblurring n = 65,536, k = 100 (FP32 operators, FP64 vectors)."""
    P = problem("deblur2d", "full")
    say("case gks deblur2d full")
    ref = O.gks(P.A, P.L, P.b, P.mu, P.k, ell=P.ell, keep_history=True)
    S = gks_gpu(P, P.k)
    done = 0
    for k in (10, 50, 100):
        S.iterate(k - done)
        done = k
        e = rel(S.solution().cpu().numpy(), ref.x_hist[k])
        say(f"  k={k} rel err {e:.3e}")
        assert e <= 1e-8
    check_gks_state(S, P)
    S.close()


@pytest.mark.parametrize("gradient,passes", [("direct", 2), ("maintained", 1)])
def test_gks_options(gradient, passes):
    """The direct gradient form and a single projection in the QR appends (the oracle's
    qr_passes = 1)."""
    P = problem("deblur2d", "small")
    say("case gks options", gradient, passes)
    ref = O.gks(P.A, P.L, P.b, P.mu, P.k, ell=P.ell, qr_passes=passes)
    S = gks_gpu(P, P.k, gradient=gradient, qr_passes=passes)
    S.iterate(P.k)
    e = rel(S.solution().cpu().numpy(), ref.x)
    say(f"  rel err {e:.3e}")
    assert e <= 1e-9
    S.close()


def test_gks_breakdown_and_refusals():
    import scipy.sparse as sp
    n = 64
    I = sp.identity(n, format="csr")
    I.indices = I.indices.astype(np.int32)
    I.indptr = I.indptr.astype(np.int32)
    Id = G.DeviceCsr.from_scipy(I)
    bh = np.linspace(1.0, 2.0, n)
    b = torch.as_tensor(bh, device="cuda")
    say("case gks breakdown / refusals")
    # K_1(A^T A, A^T b) = span{b} holds the solution: the projected gradient vanishes
    S = G.SGKS(Id, Id, b, 0.5, 1, 0, ell=1, max_iters=4, method="gks")
    S.iterate(4)
    rc, it = S.status()
    ref = O.gks(I, I, bh, 0.5, 4, ell=1)
    assert ref.status == O.STATUS_BREAKDOWN and ref.iters == 0
    assert rc == G.BREAKDOWN and it == 0
    assert rel(S.solution().cpu().numpy(), ref.x) <= 1e-12
    with pytest.raises(G.SgksError) as e:
        S.backward(torch.zeros(n, dtype=torch.float64, device="cuda"))
    assert e.value.code == -1
    S.close()
    with pytest.raises(G.SgksError) as e:
        G.SGKS(Id, Id, b, 0.5, 1, 0, ell=1, max_iters=4, method="gks", refine_steps=1)
    assert e.value.code == -1
    with pytest.raises(G.SgksError) as e:
        G.SGKSBatch([(Id, Id, b, 0.5, 8, 0)], ell=1, max_iters=4, method="gks")
    assert e.value.code == -1


def test_gks_profile_and_residual():
    """Launch counts per phase; the residual norm of the projected problem equals the
    true Tikhonov residual (no sketch: d_A = Q_A^T b)."""
    P = problem("deblur2d", "small")
    S = gks_gpu(P, 10)
    S.profile(True).iterate(10)
    ms, cnt = S.profile_read()
    n = {name: cnt[i] for i, name in enumerate(G.PHASE_NAMES)}
    say("  launches", n)
    assert n["spmv_new_column"] == 10 and n["adjoint"] == 10 and n["sketch_scatter"] == 0
    tn, sn = S.residual_norm()
    x = S.solution().cpu().numpy()
    ref = O.tikhonov_residual(P.A, P.L, P.b, P.mu, x)
    assert abs(tn - ref) <= 1e-10 * ref
    assert abs(sn - ref) <= 1e-8 * ref
    S.close()
