"""The SRTT embedding (eq:sketching_trig) on the GPU against the oracle's, through the
C ABI: the sketch itself, sGKS trajectories, the backward, and the independence of the
method from the embedding (Sec. 2.2): at equal s, SRTT and sparse-sign sketches give
reconstructions of the same quality."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_common import check_state_consistency, problem, rel, say  # noqa: E402
from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402


def _oracle(P, k=None, **kw):
    return O.sgks(P.A, P.L, P.b, P.mu, P.k if k is None else k, P.s, P.seed, zeta=P.zeta,
                  ell=P.ell, refine_steps=P.refine_steps, sketch="srtt", **kw)


@pytest.mark.parametrize("name", ["deblur1d", "deblur2d", "dynamic_ct"])
def test_srtt_sketch_of_b(name):
    P = problem(name, "small")
    say("case srtt S_A b", name, P.m, P.s)
    A, L, b = G.upload_problem(P)
    S = G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k, sketch="srtt")
    S_A, _ = O.make_sketches(P.m, P.p, P.s, P.seed, kind="srtt")
    ref = S_A @ P.b
    e = np.max(np.abs(S.state("c_b") - ref)) / np.max(np.abs(ref))
    say(f"  max rel diff {e:.2e}")
    assert e <= 1e-12
    S.close()


@pytest.mark.parametrize("name,tol", [("deblur1d", 1e-10), ("deblur2d", 1e-8), ("ct2d", 1e-8),
                                      ("dynamic_ct", 1e-8)])
def test_srtt_small_matches_oracle(name, tol):
    P = problem(name, "small")
    say("case srtt small", name, P.n, P.k, P.s)
    ref = _oracle(P)
    S, x = G.solve_problem(P, sketch="srtt")
    e = rel(x.cpu().numpy(), ref.x)
    say(f"  rel err {e:.3e}")
    assert e <= tol
    assert S.status() == (0, P.k)
    check_state_consistency(S, P, sketch="srtt")
    S.close()


def test_srtt_deblur2d_full_and_sketch_independence():
    """n = 65,536, k = 100, s = 400: the SRTT run against the oracle's SRTT run, and its
    reconstruction error against the sparse-sign run's at the same s (Sec. 2.2: the
    method does not depend on the embedding)."""
    P = problem("deblur2d", "full")
    say("case srtt deblur2d full")
    ref = _oracle(P)
    S, x = G.solve_problem(P, sketch="srtt")
    x = x.cpu().numpy()
    e = rel(x, ref.x)
    S2, x2 = G.solve_problem(P)
    x2 = x2.cpu().numpy()
    r1, r2 = rel(x, P.x_true), rel(x2, P.x_true)
    say(f"  rel err vs oracle {e:.3e}; RRE srtt {r1:.5f}, sparse sign {r2:.5f}")
    assert e <= 1e-5
    assert abs(r1 - r2) <= 0.05 * r2
    S.close()
    S2.close()


def test_srtt_dynamic_ct_full_size_factors():
    """The dynamic CT workload at full size with the SRTT (m = 327,600: 80 blocks of 4,096
    rows; p = 1,474,560: 360 blocks in 128 ranges of two or three): ten expansions against
    the oracle's SRTT run, and the GPU's factors against the oracle's SRTT applied to the
    GPU's own basis (Q_A R_A = S_A A W, Q_L R_L = S_L L W)."""
    P = dataclasses.replace(problem("dynamic_ct", "full"), k=10)
    say("case srtt dynamic_ct full, k = 10")
    ref = _oracle(P)
    S, x = G.solve_problem(P, sketch="srtt")
    e = rel(x.cpu().numpy(), ref.x)
    say(f"  rel err vs oracle {e:.3e}")
    assert e <= 1e-8
    assert S.status() == (0, P.k)
    check_state_consistency(S, P, sketch="srtt")
    S.close()


def test_srtt_backward():
    P = problem("dynamic_ct", "small")
    say("case srtt backward")
    S, x = G.solve_problem(P, sketch="srtt")
    xh = x.cpu().numpy()
    g_x = 2 * (xh - P.x_true)
    gb, gmu = S.backward(torch.as_tensor(g_x, device="cuda"))
    res = O.Result(xh, S.state("y"), S.state("W"), S.state("Q_A"), S.state("R_A"),
                   S.state("Q_L"), S.state("R_L"), S.state("d_A"), S.state("G"),
                   S.state("c_b"), P.k, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(res, P.mu, g_x, P.A, P.L, P.s, P.seed, P.zeta,
                                         sketch="srtt")
    e = rel(gb.cpu().numpy(), gb_ref)
    say(f"  grad_b rel err {e:.3e}")
    assert e <= 1e-8
    assert abs(gmu - gmu_ref) <= 1e-8 * abs(gmu_ref)
    S.close()


def test_srtt_validation():
    P = problem("deblur2d", "small")
    A, L, b = G.upload_problem(P)
    with pytest.raises(G.SgksError) as e:      # D keeps at most m rows
        G.SGKS(A, L, b, P.mu, P.m + 1, P.seed, max_iters=P.k, sketch="srtt")
    assert e.value.code == -4
