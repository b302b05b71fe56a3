"""The paper's experiment shapes (Exp. 2 CT 500^2, Exp. 3 travel time with m = 6n and
sketches up to s = 10,000, Exp. 4 dynamic CT 256^2 x 10 in 18-degree sectors) at
reduced sizes against the oracle, and sketch sizes beyond 1,024 (the multi-workgroup
append with up to 256 workgroups, fewer LDS copies of the bins in the scatter)."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_common import check_state_consistency, oracle_run, problem, rel, say  # noqa: E402
from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402


@pytest.mark.parametrize("name", ["ct_exp2", "traveltime_exp3", "dynamic_ct_exp4"])
def test_paper_shapes_small_match_oracle(name):
    P = problem(name, "small")
    say("case paper shape small", name, P.m, P.n, P.p, P.s, P.k)
    ref = oracle_run(P)
    S, x = G.solve_problem(P)
    e = rel(x.cpu().numpy(), ref.x)
    say(f"  rel err {e:.3e}, append groups {S.tuning()['append_groups']}")
    assert e <= 1e-8
    assert S.status() == (0, P.k)
    check_state_consistency(S, P)
    S.close()


@pytest.mark.parametrize("s", [1025, 2048, 4000, 10000, 16384])
def test_large_sketch_sizes(s):
    """s above the one-workgroup append's 1,024 (multi-workgroup append, up to 256
    workgroups of at most 64 sketch rows) and above 8,192 (one LDS copy of the bins of
    more than 64 KiB in the scatter)."""
    P = dataclasses.replace(problem("deblur2d", "small"), s=s)
    k = 12
    say("case large sketch", s)
    ref = O.sgks(P.A, P.L, P.b, P.mu, k, s, P.seed, zeta=P.zeta, ell=P.ell)
    S, x = G.solve_problem(P, k=k)
    g = S.tuning()["append_groups"]
    e = rel(x.cpu().numpy(), ref.x)
    say(f"  append groups {g}, rel err {e:.3e}")
    assert g > 1
    assert e <= 1e-9
    cb = S.state("c_b")
    S_A, _ = O.make_sketches(P.m, P.p, s, P.seed, P.zeta)
    assert np.max(np.abs(cb - S_A @ P.b)) <= 1e-13 * np.max(np.abs(S_A @ P.b))
    S.close()


def test_large_sketch_backward():
    """The frozen-basis backward with s = 10,000 (the sketch transpose reads v through the
    caches instead of LDS)."""
    P = dataclasses.replace(problem("dynamic_ct", "small"), s=10000)
    say("case large sketch backward")
    S, x = G.solve_problem(P, k=8)
    xh = x.cpu().numpy()
    g_x = 2 * (xh - P.x_true)
    gb, gmu = S.backward(torch.as_tensor(g_x, device="cuda"))
    res = O.Result(xh, S.state("y"), S.state("W"), S.state("Q_A"), S.state("R_A"),
                   S.state("Q_L"), S.state("R_L"), S.state("d_A"), S.state("G"), S.state("c_b"),
                   8, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(res, P.mu, g_x, P.A, P.L, P.s, P.seed, P.zeta)
    assert rel(gb.cpu().numpy(), gb_ref) <= 1e-8
    assert abs(gmu - gmu_ref) <= 1e-8 * abs(gmu_ref)
    S.close()
