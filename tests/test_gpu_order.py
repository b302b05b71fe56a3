"""An internal order of the unknowns (a permutation the context works in, here the Morton
curve of each image frame): the same method, only the rounding order of the sparse
products changes, so the iterates agree with the caller-order run and the oracle to
rounding; outputs and the backward's input stay in the caller's order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from gpu_common import check_state_consistency, oracle_run, problem, rel, say  # noqa: E402
from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402
from workloads.generators import image_order  # noqa: E402


def _order(P):
    return torch.as_tensor(image_order(P), dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("name", ["deblur2d", "ct2d", "dynamic_ct"])
def test_order_keeps_the_iterates(name):
    P = problem(name, "small")
    say("case order", name, P.n)
    ref = oracle_run(P)
    S1, x1 = G.solve_problem(P, order=_order(P))
    S2, x2 = G.solve_problem(P)
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    e12, e1 = rel(x1, x2), rel(x1, ref.x)
    say(f"  ordered vs caller order {e12:.2e}, vs oracle {e1:.2e}")
    assert e12 <= 1e-10 and e1 <= 1e-8
    assert S1.status() == S2.status() == (0, P.k)
    check_state_consistency(S1, P)      # W copied back in the caller's order
    S1.close()
    S2.close()


def test_order_backward_and_gks():
    P = problem("dynamic_ct", "small")
    say("case order backward / gks")
    S, x = G.solve_problem(P, order=_order(P))
    xh = x.cpu().numpy()
    g_x = 2 * (xh - P.x_true)
    gb, gmu = S.backward(torch.as_tensor(g_x, device="cuda"))
    res = O.Result(xh, S.state("y"), S.state("W"), S.state("Q_A"), S.state("R_A"),
                   S.state("Q_L"), S.state("R_L"), S.state("d_A"), S.state("G"), S.state("c_b"),
                   P.k, 0, [], [])
    gb_ref, gmu_ref = O.frozen_adjoint_b(res, P.mu, g_x, P.A, P.L, P.s, P.seed, P.zeta)
    assert rel(gb.cpu().numpy(), gb_ref) <= 1e-8
    assert abs(gmu - gmu_ref) <= 1e-8 * abs(gmu_ref)
    S.close()
    g = O.gks(P.A, P.L, P.b, P.mu, P.k, ell=P.ell)
    A, L, b = G.upload_problem(P)
    Sg = G.SGKS(A, L, b, P.mu, 1, 0, ell=P.ell, max_iters=P.k, method="gks", order=_order(P))
    Sg.iterate(P.k)
    assert rel(Sg.solution().cpu().numpy(), g.x) <= 1e-10
    Sg.close()


def test_order_in_a_batch():
    Ps = problem("batch", "small")
    say("case order batch")
    orders = [image_order(P) for P in Ps]
    data = G.upload_batch(Ps, orders=orders)
    B = G.SGKSBatch(data, ell=Ps[0].ell, max_iters=Ps[0].k, zeta=Ps[0].zeta)
    B.iterate(Ps[0].k)
    for i, P in enumerate(Ps):
        S, x = G.solve_problem(P, order=torch.as_tensor(orders[i], device="cuda"))
        assert np.array_equal(B.problem(i).solution().cpu().numpy(), x.cpu().numpy()), i
        assert rel(x.cpu().numpy(), oracle_run(P).x) <= 1e-8
        S.close()
    B.close()


def test_order_must_be_a_permutation():
    P = problem("deblur2d", "small")
    A, L, b = G.upload_problem(P)
    o = _order(P)
    o[5] = o[6]
    with pytest.raises(G.SgksError) as e:
        G.SGKS(A, L, b, P.mu, P.s, P.seed, max_iters=P.k, order=o)
    assert e.value.code == -1
