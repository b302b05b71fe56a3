"""Total-derivative adjoint on the GPU (sgks_backward_total) against the oracle's
reverse sweep, and against central differences of the GPU pipeline itself.

The adjoint is not in the paper; the oracle's version is pinned by central
differences of its own forward map and by the closed form at d = n.  The
gradient seed g_x is a seeded random vector (no input comes from the HIP path).

Tolerances.  The two reverse sweeps are the same function evaluated in another
association: the oracle keeps an explicit n x d adjoint of W and factors every
projected problem afresh; the GPU forms each column's adjoint lazily from the
solves' histories and reuses the leading blocks of the final stacked factor.
The bound is stated relative to the spread between two FP64 evaluations of the
oracle's sweep (the problem with its unknowns permuted: the same map, another
rounding order), with a floor of 1e-9: rel err <= max(1e-9, 100 spread).
"""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import sgks_oracle as O  # noqa: E402
from paper_2606_18073_amd import sgks as G  # noqa: E402
from workloads import generators as gen  # noqa: E402

from gpu_common import problem, rel, say  # noqa: E402


def seed_grad(n, seed=11):
    return np.random.default_rng(seed).standard_normal(n)


def oracle_total(P, k, g_x, sketch="sparse_sign", permute=None, ell=None):
    """The oracle's total adjoint; with permute (a seed) on the problem with its unknowns
    permuted, mapped back."""
    ell = P.ell if ell is None else ell
    A, L, gx, Pm = P.A, P.L, g_x, None
    if permute is not None:
        perm = np.random.default_rng(permute).permutation(P.n)
        Pm = sp.identity(P.n, format="csr")[:, perm]
        A = (P.A @ Pm).tocsr()
        L = (P.L @ Pm).tocsr()
        A.sort_indices()
        L.sort_indices()
        gx = Pm.T @ g_x
    return O.total_adjoint(A, L, P.b, P.mu, k, P.s, P.seed, gx, zeta=P.zeta, ell=ell,
                           sketch=sketch)


def gpu_total(P, k, g_x, **kw):
    import warnings
    kw.setdefault("refine_steps", 0)
    S, x = G.solve_problem(P, k=k, keep_history=True, **kw)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)   # the estimate is logged instead
        gb, gmu, est = S.backward_total(torch.as_tensor(g_x, device="cuda"), with_error=True)
    say(f"  error estimate d eps kappa(G)^2 = {est:.2e}")
    rc, it = S.status()
    return S, gb.cpu().numpy(), gmu, rc, it


def check_against_oracle(P, k, sketch="sparse_sign", ell=None, **kw):
    g_x = seed_grad(P.n)
    S, gb, gmu, rc, it = gpu_total(P, k, g_x, sketch=sketch, **({"ell": ell} if ell else {}), **kw)
    assert rc == 0 and it == k
    gb_o, gmu_o = oracle_total(P, k, g_x, sketch=sketch, ell=ell)
    gb_p, gmu_p = oracle_total(P, k, g_x, sketch=sketch, ell=ell, permute=1)
    spread_b, spread_m = rel(gb_p, gb_o), abs(gmu_p - gmu_o) / abs(gmu_o)
    eb, em = rel(gb, gb_o), abs(gmu - gmu_o) / abs(gmu_o)
    say(f"  grad_b rel err {eb:.2e} (spread {spread_b:.2e}), grad_mu {em:.2e} "
        f"(spread {spread_m:.2e})")
    assert eb <= max(1e-9, 100 * spread_b)
    assert em <= max(1e-9, 100 * spread_m)
    return S


@pytest.mark.parametrize("name", ["deblur1d", "deblur2d", "ct2d", "dynamic_ct"])
def test_total_adjoint_small_matches_oracle(name):
    P = problem(name, "small")
    say("case total adjoint", name, P.n, P.k)
    S = check_against_oracle(P, P.k)
    S.close()


@pytest.mark.parametrize("k,ell", [(0, 3), (1, 3), (4, 1), (4, 2), (6, 5)])
def test_total_adjoint_few_expansions_and_initial_dims(k, ell):
    """k = 0 leaves only the initial Krylov basis; ell from 1 (no Gram-Schmidt reverse)
    to 5."""
    P = problem("deblur2d", "small")
    say("case total adjoint k/ell", k, ell)
    S = check_against_oracle(P, k, ell=ell)
    S.close()


@pytest.mark.parametrize("sketch,name", [("srtt", "deblur1d"), ("srtt", "dynamic_ct"),
                                         ("identity", "deblur1d")])
def test_total_adjoint_other_sketches(sketch, name):
    P = problem(name, "small")
    if sketch == "identity":
        P = _with_s(P, max(P.m, P.p))
    say("case total adjoint sketch", sketch)
    S = check_against_oracle(P, 10, sketch=sketch)
    S.close()


def _with_s(P, s):
    import copy
    Q = copy.copy(P)
    Q.s = s
    return Q


def test_total_adjoint_is_the_derivative_of_the_gpu_pipeline():
    """Central differences of g_x . x_k of the GPU solve itself (n = 64, k = 6, well
    below the full space): directional derivatives in b and the derivative in mu."""
    A_ = gen.psf_blur2d(8, sigma=1.0, half=1)
    L_ = gen.grad2d(8)
    rng = np.random.default_rng(2)
    xt_ = gen.random_ellipses(8, rng, count=3)
    b_ = gen.add_noise(A_ @ xt_, 0.01, rng)
    mu_, s_, seed_, k = 5e-3, 60, 3, 6
    A, L = G.DeviceCsr.from_scipy(A_), G.DeviceCsr.from_scipy(L_)
    g = torch.as_tensor(seed_grad(A_.shape[1], 5), device="cuda")
    say("case total adjoint central differences")

    def f(bv, mv):
        S = G.SGKS(A, L, bv, mv, s_, seed_, max_iters=k)
        S.iterate(k)
        v = float(g @ S.solution())
        S.close()
        return v

    b = torch.as_tensor(b_, device="cuda")
    S = G.SGKS(A, L, b, mu_, s_, seed_, max_iters=k, keep_history=True)
    S.iterate(k)
    gb, gmu = S.backward_total(g)
    S.close()
    for t in range(3):
        db = torch.as_tensor(np.random.default_rng(20 + t).standard_normal(b_.size), device="cuda")
        h = 1e-5 * float(b.norm()) / float(db.norm())
        fd = (f(b + h * db, mu_) - f(b - h * db, mu_)) / (2 * h)
        an = float(gb @ db)
        say(f"  direction {t}: fd {fd:.10e} adjoint {an:.10e}")
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3)
    hm = 1e-5 * mu_
    fdm = (f(b, mu_ + hm) - f(b, mu_ - hm)) / (2 * hm)
    say(f"  mu: fd {fdm:.10e} adjoint {gmu:.10e}")
    assert abs(fdm - gmu) <= 1e-6 * max(abs(fdm), 1e-3)


def test_total_adjoint_autograd_order_and_resume():
    """The autograd function with adjoint="total" returns sgks_backward_total's values;
    an internal order of the unknowns gives the same gradient to rounding; iterate(3)
    then iterate(4) gives the gradient of iterate(7)."""
    P = problem("dynamic_ct", "small")
    k = 7
    say("case total adjoint autograd/order/resume")
    g_x = seed_grad(P.n)
    gt = torch.as_tensor(g_x, device="cuda")
    A, L, b = G.upload_problem(P)
    bg = b.clone().requires_grad_(True)
    mu = torch.tensor(P.mu, dtype=torch.float64, device="cuda", requires_grad=True)
    x = G.sgks_solve(A, L, bg, mu, P.s, k, P.seed, adjoint="total")
    (x * gt).sum().backward()
    S, gb, gmu, rc, it = gpu_total(P, k, g_x)
    assert torch.equal(bg.grad.cpu(), torch.as_tensor(gb).to(bg.dtype))   # b's storage dtype
    assert mu.grad.item() == gmu
    S.close()
    # resumed iteration
    S2, _ = G.solve_problem(P, k=3, keep_history=True, refine_steps=0, max_iters=k)
    S2.iterate(4)
    gb2, gmu2 = S2.backward_total(gt)
    assert np.array_equal(gb2.cpu().numpy(), gb) and gmu2 == gmu
    S2.close()
    # a random internal order of the unknowns
    order = torch.as_tensor(np.random.default_rng(4).permutation(P.n), dtype=torch.int32,
                            device="cuda")
    S3 = G.SGKS(A, L, b, P.mu, P.s, P.seed, ell=P.ell, zeta=P.zeta, max_iters=k,
                keep_history=True, order=order)
    S3.iterate(k)
    gb3, gmu3 = S3.backward_total(gt)
    e = rel(gb3.cpu().numpy(), gb)
    say(f"  permuted order: grad_b rel diff {e:.2e}")
    assert e <= 1e-9 and abs(gmu3 - gmu) <= 1e-9 * abs(gmu)
    S3.close()


def test_total_adjoint_refusals():
    """Without keep_history the entry point refuses (no device work); keep_history is
    refused with refinement, the direct gradient form and GKS."""
    P = problem("deblur1d", "small")
    say("case total adjoint refusals")
    S, x = G.solve_problem(P, k=2)
    with pytest.raises(G.SgksError) as e:
        S.backward_total(torch.zeros_like(x))
    assert e.value.code == -1
    S.close()
    for kw in ({"refine_steps": 1}, {"gradient": "direct"}, {"method": "gks"}):
        with pytest.raises(G.SgksError) as e:
            G.solve_problem(P, k=1, keep_history=True, **kw)
        assert e.value.code == -1


def test_total_adjoint_dynamic_ct_full_size():
    """Dynamic CT at full size, k = 10, in the launch configuration of the benchmark's
    solve (a sparse-sign sketch, chain append, the H W adjoint beside it)."""
    P = problem("dynamic_ct", "full")
    k = 10
    say("case total adjoint full", P.n, P.m, k)
    g_x = seed_grad(P.n)
    S, gb, gmu, rc, it = gpu_total(P, k, g_x)
    assert rc == 0 and it == k
    gb_o, gmu_o = oracle_total(P, k, g_x)
    eb, em = rel(gb, gb_o), abs(gmu - gmu_o) / abs(gmu_o)
    say(f"  grad_b rel err {eb:.2e}, grad_mu {em:.2e}")
    assert eb <= 1e-8 and em <= 1e-8
    S.close()


def test_total_adjoint_error_estimate_bounds_the_rounding_spread():
    """Dynamic CT at full size: two rounding orders of the same solve (the unknowns in
    another internal order) give gradients whose spread stays below the returned
    estimate d eps kappa(G)^2 -- small at k = 30 (kappa ~ 2e3), large at k = 100
    (kappa ~ 3e6), where the binding warns."""
    P = problem("dynamic_ct", "full")
    A, L, b = G.upload_problem(P)
    gt = torch.as_tensor(seed_grad(P.n), device="cuda")
    order = torch.as_tensor(np.random.default_rng(4).permutation(P.n), dtype=torch.int32,
                            device="cuda")
    for k in (30, 100):
        say("case total adjoint error estimate", k)
        out = []
        for od in (None, order):
            S = G.SGKS(A, L, b, P.mu, P.s, P.seed, ell=P.ell, zeta=P.zeta, max_iters=k,
                       keep_history=True, order=od)
            S.iterate(k)
            if k == 30:
                out.append(S.backward_total(gt, with_error=True))
            else:
                with pytest.warns(RuntimeWarning):
                    out.append(S.backward_total(gt, with_error=True))
            S.close()
        (gb1, gm1, est), (gb2, gm2, _) = out
        spread = float((gb1 - gb2).norm() / gb1.norm())
        say(f"  spread {spread:.2e}, estimate {est:.2e}")
        assert spread <= est
        assert abs(gm1 - gm2) <= est * abs(gm1)
        if k == 30:
            assert est <= 1e-6


def test_total_adjoint_graph_replay_workspace_and_profiling():
    """The y history is recorded inside captured graphs of 1 and 8 expansions and in a
    caller's workspace (no device allocation), and profiling does not change it: every
    variant gives the kernel-by-kernel gradient bit for bit."""
    P = problem("dynamic_ct", "small")
    k = 12
    say("case total adjoint graph/workspace/profiling")
    g_x = seed_grad(P.n)
    gt = torch.as_tensor(g_x, device="cuda")
    S0, gb0, gm0, rc, it = gpu_total(P, k, g_x)
    S0.close()
    A, L, b = G.upload_problem(P)
    opts = dict(ell=P.ell, zeta=P.zeta, max_iters=k, refine_steps=0, keep_history=True)
    nb = G.workspace_bytes(A, L, P.s, value_dtype=P.dtype, **opts)
    nb0 = G.workspace_bytes(A, L, P.s, value_dtype=P.dtype,
                            **{**opts, "keep_history": False})
    assert nb > nb0 + 8 * P.n * k    # E alone is n max_iters doubles
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for kw in ({"graph": True}, {"workspace": ws}, {"profile": True}):
        prof = kw.pop("profile", False)
        S = G.SGKS(A, L, b, P.mu, P.s, P.seed, **opts, **kw)
        if prof:
            S.profile(True)
        S.iterate(k)
        gb, gm = S.backward_total(gt)
        assert np.array_equal(gb.cpu().numpy(), gb0) and gm == gm0, kw
        S.close()


def test_total_adjoint_after_breakdown_is_the_closed_form():
    """A = L = I with identity sketches: span{b} holds the solution, the first expansion
    breaks down, and x = b / (1 + mu) for every b.  The reverse sweep over the expansions
    done (none) gives d(g.x)/db = g / (1 + mu) and d(g.x)/dmu = -(g.b) / (1 + mu)^2."""
    I = sp.identity(64, format="csr")
    I.indices = I.indices.astype(np.int32)
    I.indptr = I.indptr.astype(np.int32)
    bh = np.linspace(1.0, 2.0, 64)
    A = G.DeviceCsr.from_scipy(I)
    b = torch.as_tensor(bh, device="cuda")
    mu = 0.5
    g = seed_grad(64, 3)
    say("case total adjoint after breakdown")
    S = G.SGKS(A, A, b, mu, 64, 0, ell=1, max_iters=4, sketch="identity", keep_history=True)
    S.iterate(4)
    rc, it = S.status()
    assert rc == G.BREAKDOWN and it == 0
    gb, gm = S.backward_total(torch.as_tensor(g, device="cuda"))
    S.close()
    assert rel(gb.cpu().numpy(), g / (1 + mu)) <= 1e-13
    assert abs(gm + (g @ bh) / (1 + mu) ** 2) <= 1e-13 * abs(g @ bh)


def test_total_adjoint_in_a_batch():
    """Every problem of a batch (uneven sizes, one launch per step for all) keeps its y
    history; each problem's total adjoint equals that of its plain solve bit for bit.
    Also a batch of one problem."""
    Ps = problem("batch", "small")
    k = 8
    say("case total adjoint batch", [(P.name, P.n) for P in Ps])
    for sel in (Ps, Ps[:1]):
        B, _ = G.solve_batch(sel, k=k, keep_history=True, refine_steps=0)
        for i, P in enumerate(sel):
            g = seed_grad(P.n, 30 + i)
            gbB, gmB = B.problem(i).backward_total(torch.as_tensor(g, device="cuda"))
            S, gbP, gmP, rc, it = gpu_total(P, k, g, ell=sel[0].ell, zeta=sel[0].zeta)
            S.close()
            assert np.array_equal(gbB.cpu().numpy(), gbP) and gmB == gmP, i
        B.close()


def test_total_adjoint_then_iterate_further():
    """The reverse sweep leaves the forward state intact: backward after 5 expansions,
    5 more expansions, backward again -- equal, bit for bit, to 10 expansions then one
    backward (and x_10 equal too)."""
    P = problem("deblur2d", "small")
    say("case total adjoint then iterate")
    g_x = seed_grad(P.n)
    gt = torch.as_tensor(g_x, device="cuda")
    S1, _ = G.solve_problem(P, k=5, keep_history=True, refine_steps=0, max_iters=10)
    S1.backward_total(gt)
    S1.iterate(5)
    gb1, gm1 = S1.backward_total(gt)
    x1 = S1.solution().cpu().numpy()
    S1.close()
    S2, gb2, gm2, rc, it = gpu_total(P, 10, g_x)
    x2 = S2.solution().cpu().numpy()
    S2.close()
    assert np.array_equal(x1, x2)
    assert np.array_equal(gb1.cpu().numpy(), gb2) and gm1 == gm2


@pytest.mark.parametrize("name", ["ct_exp2", "traveltime_exp3", "dynamic_ct_exp4"])
def test_total_adjoint_paper_shapes_small(name):
    """The paper's Exp. 2-4 shapes at small size; travel time has s = 1,500, beyond the
    one-workgroup append (the multi-workgroup append chain)."""
    P = problem(name, "small")
    say("case total adjoint paper shape", name, P.n, P.m, P.s, P.k)
    S = check_against_oracle(P, P.k)
    S.close()


def test_srtt_transposes_full_size():
    """The SRTT transposes on the matrix cores at full size (S_A^T: m = 327,600, 1,280
    blocks of 256 rows, the last one partial; S_L^T: p = 1,474,560): the frozen adjoint
    (S_A^T alone) and the total adjoint (both sides at every column) against the oracle's
    fast-DCT transposes, dynamic CT, k = 5."""
    P = problem("dynamic_ct", "full")
    k = 5
    say("case srtt transposes full size", P.m, P.p, P.s)
    g_x = seed_grad(P.n)
    S, gb, gmu, rc, it = gpu_total(P, k, g_x, sketch="srtt")
    assert rc == 0 and it == k
    fb, fmu = S.backward(torch.as_tensor(g_x, device="cuda"))
    res = O.Result(S.solution().cpu().numpy(), S.state("y"), S.state("W"), S.state("Q_A"),
                   S.state("R_A"), S.state("Q_L"), S.state("R_L"), S.state("d_A"),
                   S.state("G"), S.state("c_b"), k, 0, [], [])
    S.close()
    fb_o, fmu_o = O.frozen_adjoint_b(res, P.mu, g_x, P.A, P.L, P.s, P.seed, P.zeta,
                                     sketch="srtt")
    ef = rel(fb.cpu().numpy(), fb_o)
    gb_o, gmu_o = oracle_total(P, k, g_x, sketch="srtt")
    eb, em = rel(gb, gb_o), abs(gmu - gmu_o) / abs(gmu_o)
    say(f"  frozen grad_b rel err {ef:.2e}; total grad_b {eb:.2e}, grad_mu {em:.2e}")
    assert ef <= 1e-10
    assert eb <= 1e-9 and em <= 1e-9


@pytest.mark.parametrize("zeta,passes", [(2, 2), (4, 2), (16, 2), (8, 1)])
def test_total_adjoint_zeta_and_single_projection(zeta, passes):
    """Every instantiation of the reverse forward product's sparse-sign transposes (zeta
    entries per column gathered from the cached pattern) and the single-projection QR
    append (eq:updqr as written), against the oracle."""
    import copy
    P = copy.copy(problem("dynamic_ct", "small"))
    P.zeta = zeta
    k = 10
    say("case total adjoint zeta/passes", zeta, passes)
    g_x = seed_grad(P.n)
    S, gb, gmu, rc, it = gpu_total(P, k, g_x, qr_passes=passes)
    assert rc == 0 and it == k
    S.close()
    gb_o, gmu_o = O.total_adjoint(P.A, P.L, P.b, P.mu, k, P.s, P.seed, g_x, zeta=zeta, ell=P.ell)
    eb, em = rel(gb, gb_o), abs(gmu - gmu_o) / abs(gmu_o)
    say(f"  grad_b rel err {eb:.2e}, grad_mu {em:.2e}")
    assert eb <= 1e-9 and em <= 1e-9
