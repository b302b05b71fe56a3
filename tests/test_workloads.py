"""Closed-form checks of the seeded input generators (shared by the oracle and the HIP path)."""
import math

import numpy as np
import pytest

from workloads import generators as gen


def test_blur1d_rows_sum_to_one_and_dense():
    A = gen.blur1d_dense(256, 3.0)
    assert A.nnz == 256 * 256
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), 1.0, atol=1e-14)


def test_psf_blur_interior_rows_sum_to_one_and_exact_nnz():
    N = 256
    A = gen.psf_blur2d(N)
    # (sum over axis positions of window counts)^2, window 9 truncated at the border
    cnt = sum(min(i + 4, N - 1) - max(i - 4, 0) + 1 for i in range(N))
    assert A.nnz == cnt * cnt == 5216656
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(N, N)
    assert np.allclose(rs[4:-4, 4:-4], 1.0, atol=1e-13)   # PSF normalised before truncation
    assert np.all(rs[0, 0] < 1.0)
    assert np.abs(A - A.T).max() < 1e-15                   # symmetric PSF


def test_difference_operators():
    N = 256
    L = gen.grad2d(N)
    assert L.shape == (2 * N * N, N * N)
    assert L.nnz == 261120
    assert np.allclose(L @ np.ones(N * N), 0.0)
    # L^T L equals the paper's (N-1) x N difference blocks in Kronecker form
    n = 9
    D = gen.diff1d(n).toarray()
    I = np.eye(n)
    Lp = np.vstack([np.kron(I, D), np.kron(D, I)])
    Lg = gen.grad2d(n).toarray()
    assert np.allclose(Lg.T @ Lg, Lp.T @ Lp)
    st = gen.grad_spacetime(30, 128)
    assert st.shape == (3 * 30 * 128 * 128, 30 * 128 * 128) and st.nnz == 2900992
    assert np.allclose(st @ np.ones(st.shape[1]), 0.0)


def _chord_45(t, h):
    return max(0.0, 2 * math.sqrt(2) * h - 2 * abs(t))


def test_siddon_rows_are_chord_lengths():
    N, ndet = 32, 47
    angles = np.array([0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4])
    A = gen.parallel_beam_ct(N, angles, ndet)
    t = np.arange(ndet) - (ndet - 1) / 2.0
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(4, ndet)
    h = N / 2
    axis = np.where(np.abs(t) < h, float(N), 0.0)
    assert np.allclose(rs[0], axis, atol=1e-12)
    assert np.allclose(rs[2], axis, atol=1e-12)
    diag = np.array([_chord_45(tt, h) for tt in t])
    assert np.allclose(rs[1], diag, atol=1e-10)
    assert np.allclose(rs[3], diag, atol=1e-10)
    # axis-aligned rays through pixel centres have unit intersections
    row0 = A[:ndet].tocsr()
    assert np.allclose(row0.data, 1.0)


def test_siddon_random_angle_sum_matches_slab_formula():
    N, ndet = 20, 29
    ang = np.array([0.37, 1.1, 2.5])
    A = gen.parallel_beam_ct(N, ang, ndet)
    t = np.arange(ndet) - (ndet - 1) / 2.0
    h = N / 2
    rs = np.asarray(A.sum(axis=1)).ravel()
    k = 0
    for th in ang:
        c, s = math.cos(th), math.sin(th)
        for tt in t:
            # brute force: integrate the indicator of the square along the ray
            taus = np.linspace(-2 * N, 2 * N, 400001)
            x = tt * c - taus * s
            y = tt * s + taus * c
            inside = (np.abs(x) <= h) & (np.abs(y) <= h)
            length = inside.sum() * (taus[1] - taus[0])
            assert abs(rs[k] - length) < 2e-3
            k += 1


def test_travel_time_rows_are_segment_lengths():
    rng = np.random.default_rng(0)
    A = gen.travel_time(16, 200, rng)
    rng = np.random.default_rng(0)
    s1 = rng.integers(0, 4, size=200)
    s2 = (s1 + rng.integers(1, 4, size=200)) % 4
    P = gen.boundary_points(16, s1, rng.random(200))
    Q = gen.boundary_points(16, s2, rng.random(200))
    assert np.all(s1 != s2)
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), np.linalg.norm(Q - P, axis=1), atol=1e-9)


def test_noise_level_is_exact():
    rng = np.random.default_rng(3)
    bt = rng.standard_normal(1000)
    b = gen.add_noise(bt, 0.01, np.random.default_rng(4))
    assert abs(np.linalg.norm(b - bt) / np.linalg.norm(bt) - 0.01) < 1e-14


def test_dynamic_ct_is_block_diagonal():
    P = gen.dynamic_ct(0, nt=3, N=12, n_angles=6, n_det=17, k=5, s=40)
    ns = 144
    A = P.A.tocoo()
    assert np.all(A.row // (6 * 17) == A.col // ns)
    assert P.L.shape == (3 * P.n, P.n)


@pytest.mark.parametrize("name", ["deblur1d", "deblur2d", "ct2d", "dynamic_ct"])
def test_small_configs_are_seeded(name):
    P1 = gen.make(name, 3, "small")
    P2 = gen.make(name, 3, "small")
    assert np.array_equal(P1.b, P2.b) and (P1.A != P2.A).nnz == 0
    assert P1.A.indices.dtype == np.int32 and P1.A.has_sorted_indices
    if P1.dtype == "f32":
        assert np.array_equal(P1.A.data, P1.A.data.astype(np.float32).astype(np.float64))
        assert np.array_equal(P1.b, P1.b.astype(np.float32).astype(np.float64))


def test_morton_order_is_a_local_permutation():
    """The Morton order is a permutation; each 4 x 4 block of a frame takes 16 consecutive
    positions (the curve's locality), frames stay outermost."""
    from workloads.generators import morton_order
    N, nt = 16, 3
    o = morton_order(N, nt)
    assert sorted(o.tolist()) == list(range(N * N * nt))
    first = o[:16]
    ys, xs = first // N, first % N
    assert set(zip(ys.tolist(), xs.tolist())) == {(y, x) for y in range(4) for x in range(4)}
    assert set((o[N * N:2 * N * N] // (N * N)).tolist()) == {1}
