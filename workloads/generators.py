"""Seeded synthetic test problems for general-form Tikhonov regularisation.

This module builds inputs only: sparse operators A and L (as scipy CSR with
sorted int32 column indices), the true image x_true, the noisy data b and the
run parameters.  It holds none of the sGKS arithmetic, so both the FP64 CPU
oracle and the HIP path may consume what it produces.

Problem families (the paper's workloads stand-ins, Sec. 4):
  * 1D Gaussian deblurring with a dense Toeplitz blur (Sec. 4.1 uses PRblur;
    here a dense 256x256 Gaussian with rows normalised to sum 1).
  * 2D deblurring by a truncated 9x9 Gaussian PSF with zero boundary.
  * 2D parallel-beam CT, ray/pixel intersection lengths by Siddon tracing
    (Sec. 4.2.1 uses PRtomo).
  * Straight-ray travel-time tomography between boundary sources and
    receivers (Sec. 4.2.2 uses PRseismic, m about 6n).
  * Dynamic CT: block-diagonal A over frames, space-time difference operator
    (Sec. 4.3, eq:blockF, eq:spacetime_tik).
Noise follows Sec. 4: e is white Gaussian scaled so that ||e|| / ||A x|| is
exactly the requested level.

FP32 problems round A, L and b to float32 here; every consumer then sees the
same rounded values (the oracle upcasts them to float64).
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# container
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    name: str
    A: sp.csr_matrix          # m x n, float64 values (already FP32-rounded for f32 problems)
    L: sp.csr_matrix          # p x n
    b: np.ndarray             # m, float64 (FP32-rounded for f32 problems)
    x_true: np.ndarray        # n, float64
    mu: float                 # regularisation parameter (lambda in the paper)
    k: int                    # number of sGKS expansions
    s: int                    # sketch rows (s_A = s_L = s)
    seed: int                 # seed of the sketch (and of the data)
    dtype: str = "f64"        # bulk dtype of the GPU path: "f32" or "f64"
    zeta: int = 8             # nonzeros per sketch column
    ell: int = 3              # initial Krylov dimension
    refine_steps: int = 0     # iterative-refinement steps per projected solve
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def n(self):
        return self.A.shape[1]

    @property
    def p(self):
        return self.L.shape[0]


def _csr(rows, cols, vals, shape):
    M = sp.coo_matrix((vals, (rows, cols)), shape=shape).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return M


def _round32(M):
    M = M.copy()
    M.data = M.data.astype(np.float32).astype(np.float64)
    return M


def add_noise(b_true, level, rng):
    """b = b_true + e with ||e|| = level * ||b_true|| exactly, e ~ white Gaussian."""
    g = rng.standard_normal(b_true.shape[0])
    e = level * np.linalg.norm(b_true) * g / np.linalg.norm(g)
    return b_true + e


# ----------------------------------------------------------------------------
# regularisation operators
# ----------------------------------------------------------------------------

def diff1d(n):
    """(n-1) x n forward difference: row i is -e_i + e_{i+1} (eq: reg_matrix, D)."""
    i = np.arange(n - 1)
    rows = np.concatenate([i, i])
    cols = np.concatenate([i, i + 1])
    vals = np.concatenate([-np.ones(n - 1), np.ones(n - 1)])
    return _csr(rows, cols, vals, (n - 1, n))


def diff_axis(shape, axis):
    """Forward difference along one axis of a row-major grid, one row per unknown.

    Rows whose forward neighbour falls outside the grid are empty, so the
    operator has prod(shape) rows and L^T L equals that of the paper's
    (N-1) x N difference blocks."""
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    stride = int(np.prod(shape[axis + 1:]))
    sl = [slice(None)] * len(shape)
    sl[axis] = slice(0, shape[axis] - 1)
    src = idx[tuple(sl)].ravel()
    rows = np.concatenate([src, src])
    cols = np.concatenate([src, src + stride])
    vals = np.concatenate([-np.ones(src.size), np.ones(src.size)])
    return _csr(rows, cols, vals, (n, n))


def grad2d(N):
    """L = [I (x) D_x ; D_y (x) I] on an N x N image, x the fast index (2n rows)."""
    return sp.vstack([diff_axis((N, N), 1), diff_axis((N, N), 0)], format="csr")


def grad_spacetime(nt, N):
    """Psi = [spatial x; spatial y; temporal] on nt frames of N x N (3n rows)."""
    shape = (nt, N, N)
    return sp.vstack([diff_axis(shape, 2), diff_axis(shape, 1), diff_axis(shape, 0)],
                     format="csr")


def _fix_csr(M):
    M = M.tocsr()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return M


# ----------------------------------------------------------------------------
# forward operators
# ----------------------------------------------------------------------------

def blur1d_dense(n, sigma):
    """Dense Gaussian Toeplitz blur, every row normalised to sum 1 (all n^2 entries stored)."""
    i = np.arange(n)
    K = np.exp(-((i[:, None] - i[None, :]) ** 2) / (2.0 * sigma * sigma))
    K /= K.sum(axis=1, keepdims=True)
    rows = np.repeat(i, n)
    cols = np.tile(i, n)
    return _csr(rows, cols, K.ravel(), (n, n))


def psf_blur2d(N, sigma=2.0, half=4):
    """Convolution with a (2*half+1)^2 Gaussian PSF normalised to sum 1, zero boundary."""
    off = np.arange(-half, half + 1)
    dy, dx = np.meshgrid(off, off, indexing="ij")
    w = np.exp(-(dx ** 2 + dy ** 2) / (2.0 * sigma * sigma))
    w /= w.sum()
    iy, ix = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    iy = iy.ravel()
    ix = ix.ravel()
    rows, cols, vals = [], [], []
    for a in range(off.size):
        for c in range(off.size):
            qy = iy + off[a]
            qx = ix + off[c]
            ok = (qy >= 0) & (qy < N) & (qx >= 0) & (qx < N)
            rows.append((iy * N + ix)[ok])
            cols.append((qy * N + qx)[ok])
            vals.append(np.full(int(ok.sum()), w[a, c]))
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), (N * N, N * N))


def _siddon(N, p0, dirv, t0, t1):
    """Intersection lengths of straight segments with the pixels of an N x N grid.

    The grid covers [-N/2, N/2]^2 with unit pixels; pixel (iy, ix) is
    [-N/2+ix, -N/2+ix+1] x [-N/2+iy, -N/2+iy+1] and has index iy*N + ix.
    Segment r is {p0[r] + tau * dirv[r] : t0[r] <= tau <= t1[r]} with unit dirv.
    Returns (ray, pixel, length) triplets."""
    R = p0.shape[0]
    h = N / 2.0
    grid = np.arange(N + 1, dtype=np.float64) - h
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = (grid[None, :] - p0[:, 0:1]) / dirv[:, 0:1]
        ty = (grid[None, :] - p0[:, 1:2]) / dirv[:, 1:2]
    # clip to the square: parametric interval of the slab in each axis
    big = 1e300
    def slab(t, d):
        lo = np.where(np.abs(d) > 0, np.minimum(t[:, 0], t[:, -1]), -big)
        hi = np.where(np.abs(d) > 0, np.maximum(t[:, 0], t[:, -1]), big)
        return lo, hi
    lox, hix = slab(tx, dirv[:, 0])
    loy, hiy = slab(ty, dirv[:, 1])
    # rays parallel to an axis must lie strictly inside that axis' slab
    inx = np.where(np.abs(dirv[:, 0]) > 0, True, (p0[:, 0] > -h) & (p0[:, 0] < h))
    iny = np.where(np.abs(dirv[:, 1]) > 0, True, (p0[:, 1] > -h) & (p0[:, 1] < h))
    tmin = np.maximum(np.maximum(lox, loy), t0)
    tmax = np.minimum(np.minimum(hix, hiy), t1)
    ok = inx & iny & (tmax > tmin)
    tx = np.where(np.isfinite(tx), tx, np.nan)
    ty = np.where(np.isfinite(ty), ty, np.nan)
    T = np.concatenate([tx, ty, tmin[:, None], tmax[:, None]], axis=1)
    T = np.where((T >= tmin[:, None]) & (T <= tmax[:, None]), T, np.nan)
    T.sort(axis=1)                                   # NaN last
    dt = T[:, 1:] - T[:, :-1]
    mid = 0.5 * (T[:, 1:] + T[:, :-1])
    good = np.isfinite(dt) & (dt > 1e-12) & ok[:, None]
    rr, cc = np.nonzero(good)
    tm = mid[rr, cc]
    px = p0[rr, 0] + tm * dirv[rr, 0]
    py = p0[rr, 1] + tm * dirv[rr, 1]
    ix = np.floor(px + h).astype(np.int64)
    iy = np.floor(py + h).astype(np.int64)
    inside = (ix >= 0) & (ix < N) & (iy >= 0) & (iy < N)
    return rr[inside], (iy * N + ix)[inside], dt[rr, cc][inside]


def parallel_beam_ct(N, angles, ndet, det_spacing=1.0):
    """Parallel-beam CT matrix: one row per (angle, detector), angle-major.

    Detector offsets are (j - (ndet-1)/2) * spacing; the ray for angle theta
    and offset t is {t (cos th, sin th) + tau (-sin th, cos th)}."""
    t = (np.arange(ndet) - (ndet - 1) / 2.0) * det_spacing
    rows, cols, vals = [], [], []
    for a, th in enumerate(angles):
        c, s = math.cos(th), math.sin(th)
        p0 = np.stack([t * c, t * s], axis=1)
        d = np.tile(np.array([-s, c]), (ndet, 1))
        d[np.abs(d) < 1e-15] = 0.0
        r, q, v = _siddon(N, p0, d, np.full(ndet, -1e300), np.full(ndet, 1e300))
        rows.append(r + a * ndet)
        cols.append(q)
        vals.append(v)
    m = len(angles) * ndet
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), (m, N * N))


def boundary_points(N, side, u):
    """Point on side 0..3 (bottom, right, top, left) of the square [-N/2,N/2]^2 at fraction u."""
    h = N / 2.0
    pos = -h + u * N
    x = np.select([side == 0, side == 1, side == 2, side == 3], [pos, np.full_like(u, h), pos, np.full_like(u, -h)])
    y = np.select([side == 0, side == 1, side == 2, side == 3], [np.full_like(u, -h), pos, np.full_like(u, h), pos])
    return np.stack([x, y], axis=1)


def travel_time(N, m, rng):
    """Straight-ray travel-time matrix: m source/receiver pairs on different boundary sides."""
    s1 = rng.integers(0, 4, size=m)
    s2 = (s1 + rng.integers(1, 4, size=m)) % 4
    P = boundary_points(N, s1, rng.random(m))
    Q = boundary_points(N, s2, rng.random(m))
    d = Q - P
    ln = np.linalg.norm(d, axis=1)
    d = d / ln[:, None]
    d[np.abs(d) < 1e-15] = 0.0
    rows, cols, vals = [], [], []
    chunk = 4096
    for c0 in range(0, m, chunk):
        sl = slice(c0, min(m, c0 + chunk))
        r, q, v = _siddon(N, P[sl], d[sl], np.zeros(sl.stop - sl.start), ln[sl])
        rows.append(r + c0)
        cols.append(q)
        vals.append(v)
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), (m, N * N))


def perimeter_points(N, count, offset=0.0, inset=0.25):
    """count points equally spaced along the boundary of [-N/2, N/2]^2 (counter-clockwise
    from the bottom-left corner, arc-length parameter (j + offset) 4N / count), moved
    inset pixels into the square so that no ray runs along its edge."""
    u = (np.arange(count) + offset) * (4.0 * N / count)
    side = np.minimum((u // N).astype(np.int64), 3)
    h = N / 2.0 - inset
    pos = -h + (u - side * N) / N * (2 * h)
    x = np.select([side == 0, side == 1, side == 2, side == 3], [pos, np.full_like(u, h), -pos, np.full_like(u, -h)])
    y = np.select([side == 0, side == 1, side == 2, side == 3], [np.full_like(u, -h), pos, np.full_like(u, h), -pos])
    return np.stack([x, y], axis=1)


def travel_time_pairs(N, n_src, n_rec):
    """Straight-ray travel-time matrix between every source and every receiver (one row per
    pair, source-major): n_src sources and n_rec receivers equally spaced along the
    boundary, receivers offset by half a spacing."""
    S = perimeter_points(N, n_src, 0.0)
    R = perimeter_points(N, n_rec, 0.5)
    P = np.repeat(S, n_rec, axis=0)
    Q = np.tile(R, (n_src, 1))
    d = Q - P
    ln = np.linalg.norm(d, axis=1)
    d = d / ln[:, None]
    d[np.abs(d) < 1e-15] = 0.0
    m = P.shape[0]
    rows, cols, vals = [], [], []
    chunk = 4096
    for c0 in range(0, m, chunk):
        sl = slice(c0, min(m, c0 + chunk))
        r, q, v = _siddon(N, P[sl], d[sl], np.zeros(sl.stop - sl.start), ln[sl])
        rows.append(r + c0)
        cols.append(q)
        vals.append(v)
    return _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), (m, N * N))


# ----------------------------------------------------------------------------
# images
# ----------------------------------------------------------------------------

def _ellipse_mask(N, cx, cy, a, b, phi):
    c = np.arange(N) + 0.5
    Y, X = np.meshgrid(c, c, indexing="ij")
    dx = X - cx
    dy = Y - cy
    u = (dx * math.cos(phi) + dy * math.sin(phi)) / a
    v = (-dx * math.sin(phi) + dy * math.cos(phi)) / b
    return (u * u + v * v) <= 1.0


def random_ellipses(N, rng, count=8):
    img = np.zeros((N, N))
    for _ in range(count):
        cx, cy = rng.uniform(0.15, 0.85, size=2) * N
        a, b = rng.uniform(0.05, 0.25, size=2) * N
        phi = rng.uniform(0.0, math.pi)
        img[_ellipse_mask(N, cx, cy, a, b, phi)] += rng.uniform(0.2, 1.0)
    return img.ravel()


def phantom_ct(N, rng, inner=8):
    """An outer ellipse of intensity 1 plus random inner ellipses, clipped at zero."""
    img = np.zeros((N, N))
    img[_ellipse_mask(N, 0.5 * N, 0.5 * N, 0.46 * N, 0.36 * N, 0.0)] = 1.0
    for _ in range(inner):
        cx, cy = rng.uniform(0.3, 0.7, size=2) * N
        a, b = rng.uniform(0.04, 0.15, size=2) * N
        phi = rng.uniform(0.0, math.pi)
        img[_ellipse_mask(N, cx, cy, a, b, phi)] += rng.uniform(-0.5, 0.5)
    return np.clip(img, 0.0, None).ravel()


def step_signal(n, rng, pieces=6):
    br = np.sort(rng.choice(np.arange(1, n), size=pieces - 1, replace=False))
    h = rng.uniform(0.0, 1.0, size=pieces)
    x = np.empty(n)
    edges = np.concatenate([[0], br, [n]])
    for j in range(pieces):
        x[edges[j]:edges[j + 1]] = h[j]
    return x


def moving_ellipses(nt, N, rng, count=4):
    """count ellipses moving linearly at 1-2 px per frame; frames outermost."""
    params = []
    for _ in range(count):
        cx, cy = rng.uniform(0.3, 0.7, size=2) * N
        a, b = rng.uniform(0.06, 0.14, size=2) * N
        phi = rng.uniform(0.0, math.pi)
        speed = rng.uniform(1.0, 2.0)
        ang = rng.uniform(0.0, 2 * math.pi)
        vx, vy = speed * math.cos(ang), speed * math.sin(ang)
        # keep the whole track inside the image by starting it back by half the path
        cx -= 0.5 * (nt - 1) * vx
        cy -= 0.5 * (nt - 1) * vy
        params.append((cx, cy, a, b, phi, vx, vy, rng.uniform(0.3, 1.0)))
    frames = []
    for t in range(nt):
        img = np.zeros((N, N))
        for (cx, cy, a, b, phi, vx, vy, val) in params:
            img[_ellipse_mask(N, cx + t * vx, cy + t * vy, a, b, phi)] += val
        frames.append(img.ravel())
    return np.concatenate(frames)


# ----------------------------------------------------------------------------
# the five workloads (plus reduced-size variants for tests)
# ----------------------------------------------------------------------------

def deblur1d(seed=0, n=256, k=30, s=120, mu=1e-2, noise=0.01):
    rng = np.random.default_rng(seed)
    A = blur1d_dense(n, 3.0)
    L = diff1d(n)
    x = step_signal(n, rng)
    b = add_noise(A @ x, noise, rng)
    return Problem("deblur1d", A, L, b, x, mu, k, s, seed, dtype="f64",
                   meta=dict(n=n))


def deblur2d(seed=0, N=256, k=100, s=400, mu=5e-3, noise=0.01, dtype="f32"):
    rng = np.random.default_rng(seed)
    A = psf_blur2d(N)
    L = grad2d(N)
    x = random_ellipses(N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("deblur2d", A, L, b, x, mu, k, s, seed, dtype=dtype, meta=dict(N=N))


def ct2d(seed=0, N=256, n_angles=180, n_det=362, k=150, s=600, mu=1e-2, noise=0.01,
         refine_steps=2, dtype="f32"):
    rng = np.random.default_rng(seed)
    A = _ct_matrix(N, n_angles, n_det)
    L = grad2d(N)
    x = phantom_ct(N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("ct2d", A, L, b, x, mu, k, s, seed, dtype=dtype,
                   refine_steps=refine_steps, meta=dict(N=N, n_angles=n_angles, n_det=n_det))


@functools.lru_cache(maxsize=8)
def _ct_matrix(N, n_angles, n_det):
    angles = np.arange(n_angles) * math.pi / n_angles
    return parallel_beam_ct(N, angles, n_det)


def traveltime2d(seed=0, N=64, k=80, s=320, mu=1e-2, noise=0.01, dtype="f32", ratio=2):
    rng = np.random.default_rng(seed)
    A = travel_time(N, ratio * N * N, rng)
    L = grad2d(N)
    x = random_ellipses(N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("traveltime2d", A, L, b, x, mu, k, s, seed, dtype=dtype, meta=dict(N=N))


def dynamic_ct(seed=0, nt=30, N=128, n_angles=60, n_det=182, k=200, s=800, mu=1e-2,
               noise=0.01, dtype="f32"):
    """Block-diagonal dynamic CT: frame t uses angles i*pi/n_angles + t*pi/(n_angles*nt)."""
    rng = np.random.default_rng(seed)
    blocks = []
    for t in range(nt):
        ang = np.arange(n_angles) * math.pi / n_angles + t * math.pi / (n_angles * nt)
        blocks.append(parallel_beam_ct(N, ang, n_det))
    A = _fix_csr(sp.block_diag(blocks, format="csr"))
    L = _fix_csr(grad_spacetime(nt, N))
    x = moving_ellipses(nt, N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("dynamic_ct", A, L, b, x, mu, k, s, seed, dtype=dtype,
                   meta=dict(nt=nt, N=N, n_angles=n_angles, n_det=n_det))


# ----------------------------------------------------------------------------
# an order of the unknowns along a space-filling curve (Morton, per frame):
# neighbouring pixels get neighbouring positions, so the rows of A and L gather
# entries that share cache lines
# ----------------------------------------------------------------------------

def morton_order(N, nt=1):
    """order[i] = the row-major unknown (frame-major, then y, then x) at position i when
    each N x N frame is traversed along the Morton (Z) curve."""
    idx = np.arange(N * N, dtype=np.int64)
    y, x = idx // N, idx % N
    key = np.zeros(N * N, dtype=np.int64)
    for bit in range(16):
        key |= ((x >> bit) & 1) << (2 * bit)
        key |= ((y >> bit) & 1) << (2 * bit + 1)
    frame = np.argsort(key, kind="stable")
    return np.concatenate([t * N * N + frame for t in range(nt)]).astype(np.int32)


def image_order(P):
    """The Morton order of the unknowns of an image problem (None for the 1D deblurring)."""
    N = P.meta.get("N")
    if N is None:
        return None
    nt = P.meta.get("nt", 1)
    return morton_order(N, nt) if N * N * nt == P.n else None


# ----------------------------------------------------------------------------
# the paper's experiment shapes (Sec. 4.2.1, Sec. 4.2.2, Sec. 4.3) on synthetic data
# ----------------------------------------------------------------------------

def ct_exp2(seed=0, N=500, n_angles=120, n_det=500, k=300, s=606, mu=35.9, noise=0.01,
            dtype="f32"):
    """Exp. 2 shape: N x N parallel-beam CT, n_angles angles equally spaced over
    [0, 179] degrees, n_det unit-spaced detectors (m = 60,000 at the paper's size),
    first-difference L, 1% noise, the paper's lambda* = 35.9, s = 606, k = 300."""
    rng = np.random.default_rng(seed)
    angles = np.linspace(0.0, 179.0, n_angles) * math.pi / 180.0
    A = parallel_beam_ct(N, angles, n_det)
    L = grad2d(N)
    x = phantom_ct(N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("ct_exp2", A, L, b, x, mu, k, s, seed, dtype=dtype,
                   meta=dict(N=N, n_angles=n_angles, n_det=n_det))


def traveltime_exp3(seed=0, N=256, k=300, s=1000, mu=37.3, noise=0.01, dtype="f32"):
    """Exp. 3 shape: N x N travel-time tomography, 3N sources and 2N receivers along the
    boundary, every pair a ray (m = 6 N^2 = 393,216 at N = 256), first-difference L, 1%
    noise, the paper's lambda* ~ 37.3, k = 300, s one of the paper's sketch sizes."""
    rng = np.random.default_rng(seed)
    A = travel_time_pairs(N, 3 * N, 2 * N)
    L = grad2d(N)
    x = random_ellipses(N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("traveltime_exp3", A, L, b, x, mu, k, s, seed, dtype=dtype, meta=dict(N=N))


def dynamic_ct_exp4(seed=0, nt=10, N=256, n_angles=30, n_det=512, k=400, s=806, mu=6.81,
                    noise=0.001, dtype="f32"):
    """Exp. 4 shape: nt frames of N x N; frame t sees n_angles angles equally spaced in the
    t-th of nt equal sectors of [0, pi) (18 degrees each at nt = 10), n_det detectors
    (m = 153,600 at the paper's size), block-diagonal A, space-time L, 0.1% noise, the
    paper's lambda*_sGKS = 6.81, s = 806, k = 400."""
    rng = np.random.default_rng(seed)
    sector = math.pi / nt
    blocks = [parallel_beam_ct(N, t * sector + np.arange(n_angles) * sector / n_angles, n_det)
              for t in range(nt)]
    A = _fix_csr(sp.block_diag(blocks, format="csr"))
    L = _fix_csr(grad_spacetime(nt, N))
    x = moving_ellipses(nt, N, rng)
    b = add_noise(A @ x, noise, rng)
    if dtype == "f32":
        A, L, b = _round32(A), _round32(L), b.astype(np.float32).astype(np.float64)
    return Problem("dynamic_ct_exp4", A, L, b, x, mu, k, s, seed, dtype=dtype,
                   meta=dict(nt=nt, N=N, n_angles=n_angles, n_det=n_det))


def batch_specs(seed=0, count=32, sides=(64, 256)):
    """(kind, N, mu) of every problem of the uneven batch: types cycle deblur / CT /
    travel time; sides and mu log-uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(round(math.exp(rng.uniform(math.log(sides[0]), math.log(sides[1])))))
        mu = float(math.exp(rng.uniform(math.log(1e-3), math.log(1e-1))))
        out.append((("deblur2d", "ct2d", "traveltime2d")[i % 3], N, mu))
    return out


def batch_problem(i, seed=0, count=32, k=80, s=320, sides=(64, 256), dtype="f32"):
    """Problem i of the uneven batch (as batch_problems builds it)."""
    kind, N, mu = batch_specs(seed, count, sides)[i]
    if kind == "deblur2d":
        P = deblur2d(seed=seed + i, N=N, k=k, s=s, mu=mu, dtype=dtype)
    elif kind == "ct2d":
        n_det = int(math.ceil(N * math.sqrt(2.0)))
        P = ct2d(seed=seed + i, N=N, n_angles=max(8, (180 * N) // 256), n_det=n_det,
                 k=k, s=s, mu=mu, refine_steps=0, dtype=dtype)
    else:
        P = traveltime2d(seed=seed + i, N=N, k=k, s=s, mu=mu, dtype=dtype)
    P.seed = seed + i
    return P


def batch_problems(seed=0, count=32, k=80, s=320, sides=(64, 256), dtype="f32"):
    """Uneven batch: types cycle deblur / CT / travel time; sides log-uniform; mu log-uniform."""
    return [batch_problem(i, seed, count, k, s, sides, dtype) for i in range(count)]


def make(config, seed=0, scale="full"):
    """Problem(s) of one named workload.  scale="small" gives the reduced test sizes."""
    small = scale == "small"
    if config == "deblur1d":
        return deblur1d(seed) if not small else deblur1d(seed, n=96, k=20, s=60)
    if config == "deblur2d":
        return deblur2d(seed) if not small else deblur2d(seed, N=40, k=24, s=120)
    if config == "ct2d":
        return ct2d(seed) if not small else ct2d(seed, N=40, n_angles=45, n_det=57, k=20, s=100)
    if config == "dynamic_ct":
        return dynamic_ct(seed) if not small else dynamic_ct(seed, nt=4, N=24, n_angles=12,
                                                              n_det=35, k=20, s=100)
    if config == "ct_exp2":
        return ct_exp2(seed) if not small else ct_exp2(seed, N=40, n_angles=24, n_det=40, k=20,
                                                       s=60)
    if config == "traveltime_exp3":
        return (traveltime_exp3(seed) if not small else
                traveltime_exp3(seed, N=24, k=20, s=1500))
    if config == "dynamic_ct_exp4":
        return (dynamic_ct_exp4(seed) if not small else
                dynamic_ct_exp4(seed, nt=4, N=24, n_angles=8, n_det=48, k=20, s=100))
    if config == "batch":
        return batch_problems(seed) if not small else batch_problems(seed, count=5, k=12, s=60,
                                                                     sides=(16, 40))
    raise KeyError(config)


CONFIGS = ("deblur1d", "deblur2d", "ct2d", "batch", "dynamic_ct")
# the paper's experiment shapes (NEXT beyond the configs above)
PAPER_SCALE = ("ct_exp2", "traveltime_exp3", "dynamic_ct_exp4")
