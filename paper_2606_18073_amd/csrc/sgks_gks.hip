// GKS (Alg. 1) on gfx950: the baseline sGKS is measured against.
//
// One expansion differs from sGKS in two places.  The new basis column (the
// gradient of eq: gradient, written to W column d by the shared gradient
// kernels) is projected on the orthonormal columns before it by the projector
// of eq:single_mgs, once, and a second time when the loss ratio of
// eq:loss_criterion reaches kGksTau; it is normalised through its column scale.
// And the QR factors are those of the unsketched A V (m x d) and L V (p x d),
// extended by rank-one appends (eq:updqr) on the m- and p-vectors A v, L v, with
// d_A gaining q^T b (eq:dA_update).  The projected solve is the stacked step of
// sGKS on the same small factors.
//
// Every product here is a tall dense matrix-vector product (n x d, m x d,
// p x d), HBM bound: the column dots stage a slab of the vector in LDS and
// each wave streams whole columns of the slab; the updates take one row per
// thread with eight column loads in flight.  Partial results are reduced in
// fixed orders (bitwise reproducible runs).  The kernels read the device State
// of one problem and skip all work once its status word is set.
#include "sgks_device.h"

namespace sgks {

constexpr int kGksBlock = 256;
constexpr int kGksMaxRows = 4096;   // rows of a slab staged in LDS (32 KiB)
constexpr int kGksMaxBlocks = 512;  // slabs per side
// tsq: five rows of kGksSumLd partial sums, indexed by the workgroup of the
// launch that writes them: 0 ||a||^2 (A-side dots), 1 ||l||^2 (L-side dots),
// 2 ||w_A||^2, 3 ||w_L||^2, 4 w_A . b (last update)
constexpr int kGksSumLd = 4096;

// partial[j] = cs_j sum_{i < nr} M[j ldm + i] v_i, j < d (cs may be null: 1),
// v (times vscale) staged in vs; wave w takes four columns at a time
__device__ void slab_coldots(const double* __restrict__ M, int64_t ldm, const double* __restrict__ v,
                             double vscale, int nr, int d, const double* __restrict__ cs,
                             double* __restrict__ partial, double* vs) {
    for (int i = threadIdx.x; i < nr; i += kGksBlock) vs[i] = vscale * v[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kGksBlock / 64;
    for (int j0 = 4 * wave; j0 < d; j0 += 4 * nw) {
        const double* c0 = M + (int64_t)j0 * ldm;
        const int jn = min(4, d - j0);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = lane; i < nr; i += 64) {
            double q[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = c < jn ? c0[(int64_t)c * ldm + i] : 0.0;
            const double vi = vs[i];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += q[c] * vi;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double a = wave_sum(acc[c]);
            if (lane == 0 && c < jn) partial[j0 + c] = cs ? a * cs[j0 + c] : a;
        }
    }
}

// Column dots of the V projection: part[b dmax + j] = w_j . v over slab b,
// v = W column d, w_j = cs_j W column j, j < d.
__global__ __launch_bounds__(kGksBlock) void kg_vdots(const State* __restrict__ SS) {
    __shared__ double vs[kGksMaxRows];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d;
    const int64_t r0 = (int64_t)blockIdx.x * S.gt_rows;
    const int nr = (int)min((int64_t)S.gt_rows, S.n - r0);
    slab_coldots(S.W + r0, S.n, S.W + (int64_t)d * S.n + r0, 1.0, nr, d, S.cs,
                 S.gpart + (int64_t)blockIdx.x * S.dmax, vs);
}

// coef[j] = sum_b part[b ld + j] over nb slabs, one workgroup per column j < d
// (the workgroups of columns >= d leave); fixed order
__device__ void colsum_body(const double* __restrict__ part, int nb, int64_t ld, int j,
                            double* out, double* red) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += kGksBlock) a += part[(int64_t)b * ld + j];
    a = block_sum(a, red);
    if (threadIdx.x == 0) *out = a;
}

// which = 0: V projection pass `pass` (coefficients to gco[pass dmax + j]);
// which = 1: tall appends pass `pass`: workgroups [0, dmax) the A side
// (gco[(2 + 2 pass) dmax + j]), [dmax, 2 dmax) the L side
// (gco[(3 + 2 pass) dmax + j]); the running sums p_A, p_L of the coefficients
// go to pacc[2 dmax + j], pacc[3 dmax + j] (the R columns)
__global__ __launch_bounds__(kGksBlock) void kg_colsum(const State* __restrict__ SS, int which,
                                                      int pass) {
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d, dmax = S.dmax;
    if (which == 0) {
        const int j = blockIdx.x;
        if (j >= d) return;
        colsum_body(S.gpart, S.ngt, dmax, j, S.gco + (int64_t)pass * dmax + j, red);
        return;
    }
    const int side = blockIdx.x >= dmax ? 1 : 0;
    const int j = blockIdx.x - side * dmax;
    if (j >= d) return;
    double* out = S.gco + (int64_t)(2 + 2 * pass + side) * dmax + j;
    colsum_body(side ? S.tpL : S.tpA, side ? S.ntL : S.ntA, dmax, j, out, red);
    if (threadIdx.x == 0) {
        double* acc = S.pacc + (int64_t)(2 + side) * dmax + j;
        *acc = (pass == 0 ? 0.0 : *acc) + *out;
    }
}

// out[i] = base_scale base[i] - sum_{j < d} M[j ldm + i] cf_j (cs_j), rows
// [r0, r1) grid-stride; returns this thread's sum of out^2 and of out * bv[i]
// (bv may be null)
__device__ void rows_update(const double* __restrict__ M, int64_t ldm, const double* __restrict__ cs,
                            const double* __restrict__ cf, int d, const double* base, double base_scale,
                            double* out, const double* __restrict__ bv, int64_t rows, int blk,
                            int nblk, double* yt, double& sq, double& sb) {
    for (int j = threadIdx.x; j < d; j += kGksBlock) yt[j] = cs ? cs[j] * cf[j] : cf[j];
    __syncthreads();
    sq = 0.0;
    sb = 0.0;
    for (int64_t i = (int64_t)blk * kGksBlock + threadIdx.x; i < rows;
         i += (int64_t)nblk * kGksBlock) {
        const double* m = M + i;
        double acc = 0.0;
        int j = 0;
        for (; j + 8 <= d; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = m[(int64_t)(j + u) * ldm];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u] * yt[j + u];
        }
        for (; j < d; ++j) acc += m[(int64_t)j * ldm] * yt[j];
        const double o = base_scale * base[i] - acc;
        out[i] = o;
        sq += o * o;
        if (bv) sb += o * bv[i];
    }
}

// V projection update of pass `pass`: W column d -= V gco[pass] (V = W columns
// scaled by cs); partial sums of ||v||^2 to vsq[pass 2048 + blk].  Pass 1 runs
// only when the loss ratio after pass 0, ||V^T v|| / ||v|| (eq:loss_criterion),
// is at least kGksTau; every workgroup evaluates it from the same partial sums in
// the same order, and workgroup 0 records the decision in scal[7].
__global__ __launch_bounds__(kGksBlock) void kg_vupdate(const State* __restrict__ SS, int pass) {
    __shared__ double yt[kMaxD];
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d, dmax = S.dmax;
    const double* cf = S.gco + (int64_t)pass * dmax;
    if (pass == 1) {
        double c2 = 0.0, v2 = 0.0;
        for (int j = threadIdx.x; j < d; j += kGksBlock) c2 += cf[j] * cf[j];
        for (int b = threadIdx.x; b < (int)gridDim.x; b += kGksBlock) v2 += S.vsq[b];
        c2 = block_sum(c2, red);
        v2 = block_sum(v2, red);
        const bool second = sqrt(c2) >= kGksTau * sqrt(v2);
        if (blockIdx.x == 0 && threadIdx.x == 0) S.scal[7] = second ? 1.0 : 0.0;
        if (!second) return;
    }
    double* col = S.W + (int64_t)d * S.n;
    double sq, sb;
    rows_update(S.W, S.n, S.cs, cf, d, col, 1.0, col, nullptr, S.n, blockIdx.x, gridDim.x, yt,
                sq, sb);
    sq = block_sum(sq, red);
    if (threadIdx.x == 0) S.vsq[(int64_t)pass * 2048 + blockIdx.x] = sq;
}

// After the projection: ||v|| of the first pass decides breakdown (at most
// 1e-14 ||A^T b||: the space stopped growing), the final ||v|| the column scale.
__global__ __launch_bounds__(kGksBlock) void kg_vfinish(const State* __restrict__ SS, int nb) {
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d;
    double v0 = 0.0, v1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += kGksBlock) {
        v0 += S.vsq[b];
        v1 += S.vsq[2048 + b];
    }
    v0 = block_sum(v0, red);
    v1 = block_sum(v1, red);
    if (threadIdx.x == 0) {
        const double n0 = sqrt(v0);
        const double nf = S.scal[7] != 0.0 ? sqrt(v1) : n0;
        if (!(v0 < INFINITY) || !(nf < INFINITY))
            *S.status = kStatusNonfinite;
        else if (!(n0 > 1e-14 * S.scal[0]))
            *S.status = kStatusBreakdown;
        else
            S.cs[d] = 1.0 / nf;
    }
}

// Column dots of the tall appends, pass `pass`: workgroups [0, ntA) slabs of
// the m rows of Q_A with a = cs_d u (pass 0) or the working wat (pass 1),
// workgroups [ntA, ntA + ntL) slabs of the p rows of Q_L with cs_d t or wlt.
// Pass 0 also sums ||a||^2 (||l||^2) of its slab into tsq row 0 (row 1).
__global__ __launch_bounds__(kGksBlock) void kg_tdots(const State* __restrict__ SS, int pass) {
    __shared__ double vs[kGksMaxRows];
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d;
    const int side = (int)blockIdx.x >= S.ntA ? 1 : 0;
    const int b = blockIdx.x - side * S.ntA;
    const int rows_per = side ? S.trL : S.trA;
    const int64_t rows = side ? S.p : S.m;
    const int64_t r0 = (int64_t)b * rows_per;
    const int nr = (int)min((int64_t)rows_per, rows - r0);
    const double* v = pass == 0 ? (side ? S.t : S.u) : (side ? S.wlt : S.wat);
    const double sc = pass == 0 ? S.cs[d] : 1.0;
    slab_coldots((side ? S.QLt : S.QAt) + r0, rows, v + r0, sc, nr, d, nullptr,
                 (side ? S.tpL : S.tpA) + (int64_t)b * S.dmax, vs);
    if (pass == 0) {
        double sq = 0.0;
        for (int i = threadIdx.x; i < nr; i += kGksBlock) sq += vs[i] * vs[i];
        sq = block_sum(sq, red);
        if (threadIdx.x == 0) S.tsq[(int64_t)side * kGksSumLd + blockIdx.x] = sq;
    }
}

// Update of the tall appends, pass `pass`: wat = (pass 0 ? cs_d u : wat) - Q_A c,
// wlt likewise with Q_L; the last pass sums ||wat||^2, ||wlt||^2 and wat . b
// per workgroup (tsq rows 2, 3, 4).  Workgroups [0, gA) take the A side.
__global__ __launch_bounds__(kGksBlock) void kg_tupdate(const State* __restrict__ SS, int pass,
                                                       int last, int gA) {
    __shared__ double yt[kMaxD];
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d, dmax = S.dmax;
    const int side = (int)blockIdx.x >= gA ? 1 : 0;
    const int blk = blockIdx.x - side * gA, nblk = side ? (int)gridDim.x - gA : gA;
    const double* cf = S.gco + (int64_t)(2 + 2 * pass + side) * dmax;
    double* w = side ? S.wlt : S.wat;
    const double* base = pass == 0 ? (side ? S.t : S.u) : w;
    const double bsc = pass == 0 ? S.cs[d] : 1.0;
    double sq, sb;
    rows_update(side ? S.QLt : S.QAt, side ? S.p : S.m, nullptr, cf, d, base, bsc, w,
                (last && !side) ? S.b : nullptr, side ? S.p : S.m, blk, nblk, yt, sq, sb);
    if (!last) return;
    sq = block_sum(sq, red);
    sb = block_sum(sb, red);
    if (threadIdx.x == 0) {
        S.tsq[(int64_t)(2 + side) * kGksSumLd + blockIdx.x] = sq;
        if (!side) S.tsq[(int64_t)4 * kGksSumLd + blockIdx.x] = sb;
    }
}

// Finish of the tall appends: every workgroup reduces the sums (same order),
// rho = ||w_perp|| (0 and q = 0 when it keeps at most 1e-14 of ||a||), writes
// its slab of the new Q columns; workgroup 0 writes the R columns (p from pacc,
// rho on the diagonal), d_A[d] = q_A . b and rho_A, rho_L for the stacked step.
__global__ __launch_bounds__(kGksBlock) void kg_tfinish(const State* __restrict__ SS, int gA,
                                                       int gL) {
    __shared__ double red[kGksBlock / 64];
    const State S = load_state(SS, 0);
    if (*S.status != 0) return;
    const int d = *S.d, dmax = S.dmax;
    const int64_t ld = kGksSumLd;
    double a2 = 0.0, l2 = 0.0, ra = 0.0, rl = 0.0, db = 0.0;
    for (int b = threadIdx.x; b < S.ntA + S.ntL; b += kGksBlock) {
        a2 += b < S.ntA ? S.tsq[b] : 0.0;
        l2 += b >= S.ntA ? S.tsq[ld + b] : 0.0;
    }
    for (int b = threadIdx.x; b < gA + gL; b += kGksBlock) {
        ra += b < gA ? S.tsq[2 * ld + b] : 0.0;
        rl += b >= gA ? S.tsq[3 * ld + b] : 0.0;
        db += b < gA ? S.tsq[4 * ld + b] : 0.0;
    }
    a2 = block_sum(a2, red);
    l2 = block_sum(l2, red);
    ra = block_sum(ra, red);
    rl = block_sum(rl, red);
    db = block_sum(db, red);
    double rhoA = sqrt(ra), rhoL = sqrt(rl);
    const bool degA = !(rhoA > 1e-14 * sqrt(a2)), degL = !(rhoL > 1e-14 * sqrt(l2));
    if (degA) rhoA = 0.0;
    if (degL) rhoL = 0.0;
    const double qa = degA ? 0.0 : 1.0 / rhoA, ql = degL ? 0.0 : 1.0 / rhoL;
    const int side = (int)blockIdx.x >= gA ? 1 : 0;
    const int blk = blockIdx.x - side * gA, nblk = side ? gL : gA;
    const int64_t rows = side ? S.p : S.m;
    const double* w = side ? S.wlt : S.wat;
    double* q = (side ? S.QLt : S.QAt) + (int64_t)d * rows;
    const double sc = side ? ql : qa;
    for (int64_t i = (int64_t)blk * kGksBlock + threadIdx.x; i < rows;
         i += (int64_t)nblk * kGksBlock)
        q[i] = w[i] * sc;
    if (blockIdx.x != 0) return;
    for (int j = threadIdx.x; j < d; j += kGksBlock) {
        S.RA[(int64_t)d * dmax + j] = S.pacc[2 * dmax + j];
        S.RL[(int64_t)d * dmax + j] = S.pacc[3 * dmax + j];
    }
    if (threadIdx.x == 0) {
        S.RA[(int64_t)d * dmax + d] = rhoA;
        S.RL[(int64_t)d * dmax + d] = rhoL;
        S.scal[12] = rhoA;
        S.scal[13] = rhoL;
        S.dA[d] = degA ? 0.0 : db / rhoA;
        if (!(ra < INFINITY) || !(rl < INFINITY)) *S.status = kStatusNonfinite;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int gks_tall_blocks(int64_t rows, int* rows_per_block) {
    int64_t rpb = (rows + kGksMaxBlocks - 1) / kGksMaxBlocks;
    rpb = ((rpb + 63) / 64) * 64;
    if (rpb < 256) rpb = 256;
    if (rpb > kGksMaxRows) rpb = kGksMaxRows;
    *rows_per_block = (int)rpb;
    return (int)((rows + rpb - 1) / rpb);
}

static int update_blocks(int64_t rows) { return grid_for(rows, kGksBlock, 2048); }

void gks_project(const State& S, const State* Sdev, hipStream_t st) {
    const int nb = update_blocks(S.n);
    for (int pass = 0; pass < 2; ++pass) {
        SGKS_LAUNCH(kg_vdots, dim3(S.ngt), dim3(kGksBlock), 0, st, Sdev);
        SGKS_LAUNCH(kg_colsum, dim3(S.dmax), dim3(kGksBlock), 0, st, Sdev, 0, pass);
        SGKS_LAUNCH(kg_vupdate, dim3(nb), dim3(kGksBlock), 0, st, Sdev, pass);
    }
    SGKS_LAUNCH(kg_vfinish, dim3(1), dim3(kGksBlock), 0, st, Sdev, nb);
}

void gks_append(const State& S, const State* Sdev, hipStream_t st) {
    const int gA = update_blocks(S.m), gL = update_blocks(S.p);
    for (int pass = 0; pass < S.passes; ++pass) {
        const int last = pass == S.passes - 1;
        SGKS_LAUNCH(kg_tdots, dim3(S.ntA + S.ntL), dim3(kGksBlock), 0, st, Sdev, pass);
        SGKS_LAUNCH(kg_colsum, dim3(2 * S.dmax), dim3(kGksBlock), 0, st, Sdev, 1, pass);
        SGKS_LAUNCH(kg_tupdate, dim3(gA + gL), dim3(kGksBlock), 0, st, Sdev, pass, last, gA);
    }
    SGKS_LAUNCH(kg_tfinish, dim3(gA + gL), dim3(kGksBlock), 0, st, Sdev, gA, gL);
}

}  // namespace sgks
