// HIP kernels of the sGKS hot path for gfx950 (CDNA4, wave64).
//
// Bulk kernels are bandwidth bound (sparse and dense matrix-vector products,
// O(1) flop per byte): CSR rows are processed by groups of `lanes` lanes of a
// wavefront with a power-of-two group width, FP64 accumulation, and shuffle
// reductions inside the group; workgroups take row ranges in an XCD-aware
// order.  The sparse-sign sketch is a scatter of the new column's images
// through the embedding's pattern (computed once from its counter-based hash
// and kept as int16 signed rows): each wave adds its tiles into private LDS
// bins and the partial bins are merged in a fixed order, so results are
// reproducible run to run.  The small FP64 steps (rank-one QR appends on the
// sketched matrices, the stacked projected factor and the projected solve)
// are a few one-workgroup launches per problem, or, for large sketches, a
// chain of launches whose workgroups each own a slab of rows.  Every kernel
// reads its problem from a device array of States through a table of
// workgroup ranges, so a batch of problems shares each launch.
#include <hipcub/hipcub.hpp>

#include <vector>

#include "sgks_device.h"

namespace sgks {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Totals of N = 2^m values per lane over the 64 lanes of a wave, transposed:
// each of the first m butterfly steps sends half of the lane's values to its
// partner and keeps the other half, so that lane l ends with value
// l / (64 / N); the remaining steps sum within groups of 64 / N lanes.  Every
// lane of a group returns the same total (a fixed order, as for wave_sum), at
// about 2 N + 6 - m shuffles instead of 6 N.
template <int N>
__device__ __forceinline__ double wave_sum_scatter(const double (&v)[N]) {
    static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "power-of-two count");
    const int lane = threadIdx.x & 63;
    double w[N];
#pragma unroll
    for (int n = 0; n < N; ++n) w[n] = v[n];
    int off = 32;
#pragma unroll
    for (int half = N / 2; half >= 1; half >>= 1) {
        const bool up = (lane & off) != 0;
#pragma unroll
        for (int n = 0; n < half; ++n) {
            const double send = up ? w[n] : w[n + half];
            const double keep = up ? w[n + half] : w[n];
            w[n] = keep + __shfl_xor(send, off);
        }
        off >>= 1;
    }
    double t = w[0];
#pragma unroll
    for (int o = 32 / N; o > 0; o >>= 1) t += __shfl_xor(t, o);
    return t;
}

template <int V>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = V / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int B = 16>
__device__ __forceinline__ double strided_dot(const double* __restrict__ p, int64_t stride,
                                              const double* v, int n) {
    double acc = 0.0;
    for (int k = 0; k < n; k += B) {
        double w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) w[u] = p[(int64_t)min(k + u, n - 1) * stride];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < n) acc += w[u] * v[k + u];
    }
    return acc;
}

// Element (i, j) of an upper-triangular matrix in memory at p[i rs + j cs]
// (only i <= j is read).
struct GTri {
    const double* __restrict__ p;
    int64_t rs, cs;
    __device__ __forceinline__ double operator()(int i, int j) const {
        return p[(int64_t)i * rs + (int64_t)j * cs];
    }
};
// Product of an upper-triangular d x d matrix M with v by the first NT
// threads of the block (the others return at once):
//   trans = 0: out[k] = sum_{j >= k} M(k, j) v[j]
//   trans = 1: out[k] = sum_{i <= k} M(i, k) v[i]
// Loads in flight per lane in the small triangular products (latency bound:
// one workgroup, the matrix in L2).  16 and 32 measured slower than 8 (the
// one-workgroup append launch 48.3 and 56.4 vs 44.8 us on the deblurring
// workload): more clamped loads past the row ends and fewer waves.
constexpr int kTriChunk = 8;

// Groups of tpr lanes share one output, each lane taking every tpr-th term
// with kTriChunk loads in flight; the group sums with shuffles (fixed order, the
// same for every accessor).
template <class Mat>
__device__ void tri_mv_t(const Mat& M, int d, int trans, const double* v, double* out,
                         int NT) {
    if ((int)threadIdx.x >= NT) return;
    int tpr = 64;
    while (tpr > 1 && NT / tpr < d) tpr >>= 1;
    const int rpp = NT / tpr;
    const int c = threadIdx.x % tpr;
    for (int base = 0; base < d; base += rpp) {
        const int k = base + threadIdx.x / tpr;
        double acc = 0.0;
        if (k < d) {
            // trans 0: row k from the diagonal on; 1: column k down to the
            // diagonal; 2: the whole row k
            const int lo = trans == 0 ? k : 0, hi = trans == 1 ? k + 1 : d;
            for (int q = lo + c; q < hi; q += kTriChunk * tpr) {
                double w[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int idx = min(q + u * tpr, hi - 1);   // clamped: loads stay unconditional
                    w[u] = trans == 1 ? M(idx, k) : M(k, idx);
                }
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int idx = q + u * tpr;
                    if (idx < hi) acc += w[u] * v[idx];
                }
            }
        }
        for (int off = tpr / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (k < d && c == 0) out[k] = acc;
    }
}

__device__ void tri_mv(const double* __restrict__ M, int64_t rs, int64_t cs, int d, int trans,
                       const double* v, double* out) {
    tri_mv_t(GTri{M, rs, cs}, d, trans, v, out, blockDim.x);
}

// out1[k] = sum_{j >= k, j < d} M(k, j) v1[j], out2[k] likewise with v2; the
// tri_mv scheme with both products sharing the loads of M.
template <class Mat>
__device__ void tri_mv2_t(const Mat& M, int d, const double* v1, const double* v2, double* out1,
                          double* out2, int NT) {
    if ((int)threadIdx.x >= NT) return;
    int tpr = 64;
    while (tpr > 1 && NT / tpr < d) tpr >>= 1;
    const int rpp = NT / tpr;
    const int c = threadIdx.x % tpr;
    for (int base = 0; base < d; base += rpp) {
        const int k = base + threadIdx.x / tpr;
        double a1 = 0.0, a2 = 0.0;
        if (k < d) {
            for (int q = k + c; q < d; q += kTriChunk * tpr) {
                double w[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) w[u] = M(k, min(q + u * tpr, d - 1));
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int idx = q + u * tpr;
                    if (idx < d) {
                        a1 += w[u] * v1[idx];
                        a2 += w[u] * v2[idx];
                    }
                }
            }
        }
        for (int off = tpr / 2; off > 0; off >>= 1) {
            a1 += __shfl_xor(a1, off);
            a2 += __shfl_xor(a2, off);
        }
        if (k < d && c == 0) {
            out1[k] = a1;
            out2[k] = a2;
        }
    }
}

// Two upper-triangular d x d matrices Ma, Mb; groups of tpr lanes share one
// output as in tri_mv_t.
//   tri_dot2t_t:  out[k] = sum_{i <= k} (Ma(i, k) va[i] + Mb(i, k) vb[i])
//   tri_apply2_t: outa[i] = sum_{k >= i} Ma(i, k) v[k], outb[i] = sum_{k >= i} Mb(i, k) v[k]
template <class Mat>
__device__ void tri_dot2t_t(const Mat& Ma, const Mat& Mb, int d, const double* va,
                            const double* vb, double* out, int NT) {
    if ((int)threadIdx.x >= NT) return;
    int tpr = 64;
    while (tpr > 1 && NT / tpr < d) tpr >>= 1;
    const int rpp = NT / tpr;
    const int c = threadIdx.x % tpr;
    for (int base = 0; base < d; base += rpp) {
        const int k = base + threadIdx.x / tpr;
        double acc = 0.0;
        if (k < d) {
            for (int q = c; q <= k; q += kTriChunk * tpr) {
                double wa[kTriChunk], wb[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int i = min(q + u * tpr, k);
                    wa[u] = Ma(i, k);
                    wb[u] = Mb(i, k);
                }
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int i = q + u * tpr;
                    if (i <= k) acc += wa[u] * va[i] + wb[u] * vb[i];
                }
            }
        }
        for (int off = tpr / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (k < d && c == 0) out[k] = acc;
    }
}

template <class Mat>
__device__ void tri_apply2_t(const Mat& Ma, const Mat& Mb, int d, const double* v, double* outa,
                             double* outb, int NT) {
    if ((int)threadIdx.x >= NT) return;
    int tpr = 64;
    while (tpr > 1 && NT / tpr < d) tpr >>= 1;
    const int rpp = NT / tpr;
    const int c = threadIdx.x % tpr;
    for (int base = 0; base < d; base += rpp) {
        const int i = base + threadIdx.x / tpr;
        double aa = 0.0, ab = 0.0;
        if (i < d) {
            for (int q = i + c; q < d; q += kTriChunk * tpr) {
                double wa[kTriChunk], wb[kTriChunk];
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int k = min(q + u * tpr, d - 1);
                    wa[u] = Ma(i, k);
                    wb[u] = Mb(i, k);
                }
#pragma unroll
                for (int u = 0; u < kTriChunk; ++u) {
                    const int k = q + u * tpr;
                    if (k < d) {
                        aa += wa[u] * v[k];
                        ab += wb[u] * v[k];
                    }
                }
            }
        }
        for (int off = tpr / 2; off > 0; off >>= 1) {
            aa += __shfl_xor(aa, off);
            ab += __shfl_xor(ab, off);
        }
        if (i < d && c == 0) {
            outa[i] = aa;
            outb[i] = ab;
        }
    }
}

__device__ void tri_mv2(const double* __restrict__ M, int64_t rs, int64_t cs, int d,
                        const double* v1, const double* v2, double* out1, double* out2) {
    tri_mv2_t(GTri{M, rs, cs}, d, v1, v2, out1, out2, blockDim.x);
}

__device__ void tri_dot2t(const double* __restrict__ Ma, const double* __restrict__ Mb,
                          int64_t rs, int64_t cs, int d, const double* va, const double* vb,
                          double* out) {
    tri_dot2t_t(GTri{Ma, rs, cs}, GTri{Mb, rs, cs}, d, va, vb, out, blockDim.x);
}

__device__ void tri_apply2(const double* __restrict__ Ma, const double* __restrict__ Mb,
                           int64_t rs, int64_t cs, int d, const double* v, double* outa,
                           double* outb) {
    tri_apply2_t(GTri{Ma, rs, cs}, GTri{Mb, rs, cs}, d, v, outa, outb, blockDim.x);
}

// Dot product of one CSR row with x by the V lanes of a group (lane g of V).
// acc += sum_u va[k + u V] x[ci[k + u V]], u < U, in u order: all U index and
// value loads are issued before the gathers
template <int U, int V, typename T>
__device__ __forceinline__ void row_chunk(const int32_t* __restrict__ ci, const T* __restrict__ va,
                                          const double* __restrict__ x, int k, double& acc) {
    int c[U];
    T w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        c[u] = ci[k + u * V];
        w[u] = va[k + u * V];
    }
    double xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (double)w[u] * xv[u];
}

// In the masked form, rows split over at least this many lanes take masked
// chunks (below).
constexpr int kMaskedRowMinLanes = 8;

template <int V, typename T, bool Masked = false>
__device__ __forceinline__ double row_dot(const Csr& M, const double* __restrict__ x, int64_t row,
                                          int g) {
    const int32_t* __restrict__ ci = M.col;
    const T* __restrict__ va = (const T*)M.val;
    const int beg = M.rowptr[row], end = M.rowptr[row + 1];
    double acc = 0.0;
    if constexpr (Masked && V >= kMaskedRowMinLanes) {
        // wide groups: a lane's share of a row is short, so every chunk is eight
        // (index, value) loads from clamped addresses (all in flight, then the
        // eight gathers) and the terms past the row's end are masked: one
        // dependent round trip per eight entries of a lane instead of separate
        // chunks of eight, four, two and one.  Same terms in the same order.
        // Faster for the batch (its long ray rows on 16 to 64 lanes: 27,900 vs
        // 25,000 problem-expansions/s); slower for a single problem, whose
        // adjoint then takes wave slots and issue cycles from the append chain
        // beside it (CT 3,914 vs 4,080 iterations/s), so only batched plans use it.
        for (int k = beg + g; k < end; k += 8 * V) {
            int c[8];
            T w[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = min(k + u * V, end - 1);
                c[u] = ci[q];
                w[u] = va[q];
            }
            double xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k + u * V < end) acc += (double)w[u] * xv[u];
        }
        return group_sum<V>(acc);
    }
    int k = beg + g;
    // eight (then four, two) entries per lane in flight before the gathers of x
    for (; k + 7 * V < end; k += 8 * V) row_chunk<8, V>(ci, va, x, k, acc);
    if (k + 3 * V < end) {
        row_chunk<4, V>(ci, va, x, k, acc);
        k += 4 * V;
    }
    if (k + V < end) {
        row_chunk<2, V>(ci, va, x, k, acc);
        k += 2 * V;
    }
    if (k < end) acc += (double)va[k] * x[ci[k]];
    return group_sum<V>(acc);
}

#define SGKS_LANES_SWITCH(lanes, ...)                                   \
    switch (lanes) {                                                    \
        case 1: { constexpr int V = 1; __VA_ARGS__ } break;            \
        case 2: { constexpr int V = 2; __VA_ARGS__ } break;            \
        case 4: { constexpr int V = 4; __VA_ARGS__ } break;            \
        case 8: { constexpr int V = 8; __VA_ARGS__ } break;            \
        case 16: { constexpr int V = 16; __VA_ARGS__ } break;          \
        case 32: { constexpr int V = 32; __VA_ARGS__ } break;          \
        default: { constexpr int V = 64; __VA_ARGS__ } break;          \
    }

// ---------------------------------------------------------------------------
// sparse-sign pattern: SplitMix64 finaliser, zeta distinct rows per column
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

// Rows and signs of column j of the stream's embedding (s rows).  Slot q
// takes successive draws until its row is new for the column.  The cap on
// draws only guards termination (s >= Z is validated on the host; needing it
// is astronomically unlikely).
template <int Z>
__device__ __forceinline__ void sketch_column(uint64_t seed, int stream, int64_t j, int s,
                                              int* bin, double* sg) {
    const uint64_t gam = 0x9E3779B97F4A7C15ull;
    const uint64_t key = mix64(seed + gam * (uint64_t)(2 * j + stream + 1));
    uint64_t c = 1;
#pragma unroll
    for (int q = 0; q < Z; ++q) {
        for (;;) {
            const uint64_t z = mix64(key + gam * c);
            ++c;
            const int row = (int)(((z >> 32) * (uint64_t)(uint32_t)s) >> 32);
            bool dup = false;
#pragma unroll
            for (int u = 0; u < q; ++u) dup |= (bin[u] == row);
            if (!dup || c > 4096) {
                bin[q] = row;
                sg[q] = dup ? 0.0 : ((z & 1ull) ? -1.0 : 1.0);
                break;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// conversions and small reductions
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_f64(const T* __restrict__ src,
                                                  double* __restrict__ dst, int64_t n,
                                                  double* part) {
    __shared__ double red[kWaves];
    double sq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double v = (double)src[i];
        dst[i] = v;
        sq += v * v;
    }
    const double t = block_sum(sq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_sum_parts(const double* part, int nb, double* out) {
    __shared__ double red[kWaves];
    const double t = block_sum(thread_strided_sum(part, nb, kBlock), red);
    if (threadIdx.x == 0) out[0] = t;
}

// ---------------------------------------------------------------------------
// XCD-aware workgroup order
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Logical index of workgroup j of n: the workgroups of one XCD get
// consecutive logical indices, hence neighbouring rows, so the vector entries
// their rows gather stay in that XCD's L2 (a bijection on [0, n)).
__device__ __forceinline__ int xcd_order(int j, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X, k = j % X;
    return k * q + min(k, r) + j / X;
}

__device__ __forceinline__ int rows_blocks_of(const Csr& M) {
    const uint32_t per = (uint32_t)(kBlock / M.lanes);   // rows < 2^31: 32-bit arithmetic
    return (int)(((uint32_t)M.rows + per - 1u) / per);
}

// ---------------------------------------------------------------------------
// forward products: u = A x - b (optional b), t = L x
// workgroups [0, nbA) take rows of A, the rest rows of L
// ---------------------------------------------------------------------------

template <typename T, bool Masked = false>
__device__ __forceinline__ void forward_body(const Csr& A, const Csr& L, int nbA, int nb_all,
                                             const double* __restrict__ x,
                                             const double* __restrict__ b,
                                             double* __restrict__ u, double* __restrict__ t,
                                             double* upart, double* tpart, int blk_all,
                                             double* red) {
    const bool isA = blk_all < nbA;
    const Csr& M = isA ? A : L;
    const int blk = isA ? xcd_order(blk_all, nbA) : xcd_order(blk_all - nbA, nb_all - nbA);
    double* out = isA ? u : t;
    const double* sub = isA ? b : nullptr;
    double* part = isA ? upart : tpart;
    double sq = 0.0;
    SGKS_LANES_SWITCH(M.lanes, {
        const int64_t row = (int64_t)blk * (kBlock / V) + threadIdx.x / V;
        const int g = threadIdx.x % V;
        if (row < M.rows) {
            double v = row_dot<V, T, Masked>(M, x, row, g);
            if (sub) v -= sub[row];
            if (g == 0) {
                out[row] = v;
                sq = v * v;
            }
        }
    })
    if (part) {
        const double tot = block_sum(sq, red);
        if (threadIdx.x == 0) part[blk] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_forward(Csr A, Csr L, int nbA,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ u, double* __restrict__ t,
                                                   double* upart, double* tpart) {
    __shared__ double red[kWaves];
    forward_body<T>(A, L, nbA, (int)gridDim.x, x, b, u, t, upart, tpart, (int)blockIdx.x, red);
}

// Iteration form: newcol = 0: u = A x - b, t = L x from the state's x;
// newcol = 1: u = A w, t = L w for the basis column d (skipped on a set status),
// and workgroup 0 also sums ||w||^2 into scal[14].
template <typename T, bool Masked>
__global__ __launch_bounds__(kBlock) void kb_forward(const State* __restrict__ SS, BTab tab,
                                                    int newcol) {
    __shared__ double red[kWaves];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (newcol && *S.status != 0) return;
    const double* x = newcol ? S.W + (int64_t)(*S.d) * S.n : S.x;
    if (newcol && sl.blk == 0 && threadIdx.x == 0) S.scal[15] = (double)(*S.d);   // H W column
    forward_body<T, Masked>(S.A, S.L, rows_blocks_of(S.A), sl.nblk, x, newcol ? nullptr : S.b, S.u,
                            S.t, nullptr, nullptr, sl.blk, red);
    if (newcol && sl.blk == 0) {
        // ||r||^2 of the new (unnormalised) column from the adjoint's partial sums,
        // for the column scale of the append
        const double t = block_sum(thread_strided_sum(S.norm_part, S.n_norm_part, kBlock), red);
        if (threadIdx.x == 0) S.scal[14] = t;
    }
}

// ---------------------------------------------------------------------------
// adjoint products: r = A^T u + mu L^T t written to dst, with per-workgroup
// partial sums of r^2 (grid-stride over the n rows)
// ---------------------------------------------------------------------------

template <typename T, int NT = kBlock, bool Masked = false>
__device__ __forceinline__ void adjoint_body(const Csr& At, const Csr& Lt, int withL, double mu,
                                             const double* __restrict__ u,
                                             const double* __restrict__ t,
                                             double* __restrict__ dst, int64_t n, double* part,
                                             int blk, int nblk, double* red) {
    double sq = 0.0;
    const int lb = xcd_order(blk, nblk);
    SGKS_LANES_SWITCH(At.lanes, {
        // workgroup lb takes a contiguous range of row groups of NT / V rows
        constexpr int rpg = NT / V;
        const int64_t ng = (n + rpg - 1) / rpg;
        const int64_t g0 = ng * lb / nblk, g1 = ng * (lb + 1) / nblk;
        const int g = threadIdx.x % V;
        for (int64_t grp = g0; grp < g1; ++grp) {
            const int64_t row = grp * rpg + threadIdx.x / V;
            if (row < n) {
                double v = row_dot<V, T, Masked>(At, u, row, g);
                if (withL) v += mu * row_dot<V, T, Masked>(Lt, t, row, g);
                if (g == 0) {
                    dst[row] = v;
                    sq += v * v;
                }
            }
        }
    })
    if (part) {
        const double tot = block_sum(sq, red);
        if (threadIdx.x == 0) part[lb] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint(Csr At, Csr Lt, int withL, double mu,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ t,
                                                   double* __restrict__ dst, int64_t n,
                                                   double* part) {
    __shared__ double red[kWaves];
    adjoint_body<T>(At, Lt, withL, mu, u, t, dst, n, part, (int)blockIdx.x, (int)gridDim.x, red);
}

// Iteration form, from (u, t):
//   dst = kDstBasis: the new basis column d (skipped on a set status)
//   dst = kDstRefine: the refinement gradient
//   dst = kDstHW: column d of H W = (A^T A + mu L^T L) W from (u, t) = (A w, L w)
//                 of the new column (skipped on a set status)
constexpr int kDstBasis = 0, kDstRefine = 1, kDstHW = 2;

template <typename T, bool Masked>
__global__ __launch_bounds__(kBlock) void kb_adjoint(const State* __restrict__ SS, BTab tab,
                                                    int dst_kind) {
    __shared__ double red[kWaves];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (dst_kind != kDstRefine && *S.status != 0) return;
    // the H W column is the one the new-column SpMV recorded: beside the append
    // chain on another stream, the append may advance d while this grid runs
    double* dst = dst_kind == kDstRefine ? S.rtmp
                  : dst_kind == kDstHW   ? S.HW + (int64_t)S.scal[15] * S.n
                                         : S.W + (int64_t)(*S.d) * S.n;
    // the H W column's norm is not needed: no partial sums
    adjoint_body<T, kBlock, Masked>(S.At, S.Lt, 1, S.mu, S.u, S.t, dst, S.n,
                                    dst_kind == kDstHW ? nullptr : S.norm_part, sl.blk, sl.nblk,
                                    red);
}

// ---------------------------------------------------------------------------
// gradient from the maintained H W (H = A^T A + mu L^T L):
//   r = A^T (A x - b) + mu L^T L x = sum_j HW[:, j] cs[j] y[j] - W[:, 0],
// x = W y, W[:, 0] = A^T b (stored unnormalised).  Written to the new basis
// column d (skipped on a set status) or, to_rtmp, to the refinement gradient;
// per-workgroup partial sums of r^2 into norm_part.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void kb_gradient(const State* __restrict__ SS, BTab tab,
                                                     int to_rtmp) {
    __shared__ double yt[kMaxD];
    __shared__ double red[kWaves];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (!to_rtmp && *S.status != 0) return;
    const int d = *S.d;
    const int64_t n = S.n;
    double* __restrict__ dst = to_rtmp ? S.rtmp : S.W + (int64_t)d * n;
    const double* __restrict__ HW = S.HW;
    const double* __restrict__ g0 = S.W;
    for (int j = threadIdx.x; j < d; j += kBlock) yt[j] = S.cs[j] * S.y[j];
    __syncthreads();
    double sq = 0.0;
    for (int64_t i = (int64_t)sl.blk * kBlock + threadIdx.x; i < n; i += (int64_t)sl.nblk * kBlock) {
        const double* h = HW + i;
        double acc = 0.0;
        int j = 0;
        for (; j + 8 <= d; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = h[(int64_t)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u] * yt[j + u];
        }
        for (; j < d; ++j) acc += h[(int64_t)j * n] * yt[j];
        const double r = acc - g0[i];
        dst[i] = r;
        sq += r * r;
    }
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) S.norm_part[sl.blk] = tot;
}

// ---------------------------------------------------------------------------
// sparse-sign sketch of two vectors: bins_A += S_A zA (m entries, stream 0),
// bins_L += S_L zL (p entries, stream 1).  Workgroups [0, nbA) take zA.  Each
// wave walks 64-entry tiles: a coalesced load, the pattern of every entry
// regenerated from its hash, and zeta LDS atomic adds into the wave's private
// copy of the s bins.  Each workgroup writes its raw bins (no 1/sqrt(zeta), no
// column scale); partial bins are merged in fixed orders downstream.
// ---------------------------------------------------------------------------

// the zeta pattern entries of row i (see State::patA)
template <int Z>
__device__ __forceinline__ void load_pattern(const int16_t* __restrict__ pat, int64_t i,
                                             int* bin, double* sg) {
    uint32_t w[Z / 2];
    const uint32_t* p = (const uint32_t*)(pat + i * Z);
    if constexpr (Z == 2) {
        w[0] = p[0];
    } else if constexpr (Z == 4) {
        const uint2 v = *(const uint2*)p;
        w[0] = v.x; w[1] = v.y;
    } else {
#pragma unroll
        for (int k = 0; k < Z / 8; ++k) {
            const uint4 v = ((const uint4*)p)[k];
            w[4 * k] = v.x; w[4 * k + 1] = v.y; w[4 * k + 2] = v.z; w[4 * k + 3] = v.w;
        }
    }
#pragma unroll
    for (int q = 0; q < Z; ++q) {
        const int e = (int)(int16_t)((q & 1) ? (w[q / 2] >> 16) : (w[q / 2] & 0xffffu));
        bin[q] = e > 0 ? e - 1 : (e < 0 ? -e - 1 : 0);
        sg[q] = e > 0 ? 1.0 : (e < 0 ? -1.0 : 0.0);
    }
}

template <int Z>
__global__ __launch_bounds__(kBlock) void k_make_pattern(int16_t* __restrict__ pat, int64_t rows,
                                                        int s, uint64_t seed, int stream) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * kBlock) {
        int bin[Z];
        double sg[Z];
        sketch_column<Z>(seed, stream, i, s, bin, sg);
#pragma unroll
        for (int q = 0; q < Z; ++q)
            pat[i * Z + q] = (int16_t)(sg[q] > 0.0 ? bin[q] + 1 : (sg[q] < 0.0 ? -(bin[q] + 1) : 0));
    }
}

template <int Z>
__device__ __forceinline__ void scatter_body(const double* __restrict__ zA, int64_t m,
                                             const double* __restrict__ zL, int64_t p, int nbA,
                                             int nbL, int s, uint64_t seed, int identity,
                                             const int16_t* patA, const int16_t* patL,
                                             double* partA, double* partL, int blk_all,
                                             double* sm, int lds_doubles) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // sketch rows in ranges of at most kScatterRange (one LDS copy each): workgroup
    // blk_all of the problem takes range blk_all / (nbA + nbL) of its tiles' bins
    const int R = (s + kScatterRange - 1) / kScatterRange;
    const int len = (s + R - 1) / R;
    const int rg = blk_all / (nbA + nbL);
    blk_all -= rg * (nbA + nbL);
    const int r0 = rg * len, r1 = min(s, r0 + len);
    // copies of the range's bins in LDS: one per wave while they fit, else shared
    const int copies = max(1, min(kSketchWaves, lds_doubles / len));
    for (int i = threadIdx.x; i < copies * len; i += kSketchBlock) sm[i] = 0.0;
    __syncthreads();
    double* bins = sm + (wave % copies) * len - r0;   // indexed by the sketch row
    const bool isA = blk_all < nbA;
    const double* __restrict__ z = isA ? zA : zL;
    const int16_t* pat = isA ? patA : patL;
    const int64_t rows = isA ? m : p;
    const int blk = isA ? blk_all : blk_all - nbA;
    const int nblk = isA ? nbA : nbL;
    const int stream = isA ? 0 : 1;
    const int64_t ntiles = (rows + 63) / 64;
    const int64_t tstride = (int64_t)nblk * kSketchWaves;
    if (pat && !identity) {
        // cached pattern: the loads of four tiles are issued before their atomics
        constexpr int TB = 4;
        for (int64_t t0 = (int64_t)blk * kSketchWaves + wave; t0 < ntiles; t0 += TB * tstride) {
            double v[TB];
            int bin[TB][Z];
            double sg[TB][Z];
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                const int64_t i = min((t0 + u * tstride) * 64 + lane, rows - 1);
                v[u] = z[i];
                load_pattern<Z>(pat, i, bin[u], sg[u]);
            }
#pragma unroll
            for (int u = 0; u < TB; ++u) {
                if ((t0 + u * tstride) * 64 + lane < rows) {
#pragma unroll
                    for (int q = 0; q < Z; ++q)
                        if (R == 1 || (bin[u][q] >= r0 && bin[u][q] < r1))
                            atomicAdd(&bins[bin[u][q]], sg[u][q] * v[u]);
                }
            }
        }
    } else {
        for (int64_t tile = (int64_t)blk * kSketchWaves + wave; tile < ntiles; tile += tstride) {
            const int64_t i = tile * 64 + lane;
            if (i < rows) {
                const double v = z[i];
                if (identity) {
                    if (i >= r0 && i < r1) atomicAdd(&bins[i], v);
                } else {
                    int bin[Z];
                    double sg[Z];
                    sketch_column<Z>(seed, stream, i, s, bin, sg);
#pragma unroll
                    for (int q = 0; q < Z; ++q)
                        if (bin[q] >= r0 && bin[q] < r1) atomicAdd(&bins[bin[q]], sg[q] * v);
                }
            }
        }
    }
    __syncthreads();
    double* out = (isA ? partA : partL) + (int64_t)blk * s + r0;
    for (int j = threadIdx.x; j < r1 - r0; j += kSketchBlock) {
        double a = 0.0;
        for (int w = 0; w < copies; ++w) a += sm[w * len + j];
        out[j] = a;
    }
}

template <int Z>
__global__ __launch_bounds__(kSketchBlock) void k_scatter(const double* __restrict__ zA,
                                                         int64_t m,
                                                         const double* __restrict__ zL,
                                                         int64_t p, int nbA, int nbL, int s,
                                                         uint64_t seed, int identity,
                                                         const int16_t* patA,
                                                         const int16_t* patL, double* partA,
                                                         double* partL, int lds_doubles) {
    extern __shared__ double sm[];
    scatter_body<Z>(zA, m, zL, p, nbA, nbL, s, seed, identity, patA, patL, partA, partL,
                    (int)blockIdx.x, sm, lds_doubles);
}

// Iteration form: the sketch of the new column's images (u, t); skipped on a
// set status.
template <int Z>
__global__ __launch_bounds__(kSketchBlock) void kb_scatter(const State* __restrict__ SS,
                                                          BTab tab, int lds_doubles) {
    extern __shared__ double sm[];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (*S.status != 0) return;
    scatter_body<Z>(S.u, S.m, S.t, S.p, S.nbA, S.nbL, S.s, S.seed, S.sketch_mode, S.patA, S.patL,
                    S.binA, S.binL, sl.blk, sm, lds_doubles);
}

// ---------------------------------------------------------------------------
// SRTT sketch (eq:sketching_trig): S = sqrt(h/s) D F E with F the orthonormal
// DCT-II of length h, E Rademacher signs, D s selected frequencies, so
//   (S z)_j = sqrt(h/s) c_k sum_i E_i z_i cos(pi k (2 i + 1) / (2 h)),  k = rows[j],
// c_0 = sqrt(1/h), c_k = sqrt(2/h).  Only the s selected outputs are formed.
// With i = 256 Q + r (chunk Q, row r) and theta = pi k / (2 h) the angle is
// phi_Q + psi_r, phi_Q = theta (512 Q + 1), psi_r = 2 theta r, so
//   sum_i y_i cos(.) = sum_Q [cos phi_Q (C Y)_Q - sin phi_Q (S Y)_Q],  y = E z,
// with C[k][r] = cos(psi_r), S[k][r] = sin(psi_r) the same s x 256 matrices for
// every chunk and Y the 256 x (chunks) matrix of y: two dense FP64 products, on
// MFMA (16 x 16 x 4 FP64 tiles).  A workgroup takes 16 frequencies and a range
// of chunk blocks (16 chunks, 4096 rows each): its four waves split the 256
// rows of the contraction, their tiles are added in LDS, and each (frequency,
// chunk) pair is rotated by phi_Q (exact sincospi from the argument reduced in
// integers) and summed over the chunks.  The range sums are partial bins added
// by the append like the scatter's.
// ---------------------------------------------------------------------------

typedef double sgks_double4 __attribute__((ext_vector_type(4)));

constexpr int kSrttB = 256;                   // rows of a chunk (the contraction)
constexpr int kSrttNB = 16;                   // chunks of a block (the MFMA N)
constexpr int kSrttBlockRows = kSrttB * kSrttNB;
constexpr int kSrttFT = 16;                   // frequencies of a workgroup (the MFMA M)
constexpr int kSrttYs = 17;                   // LDS row stride of the staged block (banks)

// C and S tables of one side: T[j * 256 + r] = cos(pi k_j r / h), then at
// offset spad * 256 the sines (rows j >= s are zero)
__global__ __launch_bounds__(kBlock) void k_srtt_tables(const int32_t* __restrict__ rows,
                                                       int64_t h, int s, int spad,
                                                       double* __restrict__ T) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= (int64_t)spad * kSrttB) return;
    const int j = (int)(e / kSrttB), r = (int)(e % kSrttB);
    double sn = 0.0, cs = 0.0;
    if (j < s) {
        const int64_t k = rows[j];
        const int64_t q = (k * r) % (2 * h);   // angle pi k r / h, reduced mod 2 pi
        sincospi((double)q / (double)h, &sn, &cs);
    }
    T[e] = cs;
    T[(int64_t)spad * kSrttB + e] = sn;
}

__device__ __forceinline__ void srtt_body(const double* __restrict__ z, int64_t h, int s,
                          const int32_t* __restrict__ rows, const double* __restrict__ T,
                          uint64_t seed, int stream, int ncb, int nr, int ft, int qr,
                          double* __restrict__ part, double* ys, double* red) {
    const uint64_t gam = 0x9E3779B97F4A7C15ull;
    const uint64_t ks = mix64(seed + gam * (uint64_t)(stream + 3));
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int spad = ((s + kSrttFT - 1) / kSrttFT) * kSrttFT;
    // MFMA operands: lane holds A[i = lane % 16][kk = lane / 16] of each 16 x 4
    // step; wave w takes rows [64 w, 64 w + 64) of the contraction (read from L2
    // for every block: held across the loop they would halve the occupancy)
    const double* Tc = T + (int64_t)(ft * kSrttFT + (lane & 15)) * kSrttB + 64 * w + (lane >> 4);
    const double* Tsn = Tc + (int64_t)spad * kSrttB;
    // combine role: thread (frequency fi, chunk qq of the block)
    const int fi = tid >> 4, qq = tid & 15;
    const int j = ft * kSrttFT + fi;
    const bool active = j < s;
    const int64_t kf = active ? rows[j] : 0;
    double accj = 0.0;
    const int cb0 = (int)((int64_t)ncb * qr / nr), cb1 = (int)((int64_t)ncb * (qr + 1) / nr);
    for (int cb = cb0; cb < cb1; ++cb) {
        __syncthreads();   // the previous block's ys and red were read by every thread
        const int64_t i0 = (int64_t)cb * kSrttBlockRows;
        {
            // the block's 16 entries of this thread: every load in flight first
            constexpr int U = kSrttBlockRows / kBlock;
            double zv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) zv[u] = z[min(i0 + tid + u * kBlock, h - 1)];
#pragma unroll 2
            for (int u = 0; u < U; ++u) {
                const int e = tid + u * kBlock;
                const int64_t gi = i0 + e;
                const double sg = (mix64(ks + gam * (uint64_t)(gi + 1)) & 1ull) ? -1.0 : 1.0;
                ys[(e & (kSrttB - 1)) * kSrttYs + (e >> 8)] = gi < h ? sg * zv[u] : 0.0;   // [row][chunk]
            }
        }
        __syncthreads();
        double ac[16], as_[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            ac[q] = Tc[4 * q];
            as_[q] = Tsn[4 * q];
        }
        sgks_double4 dc = {0.0, 0.0, 0.0, 0.0}, ds = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            // B[kk = lane / 16][chunk = lane % 16] of step q
            const double b = ys[(64 * w + 4 * q + (lane >> 4)) * kSrttYs + (lane & 15)];
            dc = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[q], b, dc, 0, 0, 0);
            ds = __builtin_amdgcn_mfma_f64_16x16x4f64(as_[q], b, ds, 0, 0, 0);
        }
        // element t of lane l holds D[i = 4 t + l / 16][chunk = l % 16] (measured
        // on gfx950 with a probe of known operands)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = 4 * t + (lane >> 4);
            red[((w * 2 + 0) * kSrttFT + i) * kSrttNB + (lane & 15)] = dc[t];
            red[((w * 2 + 1) * kSrttFT + i) * kSrttNB + (lane & 15)] = ds[t];
        }
        __syncthreads();
        double pc = 0.0, ps = 0.0;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            pc += red[((ww * 2 + 0) * kSrttFT + fi) * kSrttNB + qq];
            ps += red[((ww * 2 + 1) * kSrttFT + fi) * kSrttNB + qq];
        }
        const int64_t Q = (int64_t)cb * kSrttNB + qq;
        double val = 0.0;
        if (active && Q * kSrttB < h) {
            // phi = pi k (512 Q + 1) / (2 h), reduced mod 2 pi in integers
            const int64_t a = (kf * (2 * kSrttB * Q + 1)) % (4 * h);
            double sn, cs;
            sincospi((double)a / (double)(2 * h), &sn, &cs);
            val = cs * pc - sn * ps;
        }
        val += __shfl_xor(val, 8);
        val += __shfl_xor(val, 4);
        val += __shfl_xor(val, 2);
        val += __shfl_xor(val, 1);
        accj += val;
    }
    if (active && qq == 0) {
        const double ck = kf == 0 ? sqrt(1.0 / (double)h) : sqrt(2.0 / (double)h);
        part[(int64_t)qr * s + j] = sqrt((double)h / (double)s) * ck * accj;
    }
}

struct SrttLds {
    double ys[kSrttB * kSrttYs];
    double red[4 * 2 * kSrttFT * kSrttNB];
};

// workgroups [0, nbA nft) sketch zA (S_A, m rows), the rest zL (S_L, p rows);
// within a side, workgroup b takes range b / nft and frequency tile b % nft
__device__ __forceinline__ void srtt_pair(const State& S, const double* zA, const double* zL,
                                          int nbL, int blk, SrttLds& sh) {
    const int nft = (S.s + kSrttFT - 1) / kSrttFT;
    if (blk >= (S.nbA + nbL) * nft) return;
    const bool a = blk < S.nbA * nft;   // one call site: the body is inlined once
    const int b = a ? blk : blk - S.nbA * nft;
    srtt_body(a ? zA : zL, a ? S.m : S.p, S.s, a ? S.rowsA : S.rowsL, a ? S.srtTA : S.srtTL,
              S.seed, a ? 0 : 1, a ? S.srA : S.srL, a ? S.nbA : S.nbL, b % nft, b / nft,
              a ? S.binA : S.binL, sh.ys, sh.red);
}

__global__ __launch_bounds__(kBlock) void k_srtt(const State S, const double* zA,
                                                const double* zL, int nbL) {
    __shared__ SrttLds sh;
    srtt_pair(S, zA, zL, nbL, blockIdx.x, sh);
}

// Iteration form: the SRTT sketches of the new column's images (u, t); skipped on
// a set status.
__global__ __launch_bounds__(kBlock) void kb_srtt(const State* __restrict__ SS, BTab tab) {
    __shared__ SrttLds sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (*S.status != 0) return;
    srtt_pair(S, S.u, S.t, S.nbL, sl.blk, sh);
}

// S^T v on the matrix cores.  With i = 256 Q + r the angle of entry (k_j, i) splits
// as phi_{Q,j} + psi_{r,j}, phi = pi k_j (512 Q + 1) / (2 h), psi = pi k_j r / h, so
//   (S^T v)_i = sqrt(h/s) E_i sum_j [cos psi_{r,j} alpha_{Q,j} - sin psi_{r,j} beta_{Q,j}],
//   alpha = c_j v_j cos phi_{Q,j}, beta = c_j v_j sin phi_{Q,j}:
// a (256 x 2s) by (2s x h/256) product whose left factor is the side's cosine and
// sine tables (built at create).  A wave takes 64 rows r (four 16-row tiles) and
// 32 blocks Q (two 16-wide tiles); the right operand is formed on the fly, one
// sincospi per lane and tile for each step of 4 frequencies; the sine part goes
// into the same accumulator with its sign folded into the operand.
constexpr int kSrttTQ = 2;   // 16-wide Q tiles per wave of the transpose

__global__ __launch_bounds__(kBlock) void k_srtt_transpose_mfma(
    const double* __restrict__ vA, const double* __restrict__ vL, int s, int spad, int64_t m,
    int64_t p, const int32_t* __restrict__ rowsA, const int32_t* __restrict__ rowsL,
    const double* __restrict__ TA, const double* __restrict__ TL, uint64_t seed, int nbA,
    double* __restrict__ outA, double* __restrict__ outL) {
    const bool isA = (int)blockIdx.x < nbA;
    const int b = isA ? blockIdx.x : blockIdx.x - nbA;
    const int64_t h = isA ? m : p;
    const double* __restrict__ v = isA ? vA : vL;
    const int32_t* __restrict__ rows = isA ? rowsA : rowsL;
    const double* __restrict__ T = isA ? TA : TL;
    double* __restrict__ out = isA ? outA : outL;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nQ = (h + kSrttB - 1) / kSrttB;
    const int64_t Q0 = (int64_t)b * 16 * kSrttTQ;
    // A operand: lane l holds A[r = l % 16][kk = l / 16] = T[j0 + l / 16][r0 + l % 16]
    const double* Tc = T + (int64_t)(lane >> 4) * kSrttB + 64 * w + (lane & 15);
    const double* Tsn = Tc + (int64_t)spad * kSrttB;
    const double c0 = sqrt(1.0 / (double)h), c1 = sqrt(2.0 / (double)h);
    sgks_double4 acc[kSrttTQ][4];
#pragma unroll
    for (int qt = 0; qt < kSrttTQ; ++qt)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[qt][rt] = sgks_double4{0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < spad; j0 += 4) {
        // B operand: lane l holds B[kk = l / 16][Q = l % 16]
        const int j = j0 + (lane >> 4);
        const bool on = j < s;
        const double vj = on ? v[j] : 0.0;
        const int64_t kj = on ? rows[j] : 0;
        const double cj = (kj == 0 ? c0 : c1) * vj;
        double bc[kSrttTQ], bs[kSrttTQ];
#pragma unroll
        for (int qt = 0; qt < kSrttTQ; ++qt) {
            const int64_t Q = Q0 + 16 * qt + (lane & 15);
            const int64_t a = (kj * (2 * kSrttB * Q + 1)) % (4 * h);   // phi mod 2 pi
            double sn, cs;
            sincospi((double)a / (double)(2 * h), &sn, &cs);
            bc[qt] = cj * cs;
            bs[qt] = -cj * sn;
        }
        double tc[4], ts[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            tc[rt] = Tc[(int64_t)j0 * kSrttB + 16 * rt];
            ts[rt] = Tsn[(int64_t)j0 * kSrttB + 16 * rt];
        }
#pragma unroll
        for (int qt = 0; qt < kSrttTQ; ++qt)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                acc[qt][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(tc[rt], bc[qt], acc[qt][rt], 0, 0, 0);
                acc[qt][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ts[rt], bs[qt], acc[qt][rt], 0, 0, 0);
            }
    }
    // element t of lane l holds D[r = 4 t + l / 16][Q = l % 16]
    const uint64_t gam = 0x9E3779B97F4A7C15ull;
    const uint64_t ks = mix64(seed + gam * (uint64_t)((isA ? 0 : 1) + 3));
    const double sc = sqrt((double)h / (double)s);
#pragma unroll
    for (int qt = 0; qt < kSrttTQ; ++qt) {
        const int64_t Q = Q0 + 16 * qt + (lane & 15);
        if (Q >= nQ) continue;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = Q * kSrttB + 64 * w + 16 * rt + 4 * t + (lane >> 4);
                if (i < h) {
                    const double sg = (mix64(ks + gam * (uint64_t)(i + 1)) & 1ull) ? -1.0 : 1.0;
                    out[i] = sc * sg * acc[qt][rt][t];
                }
            }
    }
}

// ---------------------------------------------------------------------------
// dense basis products
// ---------------------------------------------------------------------------

// out[perm[i]] = [base[i] -] sum_j W[i, j] * cs[j] * coef[j], j < d (grid-stride
// rows; perm null: the identity; cs null: no column scale)
__device__ __forceinline__ void gemv_body(const double* __restrict__ W,
                                          const double* __restrict__ cs,
                                          const double* __restrict__ coef, int d, int64_t n,
                                          const double* __restrict__ base,
                                          double* __restrict__ out, int blk, int nblk,
                                          double* yt, const int32_t* __restrict__ perm = nullptr) {
    for (int j = threadIdx.x; j < d; j += kBlock) yt[j] = cs ? cs[j] * coef[j] : coef[j];
    __syncthreads();
    for (int64_t i = (int64_t)blk * kBlock + threadIdx.x; i < n; i += (int64_t)nblk * kBlock) {
        const double* w = W + i;
        double acc = 0.0;
        int j = 0;
        for (; j + 8 <= d; j += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = w[(int64_t)(j + u) * n];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u] * yt[j + u];
        }
        for (; j < d; ++j) acc += w[(int64_t)j * n] * yt[j];
        out[perm ? (int64_t)perm[i] : i] = base ? base[i] - acc : acc;
    }
}

__global__ __launch_bounds__(kBlock) void k_gemv(const double* __restrict__ W,
                                                const double* __restrict__ cs,
                                                const double* __restrict__ coef, const int* dptr,
                                                int ncols_fixed, int64_t n,
                                                const double* __restrict__ base,
                                                double* __restrict__ out,
                                                const int32_t* __restrict__ perm) {
    __shared__ double yt[kMaxD];
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    gemv_body(W, cs, coef, d, n, base, out, (int)blockIdx.x, (int)gridDim.x, yt, perm);
}

// Iteration form: x = W y on the current d columns.
__global__ __launch_bounds__(kBlock) void kb_gemv(const State* __restrict__ SS, BTab tab) {
    __shared__ double yt[kMaxD];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    gemv_body(S.W, S.cs, S.y, *S.d, S.n, nullptr, S.x, sl.blk, sl.nblk, yt);
}

// part[blk * ld + j] = cs[j] * sum_{i in the workgroup's rows} W[i, j] v[i], j < d
// (cs null: no column scale)
__device__ __forceinline__ void gemvt_body(const double* __restrict__ W,
                                           const double* __restrict__ cs,
                                           const double* __restrict__ v, int d, int64_t n,
                                           int rows_per_block, double* __restrict__ part, int ld,
                                           int blk, double* vs) {
    const int64_t r0 = (int64_t)blk * rows_per_block;
    const int nr = (int)min((int64_t)rows_per_block, n - r0);
    for (int i = threadIdx.x; i < nr; i += kBlock) vs[i] = v[r0 + i];
    __syncthreads();
    // each wave takes eight columns at a time; a lane loads its rows (lane + 64 t)
    // of all eight, four rows per column at a time, every load in flight
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nt = (nr + 63) / 64;
    for (int j0 = wave * 8; j0 < d; j0 += kWaves * 8) {
        const double* wc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) wc[c] = W + (int64_t)min(j0 + c, d - 1) * n + r0;
        double acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = 0.0;
        for (int t0 = 0; t0 < nt; t0 += 4) {
            double w[8][4], vv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = min(lane + 64 * (t0 + t), nr - 1);   // clamped; masked below
                vv[t] = (t0 + t < nt && lane + 64 * (t0 + t) < nr) ? vs[i] : 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) w[c][t] = wc[c][i];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] += w[c][t] * vv[t];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double a = wave_sum(acc[c]);
            if (lane == 0 && j0 + c < d)
                part[(int64_t)blk * ld + j0 + c] = cs ? a * cs[j0 + c] : a;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_gemvt(const double* __restrict__ W,
                                                 const double* __restrict__ cs,
                                                 const double* __restrict__ v, const int* dptr,
                                                 int ncols_fixed, int64_t n, int rows_per_block,
                                                 double* __restrict__ part, int ld) {
    extern __shared__ double vs[];
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    gemvt_body(W, cs, v, d, n, rows_per_block, part, ld, (int)blockIdx.x, vs);
}

// Iteration form: partials of W^T rtmp (refinement gradient).
__global__ __launch_bounds__(kBlock) void kb_gemvt(const State* __restrict__ SS, BTab tab) {
    extern __shared__ double vs[];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (*S.status != 0) return;
    gemvt_body(S.W, S.cs, S.rtmp, *S.d, S.n, S.gt_rows, S.gpart, S.dmax, sl.blk, vs);
}

// Partials of the newest column c = d - 1 of the projected normal matrix
// M = W^T H W (raw columns: W[:, i]^T H W[:, c], i <= c, H W[:, c] the kept
// column) and of W[:, c]^T W[:, 0] (W[:, 0] = A^T b), into gpart with leading
// dimension dmax + 1 (slot c + 1 for the second).  The new column's images
// H W[:, c] are complete: the caller's stream has joined the stream that
// computed them.
__global__ __launch_bounds__(kBlock) void kb_mcol(const State* __restrict__ SS, BTab tab) {
    extern __shared__ double vs[];
    __shared__ double red[kWaves];
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (*S.status != 0) return;
    const int c = *S.d - 1;
    const int ld = S.dmax + 1;
    gemvt_body(S.W, nullptr, S.HW + (int64_t)c * S.n, c + 1, S.n, S.gt_rows, S.gpart, ld, sl.blk,
               vs);
    const int64_t r0 = (int64_t)sl.blk * S.gt_rows;
    const int nr = (int)min((int64_t)S.gt_rows, S.n - r0);
    const double* wc = S.W + (int64_t)c * S.n + r0;
    double a = 0.0;
    for (int i = threadIdx.x; i < nr; i += kBlock) a += wc[i] * S.W[r0 + i];
    a = block_sum(a, red);
    if (threadIdx.x == 0) S.gpart[(int64_t)sl.blk * ld + c + 1] = a;
}

// out[j] = sum_b part[b * ld + j], j < d
__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double* __restrict__ part, int nb,
                                                       int ld, const int* dptr, int ncols_fixed,
                                                       double* __restrict__ out) {
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    for (int j = threadIdx.x; j < d; j += kBlock) out[j] = strided_sum(part + j, ld, nb);
}

// cs[col] = 1 / ||v|| from the norm partials; optionally scal[0] = ||v||.
__global__ __launch_bounds__(kBlock) void k_set_scale(const double* part, int nb, double* cs,
                                                     int col, int store_r0, double* scal,
                                                     int* status) {
    __shared__ double red[kWaves];
    const double t = block_sum(thread_strided_sum(part, nb, kBlock), red);
    if (threadIdx.x == 0) {
        const double nr = sqrt(t);
        scal[16 + col] = nr;
        if (store_r0) scal[0] = nr;
        if (!(nr < INFINITY)) *status = kStatusNonfinite;
        cs[col] = nr > 0.0 ? 1.0 / nr : 0.0;
    }
}

// c_b = S_A b from the raw bins, and ||c_b||^2 into scal[1]
__global__ __launch_bounds__(kBlock) void k_cb(const double* __restrict__ bins, int nb, int s,
                                              double scale, double* cb, double* scal) {
    __shared__ double red[kWaves];
    double sq = 0.0;
    for (int i = threadIdx.x; i < s; i += kBlock) {
        double a = strided_sum(bins + i, s, nb);
        a *= scale;
        cb[i] = a;
        sq += a * a;
    }
    const double t = block_sum(sq, red);
    if (threadIdx.x == 0) scal[1] = t;
}

// ---------------------------------------------------------------------------
// cooperative append: reduce the sketched column, CGS append to (Q_A, R_A)
// and (Q_L, R_L), append d_A, append to the stacked factor (U, G, h),
// update G^{-1} and y = G^{-1} h.
// ---------------------------------------------------------------------------

// The append runs as a chain of small kernels, each with G <= 256 workgroups.
// Workgroup g owns sketch rows [lo, hi) of Q_A and Q_L and rows [ulo, uhi)
// of both halves of U.  Each kernel finishes the previous projection with the
// coefficients reduced (in workgroup order) from the previous kernel's
// partial vectors and writes its own partial vector into one region of
// S.coop; slot t of workgroup g lives at region[t * G + g] so that a reduction
// reads G consecutive values in one batch.
//   region r < P          : Q coefficients of projection pass r (slots [0, d) for
//                           Q_A, [dmax, dmax + d) for Q_L) and, for r = 0, ||a||^2, ||l||^2
//   region P              : U coefficients of U pass 0, ||a_perp||^2, ||l_perp||^2, a_perp . S_A b
//   region P + u, 0<u<P   : U coefficients of U pass u
//   region 2P             : gamma^2 and the new h numerator
// (P = S.passes).  Workgroup 0 keeps the running sums p = sum of the Q
// coefficients (S.pacc[0, 2 dmax), the final p in S.pacc[2 dmax, 4 dmax)) and
// gacc = sum of the U coefficients (S.gacc).  No workgroup writes memory that
// another workgroup of the same launch reads; kernel boundaries order the
// phases, and the basis size d advances in the single-workgroup k_yfix.
// Memory traffic is small (the slabs stay in L2); what these kernels pay is
// latency, so every loop issues its loads in batches.

constexpr int kSlots = 8;   // scalar slots after the 2 dmax coefficient slots

struct ApDims {
    int g, G;             // this workgroup, workgroups of the problem
    int d, s, dmax, ld2, nslot;
    int lo, ns;           // sketch-row slab
    int ulo, nu, nua;     // U-row slab (both halves), rows < d active
};

__device__ ApDims ap_dims(const State& S, int g, int G, int d) {
    ApDims D;
    D.g = g;
    D.G = G;
    D.d = d;
    D.s = S.s;
    D.dmax = S.dmax;
    D.ld2 = 2 * S.dmax;
    D.nslot = 2 * S.dmax + kSlots;
    D.lo = (int)((int64_t)S.s * g / G);
    D.ns = (int)((int64_t)S.s * (g + 1) / G) - D.lo;
    D.ulo = (int)((int64_t)S.dmax * g / G);
    D.nu = (int)((int64_t)S.dmax * (g + 1) / G) - D.ulo;
    D.nua = max(0, min(D.ulo + D.nu, d) - D.ulo);
    return D;
}

__device__ __forceinline__ double* ap_region(const State& S, const ApDims& D, int G, int r) {
    return S.coop + (int64_t)r * D.nslot * G;
}

// sum over workgroups of one slot: G consecutive values, one batch of loads
__device__ __forceinline__ double sum_g(const double* __restrict__ slot, int G) {
    double a = 0.0;
    for (int g0 = 0; g0 < G; g0 += 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = slot[min(g0 + u, G - 1)];
#pragma unroll
        for (int u = 0; u < 32; ++u)
            if (g0 + u < G) a += v[u];
    }
    return a;
}

// Column dots over a slab of rows of two column-major matrices (leading
// dimension ld, rows [0, nrows) of each column contiguous):
//   Joint:  pA[j G + g] = sum_i (MA[j ld + i] vA[i] + ML[j ld + i] vL[i])
//   !Joint: pA[j G + g] = sum_i MA[j ld + i] vA[i], pL[j G + g] = sum_i ML[j ld + i] vL[i]
// for j < d.  Thread j owns column j (strided over the workgroup) and loads
// sixteen rows of each side at a time, all in flight; vA, vL are read from
// LDS (one address per wave).  Rows are added in order: fixed sums.
template <bool Joint>
__device__ void slab_dots2(const double* __restrict__ MA, const double* __restrict__ ML,
                           int64_t ld, int nrows, int d, const double* vA, const double* vL,
                           double* pA, double* pL, int g, int G) {
    __syncthreads();   // vA, vL were just written by other threads
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const double* __restrict__ ca = MA + (int64_t)j * ld;
        const double* __restrict__ cl = ML + (int64_t)j * ld;
        double accA = 0.0, accL = 0.0;
        for (int i0 = 0; i0 < nrows; i0 += 16) {
            double wa[16], wl[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = min(i0 + u, nrows - 1);   // clamped: loads stay unconditional
                wa[u] = ca[i];
                wl[u] = cl[i];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (i0 + u < nrows) {
                    accA += wa[u] * vA[i0 + u];
                    if (Joint)
                        accA += wl[u] * vL[i0 + u];
                    else
                        accL += wl[u] * vL[i0 + u];
                }
        }
        pA[(int64_t)j * G + g] = accA;
        if (!Joint) pL[(int64_t)j * G + g] = accL;
    }
}

// outA[i] -= sum_j MA[j ld + i] cA[j] and outL[i] -= sum_j ML[j ld + i] cL[j]
// for i < nrows (MA, ML global column-major slabs; cA, cL, outA, outL in LDS).
// The two sides take the two halves of the workgroup; within a side, threads
// split the rows and contiguous chunks of j, and the chunk sums are added in
// chunk order.  scratch: blockDim.x doubles of LDS.
template <int B = 16>
__device__ void slab_apply2(const double* __restrict__ MA, const double* __restrict__ ML,
                            int64_t ld, int nrows, int d, const double* cA, const double* cL,
                            double* outA, double* outL, double* scratch) {
    const int T = blockDim.x / 2, side = threadIdx.x / T, tid = threadIdx.x % T;
    __syncthreads();   // the coefficients and out were just written by other threads
    if (nrows <= 0 || d <= 0) {
        __syncthreads();
        return;
    }
    const double* __restrict__ M = side ? ML : MA;
    const double* c = side ? cL : cA;
    double* out = side ? outL : outA;
    double* scr = scratch + side * T;
    const int nq = nrows >= T ? 1 : T / nrows;
    for (int r0 = 0; r0 < nrows; r0 += T) {
        const int nr = min(nrows - r0, T);
        const int i = r0 + tid % nr, q = tid / nr;
        if (q < nq) {
            const int j0 = (int)((int64_t)d * q / nq), j1 = (int)((int64_t)d * (q + 1) / nq);
            scr[q * nr + (i - r0)] = strided_dot<B>(M + (int64_t)j0 * ld + i, ld, c + j0, j1 - j0);
        }
        __syncthreads();
        if (tid < nr) {
            double a = 0.0;
            for (int qq = 0; qq < nq; ++qq) a += scr[qq * nr + tid];
            out[r0 + tid] -= a;
        }
        __syncthreads();
    }
}

// Two strided sums, pA[0] + pA[stride] + ... (nA terms) and likewise pL (nL
// terms), each in order, with the loads of both in flight together.
__device__ __forceinline__ void strided_sum_pair(const double* __restrict__ pA, int nA,
                                                 const double* __restrict__ pL, int nL,
                                                 int64_t stride, double& a, double& l) {
    a = 0.0;
    l = 0.0;
    const int n = max(nA, nL);
    for (int k = 0; k < n; k += 16) {
        double va[16], vl[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            va[u] = nA > 0 ? pA[(int64_t)min(k + u, nA - 1) * stride] : 0.0;
            vl[u] = nL > 0 ? pL[(int64_t)min(k + u, nL - 1) * stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (k + u < nA) a += va[u];
            if (k + u < nL) l += vl[u];
        }
    }
}

struct ApShared {
    double red[kAppendThreads / 64];
    double cA[kMaxD];
    double cL[kMaxD];
    double pA[kMaxD];
    double pL[kMaxD];
    double av[kAppendMaxSlab];
    double lv[kAppendMaxSlab];
    double cuA[kMaxD];
    double cuL[kMaxD];
    double scr[kAppendThreads];
    double sc[kSlots];
};

// Q pass 0: column scale (breakdown test), reduce the sketch bins of this
// slab, first projection coefficients.
__global__ __launch_bounds__(kAppendThreads) void k_ap_q0(const State* __restrict__ SS, BTab tab,
                                                     int scale_from_norm) {
    __shared__ ApShared sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    const int G = sl.nblk;
    if (*S.status != 0) return;
    const int d = *S.d;
    const ApDims D = ap_dims(S, sl.blk, G, d);
    const int g = sl.blk, tid = threadIdx.x, T = kAppendThreads;
    double scale;
    if (scale_from_norm) {
        const double nr2 = S.scal[14];
        const double nr = sqrt(nr2);
        if (!(nr2 < INFINITY)) {
            if (g == 0 && tid == 0) *S.status = kStatusNonfinite;
            return;
        }
        if (!(nr > 1e-14 * S.scal[0])) {
            if (g == 0 && tid == 0) *S.status = kStatusBreakdown;
            return;
        }
        scale = 1.0 / nr;
        if (g == 0 && tid == 0) S.cs[d] = scale;
    } else {
        scale = S.cs[d];
    }
    // bins of this slab: thread (row i, chunk q) sums a contiguous range of blocks
    const double bscale = S.sketch_mode == kSketchSparseSign ? scale / sqrt((double)S.zeta) : scale;
    const int nq = D.ns > 0 ? T / D.ns : 1;
    double* scrA = sh.cA;   // free until the coefficients arrive
    double* scrL = sh.cL;
    {
        const int i = D.ns > 0 ? tid % D.ns : 0, q = D.ns > 0 ? tid / D.ns : T;
        if (q < nq) {
            const int a0 = (int)((int64_t)S.nbA * q / nq), a1 = (int)((int64_t)S.nbA * (q + 1) / nq);
            const int l0 = (int)((int64_t)S.nbL * q / nq), l1 = (int)((int64_t)S.nbL * (q + 1) / nq);
            strided_sum_pair(S.binA + (int64_t)a0 * D.s + D.lo + i, a1 - a0,
                             S.binL + (int64_t)l0 * D.s + D.lo + i, l1 - l0, D.s,
                             scrA[q * D.ns + i], scrL[q * D.ns + i]);
        }
    }
    __syncthreads();
    double na2 = 0.0, nl2 = 0.0;
    if (tid < D.ns) {
        double a = 0.0, l = 0.0;
        for (int q = 0; q < nq; ++q) {
            a += scrA[q * D.ns + tid];
            l += scrL[q * D.ns + tid];
        }
        a *= bscale;
        l *= bscale;
        sh.av[tid] = a;
        sh.lv[tid] = l;
        S.wa[D.lo + tid] = a;
        S.wl[D.lo + tid] = l;
        na2 = a * a;
        nl2 = l * l;
    }
    na2 = block_sum(na2, sh.red);
    nl2 = block_sum(nl2, sh.red);
    double* reg = ap_region(S, D, G, 0);
    slab_dots2<false>(S.QA + D.lo, S.QL + D.lo, D.s, D.ns, d, sh.av, sh.lv, reg,
                      reg + (int64_t)S.dmax * G, D.g, G);
    if (tid == 0) {
        reg[(int64_t)(2 * S.dmax) * G + g] = na2;
        reg[(int64_t)(2 * S.dmax + 1) * G + g] = nl2;
    }
}

// reduce the Q coefficients of region r into sh.cA, sh.cL; workgroup 0 adds
// them to the running sum p (S.pacc) -- the first pass initialises it
__device__ void ap_take_q(const State& S, const ApDims& D, int G, int r, ApShared& sh) {
    const double* reg = ap_region(S, D, G, r);
    for (int j = threadIdx.x; j < 2 * D.d; j += blockDim.x) {
        const int slot = j < D.d ? j : S.dmax + (j - D.d);
        const double c = sum_g(reg + (int64_t)slot * G, G);
        if (j < D.d)
            sh.cA[j] = c;
        else
            sh.cL[j - D.d] = c;
        if (D.g == 0) S.pacc[slot] = (r == 0 ? 0.0 : S.pacc[slot]) + c;
    }
}

// Q pass `pass` >= 1: finish the previous projection, next coefficients.
__global__ __launch_bounds__(kAppendThreads) void k_ap_qp(const State* __restrict__ SS, BTab tab,
                                                     int pass) {
    __shared__ ApShared sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    const int G = sl.nblk;
    if (*S.status != 0) return;
    const int d = *S.d;
    const ApDims D = ap_dims(S, sl.blk, G, d);
    const int tid = threadIdx.x;
    for (int i = tid; i < D.ns; i += kAppendThreads) {
        sh.av[i] = S.wa[D.lo + i];
        sh.lv[i] = S.wl[D.lo + i];
    }
    ap_take_q(S, D, G, pass - 1, sh);
    slab_apply2(S.QA + D.lo, S.QL + D.lo, D.s, D.ns, d, sh.cA, sh.cL, sh.av, sh.lv, sh.scr);
    for (int i = tid; i < D.ns; i += kAppendThreads) {
        S.wa[D.lo + i] = sh.av[i];
        S.wl[D.lo + i] = sh.lv[i];
    }
    double* reg = ap_region(S, D, G, pass);
    slab_dots2<false>(S.QA + D.lo, S.QL + D.lo, D.s, D.ns, d, sh.av, sh.lv, reg,
                      reg + (int64_t)S.dmax * G, D.g, G);
}

// Q finish: last projection, norms and d_A numerator, U pass 0 on
// c = [p_A; sqrt(mu) p_L] (rows < d; the new rows are orthogonal to U).
__global__ __launch_bounds__(kAppendThreads) void k_ap_qf(const State* __restrict__ SS,
                                                     BTab tab) {
    __shared__ ApShared sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    const int G = sl.nblk;
    if (*S.status != 0) return;
    const int d = *S.d;
    const ApDims D = ap_dims(S, sl.blk, G, d);
    const int g = sl.blk, tid = threadIdx.x, P = S.passes;
    for (int i = tid; i < D.ns; i += kAppendThreads) {
        sh.av[i] = S.wa[D.lo + i];
        sh.lv[i] = S.wl[D.lo + i];
    }
    // the last coefficients, and p = (earlier passes) + last
    {
        const double* reg = ap_region(S, D, G, P - 1);
        for (int j = tid; j < 2 * d; j += kAppendThreads) {
            const int slot = j < d ? j : S.dmax + (j - d);
            const double c = sum_g(reg + (int64_t)slot * G, G);
            const double p = (P > 1 ? S.pacc[slot] : 0.0) + c;
            if (j < d) {
                sh.cA[j] = c;
                sh.pA[j] = p;
            } else {
                sh.cL[j - d] = c;
                sh.pL[j - d] = p;
            }
            if (g == 0) S.pacc[2 * S.dmax + slot] = p;   // the running sums stay intact
        }
    }
    slab_apply2(S.QA + D.lo, S.QL + D.lo, D.s, D.ns, d, sh.cA, sh.cL, sh.av, sh.lv, sh.scr);
    double ra = 0.0, rl = 0.0, dl = 0.0;
    for (int i = tid; i < D.ns; i += kAppendThreads) {
        S.wa[D.lo + i] = sh.av[i];
        S.wl[D.lo + i] = sh.lv[i];
        ra += sh.av[i] * sh.av[i];
        rl += sh.lv[i] * sh.lv[i];
        dl += sh.av[i] * S.cb[D.lo + i];
    }
    for (int i = tid; i < D.nua; i += kAppendThreads) {
        const int r = D.ulo + i;
        sh.cuA[i] = sh.pA[r];
        sh.cuL[i] = S.sqrt_mu * sh.pL[r];
        S.wu[r] = sh.cuA[i];
        S.wu[S.dmax + r] = sh.cuL[i];
    }
    ra = block_sum(ra, sh.red);
    rl = block_sum(rl, sh.red);
    dl = block_sum(dl, sh.red);
    double* reg = ap_region(S, D, G, P);
    slab_dots2<true>(S.U + D.ulo, S.U + S.dmax + D.ulo, D.ld2, D.nua, d, sh.cuA, sh.cuL, reg,
                     nullptr, D.g, G);
    if (tid == 0) {
        reg[(int64_t)(2 * S.dmax) * G + g] = ra;
        reg[(int64_t)(2 * S.dmax + 1) * G + g] = rl;
        reg[(int64_t)(2 * S.dmax + 2) * G + g] = dl;
    }
}

// U pass `upass` >= 1 (or, with last != 0, the finish: gamma^2 and h numerator)
__global__ __launch_bounds__(kAppendThreads) void k_ap_u(const State* __restrict__ SS, BTab tab,
                                                    int upass, int last) {
    __shared__ ApShared sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    const int G = sl.nblk;
    if (*S.status != 0) return;
    const int d = *S.d;
    const ApDims D = ap_dims(S, sl.blk, G, d);
    const int g = sl.blk, tid = threadIdx.x, P = S.passes;
    for (int i = tid; i < D.nua; i += kAppendThreads) {
        sh.cuA[i] = S.wu[D.ulo + i];
        sh.cuL[i] = S.wu[S.dmax + D.ulo + i];
    }
    {
        const double* reg = ap_region(S, D, G, P + upass - 1);
        for (int j = tid; j < d; j += kAppendThreads) {
            const double c = sum_g(reg + (int64_t)j * G, G);
            sh.cA[j] = c;
            if (g == 0) S.gacc[j] = (upass == 1 ? 0.0 : S.gacc[j]) + c;
        }
    }
    slab_apply2(S.U + D.ulo, S.U + S.dmax + D.ulo, D.ld2, D.nua, d, sh.cA, sh.cA, sh.cuA, sh.cuL,
                sh.scr);
    for (int i = tid; i < D.nua; i += kAppendThreads) {
        S.wu[D.ulo + i] = sh.cuA[i];
        S.wu[S.dmax + D.ulo + i] = sh.cuL[i];
    }
    if (!last) {
        slab_dots2<true>(S.U + D.ulo, S.U + S.dmax + D.ulo, D.ld2, D.nua, d, sh.cuA, sh.cuL,
                         ap_region(S, D, G, P + upass), nullptr, D.g, G);
        return;
    }
    double gam2 = 0.0, hnum = 0.0;
    for (int i = tid; i < D.nua; i += kAppendThreads) {
        gam2 += sh.cuA[i] * sh.cuA[i] + sh.cuL[i] * sh.cuL[i];
        hnum += sh.cuA[i] * S.dA[D.ulo + i];
    }
    gam2 = block_sum(gam2, sh.red);
    hnum = block_sum(hnum, sh.red);
    if (tid == 0) {
        double* reg = ap_region(S, D, G, 2 * P);
        reg[g] = gam2;
        reg[G + g] = hnum;
    }
}

// Commit: new columns of Q_A, Q_L, R_A, R_L, U, G (row-major), entries of
// d_A and h, the new column of G^{-1} (row-major) and y0 = G^{-1} h.
// Breakdown when the new stacked column is dependent.
__global__ __launch_bounds__(kAppendThreads) void k_ap_commit(const State* __restrict__ SS,
                                                         BTab tab) {
    __shared__ ApShared sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    const int G = sl.nblk;
    if (*S.status != 0) return;
    const int d = *S.d;
    const ApDims D = ap_dims(S, sl.blk, G, d);
    const int g = sl.blk, tid = threadIdx.x, P = S.passes, T = kAppendThreads;
    const int dmax = S.dmax;
    if (tid < 7) {
        const double* r0 = ap_region(S, D, G, 0);
        const double* rP = ap_region(S, D, G, P);
        const double* r2P = ap_region(S, D, G, 2 * P);
        const double* src[7] = {r0 + (int64_t)(2 * dmax) * G, r0 + (int64_t)(2 * dmax + 1) * G,
                                rP + (int64_t)(2 * dmax) * G, rP + (int64_t)(2 * dmax + 1) * G,
                                rP + (int64_t)(2 * dmax + 2) * G, r2P, r2P + G};
        sh.sc[tid] = sum_g(src[tid], G);
    }
    for (int j = tid; j < d; j += T) {
        sh.pA[j] = S.pacc[2 * dmax + j];
        sh.pL[j] = S.pacc[3 * dmax + j];
        sh.cA[j] = S.gacc[j];            // sum of the U coefficients (the new column of G)
    }
    __syncthreads();
    const double naTot = sh.sc[0], nlTot = sh.sc[1], ra = sh.sc[2], rl = sh.sc[3], dl = sh.sc[4];
    double gam2 = sh.sc[5], hnum = sh.sc[6];
    double rhoA = sqrt(ra), rhoL = sqrt(rl);
    const bool degA = !(rhoA > 1e-14 * sqrt(naTot));
    const bool degL = !(rhoL > 1e-14 * sqrt(nlTot));
    if (degA) rhoA = 0.0;
    if (degL) rhoL = 0.0;
    const double qsA = degA ? 0.0 : 1.0 / rhoA, qsL = degL ? 0.0 : 1.0 / rhoL;
    const double dAnew = degA ? 0.0 : dl / rhoA;
    // the new rows (rho_A, sqrt(mu) rho_L) are orthogonal to U's old columns
    gam2 += rhoA * rhoA + S.mu * rhoL * rhoL;
    hnum += rhoA * dAnew;
    const double gam = sqrt(gam2);
    if (!(gam < INFINITY)) {
        if (g == 0 && tid == 0) *S.status = kStatusNonfinite;
        return;
    }
    double c2 = 0.0;
    for (int j = tid; j < d; j += T) c2 += sh.pA[j] * sh.pA[j] + S.mu * sh.pL[j] * sh.pL[j];
    c2 = block_sum(c2, sh.red) + rhoA * rhoA + S.mu * rhoL * rhoL;
    if (!(gam > 1e-14 * sqrt(c2))) {
        // the expansion adds nothing to the projected problem: stop, no append
        if (g == 0 && tid == 0) *S.status = kStatusBreakdown;
        return;
    }
    const double hnew = hnum / gam;
    for (int i = tid; i < D.ns; i += T) {
        S.QA[(int64_t)d * D.s + D.lo + i] = S.wa[D.lo + i] * qsA;
        S.QL[(int64_t)d * D.s + D.lo + i] = S.wl[D.lo + i] * qsL;
    }
    for (int i = tid; i < D.nua; i += T) {
        S.U[(int64_t)d * D.ld2 + D.ulo + i] = S.wu[D.ulo + i] / gam;
        S.U[(int64_t)d * D.ld2 + dmax + D.ulo + i] = S.wu[dmax + D.ulo + i] / gam;
    }
    if (g == 0) {
        for (int j = tid; j < d; j += T) {
            S.RA[(int64_t)d * dmax + j] = sh.pA[j];
            S.RL[(int64_t)d * dmax + j] = sh.pL[j];
            S.G[(int64_t)j * dmax + d] = sh.cA[j];
        }
        if (tid == 0) {
            S.RA[(int64_t)d * dmax + d] = rhoA;
            S.RL[(int64_t)d * dmax + d] = rhoL;
            S.dA[d] = dAnew;
            S.U[(int64_t)d * D.ld2 + d] = rhoA / gam;
            S.U[(int64_t)d * D.ld2 + dmax + d] = S.sqrt_mu * rhoL / gam;
            S.G[(int64_t)d * dmax + d] = gam;
            S.h[d] = hnew;
            if (degA || degL) *S.degenerate += (int)degA + (int)degL;
        }
    }
    // G^{-1} gains column [-G^{-1} g / gam ; 1 / gam]; rows split over workgroups
    double* Gi = S.G + (int64_t)dmax * dmax;
    const int nrow = d + 1;
    const int ylo = (int)((int64_t)nrow * g / G), yhi = (int)((int64_t)nrow * (g + 1) / G);
    const int lane = tid & 63, wave = tid >> 6;
    for (int r = ylo + wave; r < yhi; r += T / 64) {
        double a = 0.0, yr = 0.0;
        if (r < d) {
            const double* gr = Gi + (int64_t)r * dmax;
            for (int j = r + lane; j < d; j += 64) {
                const double gij = gr[j];
                a += gij * sh.cA[j];
                yr += gij * S.h[j];
            }
            a = wave_sum(a);
            yr = wave_sum(yr);
        }
        const double nc = r < d ? -a / gam : 1.0 / gam;
        if (lane == 0) {
            Gi[(int64_t)r * dmax + d] = nc;
            S.y[r] = yr + nc * hnew;
        }
    }
}

// One residual correction of y = G^{-1} h with the triangular factor itself:
// y <- y + G^{-1} (h - G y).  It brings the explicit-inverse solve to the
// accuracy of back substitution.  One workgroup per problem; G and G^{-1}
// row-major.  Ends the append: the basis size becomes d + 1.
__global__ __launch_bounds__(1024) void k_yfix(const State* __restrict__ SS, BTab tab) {
    __shared__ double yv[kMaxD];
    __shared__ double rv[kMaxD];
    __shared__ double tv[kMaxD];
    const State S = load_state(SS, find_slot(tab).p);
    if (*S.status != 0) return;   // no append (breakdown) or an earlier stop
    const int d = *S.d + 1, dmax = S.dmax;
    for (int i = threadIdx.x; i < d; i += 1024) yv[i] = S.y[i];
    __syncthreads();
    tri_mv(S.G, dmax, 1, d, 0, yv, tv);
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += 1024) rv[i] = S.h[i] - tv[i];
    __syncthreads();
    tri_mv(S.G + (int64_t)dmax * dmax, dmax, 1, d, 0, rv, tv);
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += 1024) {
        S.y[i] = yv[i] + tv[i];
        S.yprev[i] = yv[i] + tv[i];
    }
    if (threadIdx.x == 0) *S.d = d;   // every thread read *S.d before the barriers above
}

// ---------------------------------------------------------------------------
// compact append: one workgroup per sketch side; the one that finishes second
// goes on with the stacked factor (side_then_stack).  For modest s and d the
// whole append fits the bandwidth of a few compute units, and one launch
// replaces the chain above (whose cost is the latency of its seven kernel
// boundaries and of the reductions between them).  The stacked step reads the
// other side's results only after the fences around the hand-over count.
// ---------------------------------------------------------------------------

constexpr int kAp1Threads = 512;

// Raw buffer view of the `bytes` bytes at p (the 32-bit data format of CDNA
// buffer resources, no stride): a load whose vector offset plus immediate
// offset reaches `bytes` returns zero instead of reading memory.  The scalar
// offset is added to the address but not checked.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                           uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// one element of type E (double or float) as a double
template <typename E>
__device__ __forceinline__ double buf_load_as(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
    if constexpr (sizeof(E) == 8)
        return buf_load(r, voff, 0u);
    else
        return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0u, 0));
}

// out[j] = sum_{i < s} Q[j s + i] a[i] for j < d: Q column-major s x d in
// memory, a and out in LDS.  Wave w takes C consecutive columns at a time
// (C w + C nw t); lane l holds a at rows l + 64 u (u < R, 64 R >= s, zero past
// s), so the reads of a column past row s meet zeros, and reads past the d
// columns return zero.  All C R loads of a lane are in flight together; the
// C column sums of a wave are reduced together.
template <int R, int C, typename E = double>
__device__ void col_dots(const E* __restrict__ Q, int s, int d, const double* a,
                         double* out) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    constexpr uint32_t es = sizeof(E);
    const __amdgpu_buffer_rsrc_t rq = buf_view(Q, (uint32_t)s * (uint32_t)d * es);
    double av[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = lane + 64 * u;
        av[u] = i < s ? a[i] : 0.0;
    }
    for (int j0 = C * wave; j0 < d; j0 += C * nw) {
        double q[C][R];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const uint32_t vo = ((uint32_t)(j0 + c) * (uint32_t)s + (uint32_t)lane) * es;
#pragma unroll
            for (int u = 0; u < R; ++u) q[c][u] = buf_load_as<E>(rq, vo + 64u * es * u);
        }
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc[c] = 0.0;
#pragma unroll
            for (int u = 0; u < R; ++u) acc[c] += q[c][u] * av[u];
        }
        const double t = wave_sum_scatter<C>(acc);
        const int j = j0 + lane / (64 / C);
        if (lane % (64 / C) == 0 && j < d) out[j] = t;
    }
}

// a[i] -= sum_{j < d} Q[j s + i] p[j] for i < s (Q as in col_dots, p and a in
// LDS).  Wave w takes the rows 64 (w % NR) + lane (NR = ceil(s / 64) chunks)
// and the columns of contiguous part w / NR of P = max(1, nw / NR) parts, C
// columns' loads in flight; the parts' sums meet in scr (P 64 NR doubles, at
// most max(blockDim, 64 ceil(s / 64))) and are added in part order.
template <int C>
__device__ void col_apply(const double* __restrict__ Q, int s, int d, const double* p, double* a,
                          double* scr) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int NR = (s + 63) / 64;
    const int P = NR >= nw ? 1 : nw / NR;
    const __amdgpu_buffer_rsrc_t rq = buf_view(Q, (uint32_t)s * (uint32_t)d * 8u);
    __syncthreads();   // p and a were just written by other threads
    for (int g = wave; g < NR * P; g += nw) {
        const int rc = g % NR, cp = g / NR;
        const int i = 64 * rc + lane;
        const int j0 = (int)((int64_t)d * cp / P), j1 = (int)((int64_t)d * (cp + 1) / P);
        double acc = 0.0;
        for (int j = j0; j < j1; j += C) {
            double q[C];
#pragma unroll
            for (int c = 0; c < C; ++c)
                q[c] = buf_load(rq, ((uint32_t)(j + c) * (uint32_t)s + (uint32_t)i) * 8u, 0u);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double pj = j + c < j1 ? p[j + c] : 0.0;
                acc += q[c] * pj;
            }
        }
        if (i < s) scr[cp * 64 * NR + i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += blockDim.x) {
        double t = 0.0;
        for (int cp = 0; cp < P; ++cp) t += scr[cp * 64 * NR + i];
        a[i] -= t;
    }
    __syncthreads();
}

// a[i] = scale * sum_{b < nb} bins[b s + i], i < s, blocks added in order,
// sixteen loads in flight (the block offset is a scalar).
__device__ void reduce_bins(const double* __restrict__ bins, int nb, int s, double scale,
                            double* a) {
    const __amdgpu_buffer_rsrc_t rb = buf_view(bins, (uint32_t)nb * (uint32_t)s * 8u);
    for (int i = threadIdx.x; i < s; i += blockDim.x) {
        const uint32_t vo = (uint32_t)i * 8u;
        double acc = 0.0;
        for (int b = 0; b < nb; b += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                v[u] = buf_load(rb, vo + (uint32_t)min(b + u, nb - 1) * (uint32_t)s * 8u, 0u);
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (b + u < nb) acc += v[u];
        }
        a[i] = scale * acc;
    }
    __syncthreads();
}

// Autotuning probe: one workgroup of the side-append size reduces nb partial
// bins of s entries as a side append does, into out (s entries).
__global__ __launch_bounds__(kAp1Threads) void k_reduce_bins_probe(const double* __restrict__ bins,
                                                                  int nb, int s, double* out) {
    __shared__ double a[kMaxS];
    reduce_bins(bins, nb, s, 1.0, a);
    for (int i = threadIdx.x; i < s; i += blockDim.x) out[i] = a[i];
}

// One CGS projection of the s-vector a against the d columns of Q:
// p = Q^T a, a -= Q p.  With Q32 the coefficients p come from the FP32 copy
// (the first of two projections); the update always uses the FP64 Q, so a
// stays a - Q p exactly up to FP64 rounding whatever p is.
template <int R, int C>
__device__ void side_project(const double* __restrict__ Q, const float* __restrict__ Q32, int s,
                             int d, double* a, double* p, double* scr) {
    if (Q32)
        col_dots<R, C, float>(Q32, s, d, a, p);
    else
        col_dots<R, C>(Q, s, d, a, p);
    col_apply<16>(Q, s, d, p, a, scr);
}

struct Ap1Side {
    double a[kMaxS];
    double p[kMaxD];     // coefficients of the current projection
    double pt[kMaxD];    // their sum over the projections
    double scr[kMaxS > kAp1Threads ? kMaxS : kAp1Threads];   // col_apply partials
    double red[kAp1Threads / 64];
};

// Workgroup 0 of a problem appends to (Q_A, R_A) and d_A, workgroup 1 to
// (Q_L, R_L): scale of the new column (breakdown test), sketched column from
// the partial bins, CGS projections, new columns of Q and R.  The column index
// d is beyond the basis until the stacked step advances d, so these writes
// are discarded if that step finds the expansion dependent.  rho goes to
// scal[12 + side] (0 when the column is numerically absent), the projection
// coefficients to pacc[(2 + side) dmax + j].
__device__ void ap1_side_body(const State& S, int side, int scale_from_norm, Ap1Side& sh) {
    const int d = *S.d, s = S.s, dmax = S.dmax, tid = threadIdx.x, T = kAp1Threads;
    double scale;
    if (scale_from_norm) {
        const double nr2 = S.scal[14];
        const double nr = sqrt(nr2);
        if (!(nr2 < INFINITY)) {
            if (side == 0 && tid == 0) *S.status = kStatusNonfinite;
            return;
        }
        if (!(nr > 1e-14 * S.scal[0])) {
            if (side == 0 && tid == 0) *S.status = kStatusBreakdown;
            return;
        }
        scale = 1.0 / nr;
        if (side == 0 && tid == 0) S.cs[d] = scale;
    } else {
        scale = S.cs[d];
    }
    const double bscale = S.sketch_mode == kSketchSparseSign ? scale / sqrt((double)S.zeta) : scale;
    double* Q = side ? S.QL : S.QA;
    double* R = side ? S.RL : S.RA;
    reduce_bins(side ? S.binL : S.binA, side ? S.nbL : S.nbA, s, bscale, sh.a);
    double n2 = 0.0;
    for (int i = tid; i < s; i += T) n2 += sh.a[i] * sh.a[i];
    n2 = block_sum(n2, sh.red);
    float* Q32 = side ? S.QL32 : S.QA32;
    for (int pass = 0; pass < S.passes; ++pass) {
        const float* q32 = pass == 0 && S.passes > 1 ? Q32 : nullptr;
        if (s <= 256)
            side_project<4, 4>(Q, q32, s, d, sh.a, sh.p, sh.scr);
        else if (s <= 512)
            side_project<8, 4>(Q, q32, s, d, sh.a, sh.p, sh.scr);
        else
            side_project<16, 2>(Q, q32, s, d, sh.a, sh.p, sh.scr);
        for (int j = tid; j < d; j += T) sh.pt[j] = (pass ? sh.pt[j] : 0.0) + sh.p[j];
        __syncthreads();   // p is rewritten by the next projection
    }
    double r2 = 0.0, dl = 0.0;
    for (int i = tid; i < s; i += T) {
        r2 += sh.a[i] * sh.a[i];
        if (side == 0) dl += sh.a[i] * S.cb[i];
    }
    r2 = block_sum(r2, sh.red);
    dl = block_sum(dl, sh.red);
    double rho = sqrt(r2);
    const bool deg = !(rho > 1e-14 * sqrt(n2));
    if (deg) rho = 0.0;
    const double qs = deg ? 0.0 : 1.0 / rho;
    for (int i = tid; i < s; i += T) {
        const double q = sh.a[i] * qs;
        Q[(int64_t)d * s + i] = q;
        Q32[(int64_t)d * s + i] = (float)q;
    }
    for (int j = tid; j < d; j += T) {
        R[(int64_t)d * dmax + j] = sh.pt[j];
        S.pacc[(int64_t)(2 + side) * dmax + j] = sh.pt[j];
    }
    if (tid == 0) {
        R[(int64_t)d * dmax + d] = rho;
        S.scal[12 + side] = rho;
        if (side == 0) S.dA[d] = deg ? 0.0 : dl / rho;
    }
}


struct Ap1Stack {
    double cA[kMaxD];    // working stacked column, rows < d of the R_A half
    double cL[kMaxD];    // rows < d of the sqrt(mu) R_L half
    double g[kMaxD];     // coefficients of the current projection
    double gt[kMaxD];    // their sum: the new column of G
    double hv[kMaxD + 1];
    double nc[kMaxD + 1];    // new column of G^{-1}
    double yv[kMaxD + 1];
    double rv[kMaxD + 1];
    double tv[kMaxD + 1];
    double red[kAp1Threads / 64];
};

// The stacked factor of [R_A; sqrt(mu) R_L] gains the column [p_A; sqrt(mu) p_L]
// with new-row entries (rho_A, sqrt(mu) rho_L): CGS projections on U, gamma,
// the new columns of U, G and G^{-1}, h, y = G^{-1} h and one residual
// correction y <- y + G^{-1} (h - G y); then d advances.  Breakdown when the
// projected column is dependent.  Run by one workgroup of the side-append
// launch (the one that finishes its side last).
__device__ void ap1_stack_body(const State& S, Ap1Stack& sh) {
    const int d = *S.d, dmax = S.dmax, ld2 = 2 * dmax, tid = threadIdx.x, T = kAp1Threads;
    const double rhoA = S.scal[12], rhoL = S.scal[13];
    const double dAnew = S.dA[d];
    const double new2 = rhoA * rhoA + S.mu * rhoL * rhoL;   // new rows, orthogonal to U
    double c2 = 0.0;
    for (int j = tid; j < d; j += T) {
        sh.cA[j] = S.pacc[(int64_t)2 * dmax + j];
        sh.cL[j] = S.sqrt_mu * S.pacc[(int64_t)3 * dmax + j];
        sh.hv[j] = S.h[j];
        c2 += sh.cA[j] * sh.cA[j] + sh.cL[j] * sh.cL[j];
    }
    c2 = block_sum(c2, sh.red) + new2;
    // U's halves are upper triangular (column k of each half has rows <= k):
    // U(i, k) at U[i + k ld2] (top) and U[dmax + i + k ld2] (bottom)
    for (int pass = 0; pass < S.passes; ++pass) {
        tri_dot2t(S.U, S.U + dmax, 1, ld2, d, sh.cA, sh.cL, sh.g);
        __syncthreads();
        for (int j = tid; j < d; j += T) sh.gt[j] = (pass ? sh.gt[j] : 0.0) + sh.g[j];
        tri_apply2(S.U, S.U + dmax, 1, ld2, d, sh.g, sh.rv, sh.tv);
        __syncthreads();
        for (int i = tid; i < d; i += T) {
            sh.cA[i] -= sh.rv[i];
            sh.cL[i] -= sh.tv[i];
        }
        __syncthreads();
    }
    double gam2 = 0.0, hnum = 0.0;
    for (int i = tid; i < d; i += T) {
        gam2 += sh.cA[i] * sh.cA[i] + sh.cL[i] * sh.cL[i];
        hnum += sh.cA[i] * S.dA[i];
    }
    gam2 = block_sum(gam2, sh.red) + new2;
    hnum = block_sum(hnum, sh.red) + rhoA * dAnew;
    const double gam = sqrt(gam2);
    if (!(gam < INFINITY)) {
        if (tid == 0) *S.status = kStatusNonfinite;
        return;
    }
    if (!(gam > 1e-14 * sqrt(c2))) {
        // the expansion adds nothing to the projected problem: stop, no append
        if (tid == 0) *S.status = kStatusBreakdown;
        return;
    }
    const double hnew = hnum / gam;
    for (int i = tid; i < d; i += T) {
        S.U[(int64_t)d * ld2 + i] = sh.cA[i] / gam;
        S.U[(int64_t)d * ld2 + dmax + i] = sh.cL[i] / gam;
        S.G[(int64_t)i * dmax + d] = sh.gt[i];
    }
    if (tid == 0) {
        S.U[(int64_t)d * ld2 + d] = rhoA / gam;
        S.U[(int64_t)d * ld2 + dmax + d] = S.sqrt_mu * rhoL / gam;
        S.G[(int64_t)d * dmax + d] = gam;
        S.G[(int64_t)dmax * dmax + (int64_t)d * dmax + d] = 1.0 / gam;   // G^{-1}(d, d)
        S.h[d] = hnew;
        sh.hv[d] = hnew;
        sh.nc[d] = 1.0 / gam;
        const int deg = (rhoA == 0.0 ? 1 : 0) + (rhoL == 0.0 ? 1 : 0);
        if (deg) *S.degenerate += deg;
    }
    // G^{-1} gains column [-G^{-1} g / gam; 1 / gam]; y0 = G^{-1} h.  Columns
    // below d of G^{-1} are read from memory, column d only from LDS.
    double* Gi = S.G + (int64_t)dmax * dmax;
    __syncthreads();
    tri_mv2(Gi, dmax, 1, d, sh.gt, sh.hv, sh.rv, sh.tv);
    __syncthreads();
    for (int r = tid; r < d; r += T) {
        const double nc = -sh.rv[r] / gam;
        sh.nc[r] = nc;
        sh.yv[r] = sh.tv[r] + nc * hnew;
        Gi[(int64_t)r * dmax + d] = nc;
    }
    if (tid == 0) sh.yv[d] = hnew / gam;
    __syncthreads();
    // residual correction: t = G y (column d of G from LDS), r = h - t,
    // y += G^{-1} r (column d of G^{-1} from LDS)
    tri_mv(S.G, dmax, 1, d, 0, sh.yv, sh.tv);
    __syncthreads();
    for (int k = tid; k <= d; k += T)
        sh.rv[k] = sh.hv[k] - (k < d ? sh.tv[k] + sh.gt[k] * sh.yv[d] : gam * sh.yv[d]);
    __syncthreads();
    tri_mv(Gi, dmax, 1, d, 0, sh.rv, sh.tv);
    __syncthreads();
    for (int k = tid; k <= d; k += T) {
        const double yk = sh.yv[k] + (k < d ? sh.tv[k] + sh.nc[k] * sh.rv[d] : sh.nc[d] * sh.rv[d]);
        S.y[k] = yk;
        S.yprev[k] = yk;
    }
    if (tid == 0) *S.d = d + 1;   // every thread read *S.d before the barriers above
}

// LDS of the side-append launch: a side append, then (in one workgroup per
// problem) the stacked step in the same space.
struct AppendLds {
    union {
        Ap1Side side;
        Ap1Stack stack;
    } u;
    int last;
};

// After its side append a workgroup counts itself in on the problem's
// counter; the second of the two (the counter read 1) resets the counter for
// the next expansion and runs the stacked step.  The fence before the count
// publishes this side's results, the fence after it makes the other side's
// visible; no workgroup waits for another.  Both side workgroups count on
// every path (also when a status is set), so the counter always returns to 0.
__device__ void side_then_stack(const State& S, int side, int scale_from_norm, AppendLds& sh) {
    if (*S.status == 0) ap1_side_body(S, side, scale_from_norm, sh.u.side);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned old = atomicAdd(S.sync, 1u);
        sh.last = 0;
        if (old == 1u) {
            atomicExch(S.sync, 0u);
            __threadfence();
            sh.last = *S.status == 0 ? 1 : 0;
        }
    }
    __syncthreads();
    if (sh.last) ap1_stack_body(S, sh.u.stack);
}

// The stacked step alone (one workgroup per problem): the appends of the QR
// factors ran before (the unsketched appends of GKS), their R columns in
// pacc[2 dmax ...), pacc[3 dmax ...), rho_A, rho_L in scal[12], scal[13] and d_A[d].
__global__ __launch_bounds__(kAp1Threads) void k_stack_only(const State* __restrict__ SS,
                                                           BTab tab) {
    __shared__ Ap1Stack sh;
    const State S = load_state(SS, find_slot(tab).p);
    if (*S.status != 0) return;
    ap1_stack_body(S, sh);
}

__global__ __launch_bounds__(kAp1Threads) void k_ap1_side(const State* __restrict__ SS, BTab tab,
                                                         int scale_from_norm) {
    __shared__ AppendLds sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    side_then_stack(S, sl.blk, scale_from_norm, sh);
}

// The side appends and the stacked step (workgroups 0 and 1 of each problem)
// together with the adjoint products that add column d of H W from
// (u, t) = (A w, L w) (the remaining workgroups): independent work in one
// launch, so the bandwidth-bound SpMV runs beside the latency-bound appends.
// The adjoint takes its column from scal[15] (written by the new-column
// SpMV), not from d, which the stacked step advances meanwhile.
template <typename T>
__global__ __launch_bounds__(kAp1Threads) void k_ap1_side_hw(const State* __restrict__ SS,
                                                            BTab tab, int scale_from_norm) {
    __shared__ AppendLds sh;
    const Slot sl = find_slot(tab);
    const State S = load_state(SS, sl.p);
    if (sl.blk < 2) {
        side_then_stack(S, sl.blk, scale_from_norm, sh);
        return;
    }
    if (*S.status != 0) return;
    const double cf = S.scal[15];
    const int64_t col = cf >= 0.0 && cf < (double)S.dmax ? (int64_t)cf : 0;   // always in range
    adjoint_body<T, kAp1Threads>(S.At, S.Lt, 1, S.mu, S.u, S.t, S.HW + col * S.n, S.n, nullptr,
                                 sl.blk - 2, sl.nblk - 2, sh.u.side.red);
}

// ---------------------------------------------------------------------------
// iterative refinement step (heavy ball): g = W^T r from partials,
// delta = G^{-1} G^{-T} g, y <- y - alpha delta + beta (y - y_prev)
// ---------------------------------------------------------------------------

constexpr int kRefineThreads = 1024;

__global__ __launch_bounds__(kRefineThreads) void k_refine(const State* __restrict__ SS, BTab tab) {
    __shared__ double gv[kMaxD];
    __shared__ double tv[kMaxD];
    __shared__ double dv[kMaxD];
    const State S = load_state(SS, find_slot(tab).p);
    if (*S.status != 0) return;
    const int d = *S.d;
    const int dmax = S.dmax;
    const double* Gi = S.G + (int64_t)dmax * dmax;   // row-major G^{-1}
    // g = W^T r from the per-workgroup partials: a wave sums four columns at a
    // time, its lanes over the partial rows (sixteen loads in flight)
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const int nb = S.ngt;
        for (int j0 = wave * 4; j0 < d; j0 += nw * 4) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b0 = 0; b0 < nb; b0 += 256) {
                double w[4][4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int b = b0 + lane + 64 * t;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        w[c][t] = b < nb ? S.gpart[(int64_t)b * dmax + min(j0 + c, d - 1)] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] += w[c][t];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double a = wave_sum(acc[c]);
                if (lane == 0 && j0 + c < d) gv[j0 + c] = a;
            }
        }
    }
    __syncthreads();
    tri_mv(Gi, dmax, 1, d, 1, gv, tv);   // t = G^{-T} g
    __syncthreads();
    tri_mv(Gi, dmax, 1, d, 0, tv, dv);   // delta = G^{-1} t
    __syncthreads();
    const double eta2 = fmin((double)d / (double)S.s, 0.999);
    const double alpha = (1.0 - eta2) * (1.0 - eta2), beta = eta2;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        const double yi = S.y[i], yp = S.yprev[i];
        S.y[i] = yi - alpha * dv[i] + beta * (yi - yp);
        S.yprev[i] = yi;
    }
}

// Refinement from the projected normal matrix M = W^T H W kept column by
// column.  The gradient of a refinement step, W^T r(y) for unit columns with
// r(y) = H W y - A^T b, is C (M C y - c) with C = diag(cs) and c_i =
// W[:, i]^T A^T b, an O(d^2) product instead of two passes over n x d data.
// First the newest column c = d - 1 of M and c_c from kb_mcol's partials
// (stored symmetric, row-major), then `steps` heavy-ball steps as k_refine's.
__global__ __launch_bounds__(kRefineThreads) void k_mrefine(const State* __restrict__ SS, BTab tab,
                                                           int steps) {
    __shared__ double gv[kMaxD + 1];
    __shared__ double yv[kMaxD];
    __shared__ double ypv[kMaxD];
    __shared__ double zv[kMaxD];
    __shared__ double tv[kMaxD];
    const State S = load_state(SS, find_slot(tab).p);
    if (*S.status != 0) return;
    const int d = *S.d, c = d - 1, dmax = S.dmax, ld = dmax + 1;
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const int nb = S.ngt, ns = c + 2;
        for (int j0 = wave * 4; j0 < ns; j0 += nw * 4) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b0 = 0; b0 < nb; b0 += 256) {
                double w[4][4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int b = b0 + lane + 64 * t;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        w[q][t] = b < nb ? S.gpart[(int64_t)b * ld + min(j0 + q, ns - 1)] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[q] += w[q][t];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double a = wave_sum(acc[q]);
                if (lane == 0 && j0 + q < ns) gv[j0 + q] = a;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= c; i += blockDim.x) {
        S.Mnt[(int64_t)i * dmax + c] = gv[i];
        S.Mnt[(int64_t)c * dmax + i] = gv[i];
    }
    if (threadIdx.x == 0) S.cnt[c] = gv[c + 1];
    __syncthreads();   // the new row and column are read by the whole workgroup below
    if (steps <= 0) return;
    const double* Gi = S.G + (int64_t)dmax * dmax;   // row-major G^{-1}
    const double eta2 = fmin((double)d / (double)S.s, 0.999);
    const double alpha = (1.0 - eta2) * (1.0 - eta2), beta = eta2;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        yv[i] = S.y[i];
        ypv[i] = S.yprev[i];
    }
    for (int st = 0; st < steps; ++st) {
        __syncthreads();
        for (int i = threadIdx.x; i < d; i += blockDim.x) zv[i] = S.cs[i] * yv[i];
        __syncthreads();
        tri_mv_t(GTri{S.Mnt, dmax, 1}, d, 2, zv, tv, blockDim.x);   // t = M C y
        __syncthreads();
        for (int i = threadIdx.x; i < d; i += blockDim.x) gv[i] = S.cs[i] * (tv[i] - S.cnt[i]);
        __syncthreads();
        tri_mv(Gi, dmax, 1, d, 1, gv, tv);   // G^{-T} g
        __syncthreads();
        tri_mv(Gi, dmax, 1, d, 0, tv, zv);   // delta = G^{-1} G^{-T} g
        __syncthreads();
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            const double yi = yv[i];
            yv[i] = yi - alpha * zv[i] + beta * (yi - ypv[i]);
            ypv[i] = yi;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        S.y[i] = yv[i];
        S.yprev[i] = ypv[i];
    }
}

// ---------------------------------------------------------------------------
// sketched residual from the small factors:
// out2 = ||R_A y - d_A||^2 + ||S_A b||^2 - ||d_A||^2 + mu ||R_L y||^2
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_residual_small(State S, double* out2) {
    __shared__ double red[kWaves];
    __shared__ double yv[kMaxD];
    __shared__ double a_[kMaxD];
    __shared__ double l_[kMaxD];
    const int d = *S.d, dmax = S.dmax;
    for (int i = threadIdx.x; i < d; i += kBlock) yv[i] = S.y[i];
    __syncthreads();
    tri_mv(S.RA, 1, dmax, d, 0, yv, a_);   // R_A y (column-major R: element (i, j) at j dmax + i)
    tri_mv(S.RL, 1, dmax, d, 0, yv, l_);
    __syncthreads();
    double ea = 0.0, el = 0.0, dd = 0.0;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        const double e = a_[i] - S.dA[i];
        ea += e * e;
        el += l_[i] * l_[i];
        dd += S.dA[i] * S.dA[i];
    }
    ea = block_sum(ea, red);
    el = block_sum(el, red);
    dd = block_sum(dd, red);
    if (threadIdx.x == 0) out2[0] = ea + (S.scal[1] - dd) + S.mu * el;
}

// ---------------------------------------------------------------------------
// frozen-basis adjoint, small part: z = G^{-1} G^{-T} W^T g_x,
// v = Q_A (R_A z) (s values), gmu = -(R_L z).(R_L y)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_backward_small(State S, double* v_out,
                                                          double* gmu_out) {
    __shared__ double gv[kMaxD];
    __shared__ double tv[kMaxD];
    __shared__ double zv[kMaxD];
    __shared__ double yv[kMaxD];
    __shared__ double lz[kMaxD];
    __shared__ double ly[kMaxD];
    __shared__ double red[kWaves];
    const int d = *S.d, dmax = S.dmax;
    const double* Gi = S.G + (int64_t)dmax * dmax;   // row-major G^{-1}
    for (int j = threadIdx.x; j < d; j += kBlock) {
        gv[j] = strided_sum(S.gpart + j, dmax, S.ngt);
        yv[j] = S.y[j];
    }
    __syncthreads();
    tri_mv(Gi, dmax, 1, d, 1, gv, tv);   // G^{-T} g
    __syncthreads();
    tri_mv(Gi, dmax, 1, d, 0, tv, zv);   // z = G^{-1} G^{-T} g = H^{-1} W^T grad_x
    __syncthreads();
    tri_mv(S.RA, 1, dmax, d, 0, zv, tv);   // R_A z
    tri_mv(S.RL, 1, dmax, d, 0, zv, lz);   // R_L z
    tri_mv(S.RL, 1, dmax, d, 0, yv, ly);   // R_L y
    __syncthreads();
    double prod = 0.0;
    for (int i = threadIdx.x; i < d; i += kBlock) prod += lz[i] * ly[i];
    prod = block_sum(prod, red);
    for (int r = threadIdx.x; r < S.s; r += kBlock) v_out[r] = strided_dot(S.QA + r, S.s, tv, d);
    if (threadIdx.x == 0) gmu_out[0] = -prod;
}

// ---------------------------------------------------------------------------
// total-derivative adjoint of x_k (reverse sweep over the k expansions and the
// initial Krylov basis).  In exact arithmetic the projected solve of
// eq:projected_sketched_bis on the first d_j columns is
// y_j = N_j^{-1} B_A^T S_A b with B_A = S_A A W_j = Q_A R_A, B_L = S_L L W_j =
// Q_L R_L and N_j = B_A^T B_A + mu B_L^T B_L = G_j^T G_j, G_j the leading block
// of the final stacked factor (the appends never change earlier columns).  The
// adjoint of unit column c collects, over every solve j that uses it,
//   x^_j (y_j)_c + A^T S_A^T (S_A b ubar_c - B_A C[:, c]) - mu L^T S_L^T B_L C[:, c]
// with u_j = N_j^{-1} W_j^T x^_j, ubar = sum_j u_j, C = sum_j (u_j y_j^T + y_j u_j^T)
// (zero padded) and x^_j = H e_j for j < k (x^_k = grad_x).  Column c is final
// once every solve with more than c columns is processed; then e of the
// gradient it was made from is its adjoint divided by ||r|| (its component
// along the column vanishes: x_k depends on the span of W only).
// ---------------------------------------------------------------------------

// one workgroup per problem
__global__ __launch_bounds__(kBlock) void k_record_y(const State* __restrict__ SS) {
    const State S = load_state(SS, blockIdx.x);
    const int d = *S.d;
    double* row = S.yh + (int64_t)d * S.dmax;
    for (int i = threadIdx.x; i < d; i += kBlock) row[i] = S.y[i];
}

// One workgroup of kRevThreads: the triangular products take four lanes per
// row (d <= 256) and the sum over the solves' histories four thread groups.
constexpr int kRevThreads = 1024;

__global__ __launch_bounds__(kRevThreads) void k_rev_small(State S, Rev R, int ell, int k, int j,
                                                          int c, int c_done, int fin) {
    __shared__ double gv[kMaxD];
    __shared__ double tvv[kMaxD];
    __shared__ double uv[kMaxD];
    __shared__ double l1[kMaxD];
    __shared__ double l2[kMaxD];
    __shared__ double sY[kMaxD + 1];
    __shared__ double sU[kMaxD + 1];
    __shared__ double part[4][256];
    __shared__ double red[kRevThreads / 64];
    const int dmax = S.dmax;
    const double* Gi = S.G + (int64_t)dmax * dmax;   // row-major G^{-1}
    const int dk = ell + k;
    if (c_done >= 0) {
        // (L w_c) . (L t_c) of the column just finished: its part of d loss / d mu
        const double a = block_sum(thread_strided_sum(R.ldot, R.nldot, kRevThreads), red);
        if (threadIdx.x == 0) R.rs[0] += S.cs[c_done] * a;
        __syncthreads();
    }
    if (j >= 0) {
        const int dj = ell + j;
        // W_j^T x^_j from the ngt partials: tpc lanes of a wave per column (the largest
        // power of two with tpc dj <= kRevThreads), each summing every tpc-th partial in
        // order, then a shuffle tree (fixed order)
        int tpc = 64;
        while (tpc > 1 && tpc * dj > kRevThreads) tpc >>= 1;
        for (int base = 0; base < dj; base += kRevThreads / tpc) {
            const int i = base + (int)threadIdx.x / tpc, l = threadIdx.x % tpc;
            const int cnt = l < S.ngt ? (S.ngt - l + tpc - 1) / tpc : 0;
            double a = (i < dj) ? strided_sum(S.gpart + (int64_t)l * dmax + min(i, dj - 1),
                                              (int64_t)tpc * dmax, cnt)
                                : 0.0;
            for (int off = tpc / 2; off > 0; off >>= 1) a += __shfl_xor(a, off);
            if (i < dj && l == 0) gv[i] = a;
        }
        __syncthreads();
        tri_mv(Gi, dmax, 1, dj, 1, gv, tvv);   // G_j^{-T} W_j^T x^_j
        __syncthreads();
        tri_mv(Gi, dmax, 1, dj, 0, tvv, uv);   // u_j = N_j^{-1} W_j^T x^_j
        __syncthreads();
        for (int i = threadIdx.x; i < dj; i += kRevThreads) {
            R.uh[(int64_t)dj * dmax + i] = uv[i];
            R.ubar[i] += uv[i];
        }
        __syncthreads();
    }
    if (c >= 0) {
        const int i0 = max(0, c - ell + 1);   // solves with more than c columns
        for (int i = i0 + (int)threadIdx.x; i <= k; i += kRevThreads) {
            sY[i] = S.yh[(int64_t)(ell + i) * dmax + c];
            sU[i] = R.uh[(int64_t)(ell + i) * dmax + c];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            R.rs[1] = sY[k];
            R.rs[2] = R.ubar[c];
        }
        // C[:, c] = sum_i u_i (y_i)_c + y_i (u_i)_c, rows r < dk: group g sums the
        // solves i0 + g, i0 + g + 4, ..., eight in flight; groups added in order
        const int g = threadIdx.x >> 8, rl = threadIdx.x & 255;
        for (int r0 = 0; r0 < dk; r0 += 256) {
            const int r = r0 + rl;
            const int rr = min(r, dk - 1);
            double acc = 0.0;
            for (int i = i0 + g; i <= k; i += 32) {
                double a[8], b[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int ii = min(i + 4 * q, k);
                    a[q] = R.uh[(int64_t)(ell + ii) * dmax + rr];
                    b[q] = S.yh[(int64_t)(ell + ii) * dmax + rr];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (i + 4 * q <= k) acc += a[q] * sY[i + 4 * q] + b[q] * sU[i + 4 * q];
            }
            part[g][rl] = acc;
            __syncthreads();
            if (g == 0 && r < dk) gv[r] = ((part[0][rl] + part[1][rl]) + part[2][rl]) + part[3][rl];
            __syncthreads();
        }
        tri_apply2(S.RA, S.RL, 1, dmax, dk, gv, l1, l2);   // R_A C[:, c], R_L C[:, c]
        __syncthreads();
        for (int r = threadIdx.x; r < dk; r += kRevThreads) {
            R.vA[r] = l1[r];
            R.vL[r] = l2[r];
        }
    }
    if (fin) {
        // the S_A b term of d loss / d b: S_A^T B_A ubar = S_A^T Q_A R_A ubar (negated
        // for the forward product's subtraction)
        for (int i = threadIdx.x; i < dk; i += kRevThreads) gv[i] = R.ubar[i];
        __syncthreads();
        tri_mv(S.RA, 1, dmax, dk, 0, gv, l1);
        __syncthreads();
        for (int r = threadIdx.x; r < dk; r += kRevThreads) {
            R.vA[r] = -l1[r];
            R.vL[r] = 0.0;
        }
        if (threadIdx.x == 0) R.rs[2] = 0.0;
    }
}

// mupart[j] = (R_L u_j) . (R_L y_j) (= (B_L u_j) . (B_L y_j)), one workgroup per solve j
// with d_j = ell + j columns; then the last launch subtracts them in order from
// d loss / d mu
__global__ __launch_bounds__(kBlock) void k_rev_mu(State S, Rev R, int ell) {
    __shared__ double uv[kMaxD];
    __shared__ double yv[kMaxD];
    __shared__ double l1[kMaxD];
    __shared__ double l2[kMaxD];
    __shared__ double red[kWaves];
    const int j = blockIdx.x, dj = ell + j, dmax = S.dmax;
    for (int i = threadIdx.x; i < dj; i += kBlock) {
        uv[i] = R.uh[(int64_t)dj * dmax + i];
        yv[i] = S.yh[(int64_t)dj * dmax + i];
    }
    __syncthreads();
    tri_mv2(S.RL, 1, dmax, dj, uv, yv, l1, l2);
    __syncthreads();
    double pr = 0.0;
    for (int i = threadIdx.x; i < dj; i += kBlock) pr += l1[i] * l2[i];
    pr = block_sum(pr, red);
    if (threadIdx.x == 0) R.mupart[j] = pr;
}

__global__ __launch_bounds__(kBlock) void k_rev_mu_sum(Rev R, int k) {
    __shared__ double red[kWaves];
    const double a = block_sum(thread_strided_sum(R.mupart, k + 1, kBlock), red);
    if (threadIdx.x == 0) R.rs[0] -= a;
}

// kap[c kld + i] = (y_i)_c = yh[(ell + i) dmax + c]
__global__ __launch_bounds__(kBlock) void k_rev_kap(State S, Rev R, int ell, int k) {
    const int dk = ell + k;
    const int64_t tot = (int64_t)dk * (k + 1);
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * kBlock) {
        const int c = (int)(e / (k + 1)), i = (int)(e % (k + 1));
        R.kap[(int64_t)c * R.kld + i] = S.yh[(int64_t)(ell + i) * S.dmax + c];
    }
}

// zA = Q_A vA - S_A b rs[2], zL = Q_L vL: workgroup b < nbs takes 64 rows of
// the A side, the others of the L side; the four waves split the columns
// (every fourth), their sums added in wave order
__global__ __launch_bounds__(kBlock) void k_rev_svec(State S, Rev R, int dk, int nbs) {
    __shared__ double vv[kMaxD];
    __shared__ double part[kWaves][64];
    const bool isA = (int)blockIdx.x < nbs;
    const int blk = isA ? blockIdx.x : blockIdx.x - nbs;
    const double* __restrict__ Q = isA ? S.QA : S.QL;
    const double* __restrict__ v = isA ? R.vA : R.vL;
    for (int i = threadIdx.x; i < dk; i += kBlock) vv[i] = v[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = S.s;
    const int r = blk * 64 + lane;
    const int rr = min(r, s - 1);
    double acc = 0.0;
    int q = wave;
    for (; q + 7 * kWaves < dk; q += 8 * kWaves) {
        double w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = Q[(int64_t)(q + u * kWaves) * s + rr];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += w[u] * vv[q + u * kWaves];
    }
    for (; q < dk; q += kWaves) acc += Q[(int64_t)q * s + rr] * vv[q];
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && r < s) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += part[w][lane];
        if (isA)
            R.zA[r] = t - S.cb[r] * R.rs[2];
        else
            R.zL[r] = t;
    }
}

// sum_q sign_q(i) z[bin_q(i)] over the cached pattern of row i (no scale)
template <int Z>
__device__ __forceinline__ double pattern_gather(const int16_t* __restrict__ pat, int64_t i,
                                                 const double* __restrict__ z) {
    if constexpr (Z == 0) {
        return 0.0;
    } else {
        int bin[Z];
        double sg[Z];
        load_pattern<Z>(pat, i, bin, sg);
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < Z; ++q) a += sg[q] * z[bin[q]];
        return a;
    }
}

// u = A x - S_A^T zA, t = L x - S_L^T zL, and per-workgroup partials of
// (L wc) . (L x).  Z > 0: the sparse-sign transposes formed per row from the
// cached pattern (zeta entries of the s-vector); Z = 0: taken from bA, bL.
template <typename T, int Z>
__global__ __launch_bounds__(kBlock) void k_rev_forward(Csr A, Csr L, int nbA,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ bA,
                                                       const double* __restrict__ bL,
                                                       const double* __restrict__ zA,
                                                       const double* __restrict__ zL,
                                                       const int16_t* __restrict__ patA,
                                                       const int16_t* __restrict__ patL,
                                                       double zscale,
                                                       const double* __restrict__ wc,
                                                       double* __restrict__ u,
                                                       double* __restrict__ t,
                                                       double* __restrict__ ldot) {
    __shared__ double red[kWaves];
    const int blk_all = blockIdx.x;
    const bool isA = blk_all < nbA;
    const Csr& M = isA ? A : L;
    const int nb = isA ? nbA : (int)gridDim.x - nbA;
    const int lb = isA ? blk_all : blk_all - nbA;
    const int blk = xcd_order(lb, nb);
    double dot = 0.0;
    SGKS_LANES_SWITCH(M.lanes, {
        const int64_t row = (int64_t)blk * (kBlock / V) + threadIdx.x / V;
        const int g = threadIdx.x % V;
        if (row < M.rows) {
            const double v = row_dot<V, T>(M, x, row, g);
            const double lw = isA ? 0.0 : row_dot<V, T>(M, wc, row, g);
            if (g == 0) {
                const double sub = Z > 0 ? zscale * pattern_gather<Z>(isA ? patA : patL, row,
                                                                      isA ? zA : zL)
                                         : (isA ? bA[row] : bL[row]);
                if (isA) {
                    u[row] = v - sub;
                } else {
                    t[row] = v - sub;
                    dot = v * lw;
                }
            }
        }
    })
    if (!isA) {
        const double tot = block_sum(dot, red);
        if (threadIdx.x == 0) ldot[lb] = tot;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rev_adjoint(Csr At, Csr Lt, double mu,
                                                       const double* __restrict__ u,
                                                       const double* __restrict__ t, int64_t n,
                                                       const double* __restrict__ gx,
                                                       const double* __restrict__ gcoef,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ dst) {
    const int nblk = gridDim.x;
    const int lb = xcd_order(blockIdx.x, nblk);
    const double gc = *gcoef;
    const double sc = scale ? *scale : 1.0;
    SGKS_LANES_SWITCH(At.lanes, {
        constexpr int rpg = kBlock / V;
        const int64_t ng = (n + rpg - 1) / rpg;
        const int64_t g0 = ng * lb / nblk, g1 = ng * (lb + 1) / nblk;
        const int g = threadIdx.x % V;
        for (int64_t grp = g0; grp < g1; ++grp) {
            const int64_t row = grp * rpg + threadIdx.x / V;
            if (row < n) {
                double v = row_dot<V, T>(At, u, row, g);
                v += mu * row_dot<V, T>(Lt, t, row, g);
                if (g == 0) dst[row] = sc * (v + gc * gx[row]);
            }
        }
    })
}

__global__ __launch_bounds__(kBlock) void k_lincomb(LinComb lc, int64_t n, double* __restrict__ out,
                                                   int accumulate) {
    double cf[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double f = 0.0;
        if (q < lc.nt) {
            const LinTerm& tm = lc.t[q];
            f = tm.h;
            if (tm.d1) f *= tm.inv1 ? 1.0 / *tm.d1 : *tm.d1;
            if (tm.d2) f *= *tm.d2;
        }
        cf[q] = f;
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double a = accumulate ? out[i] : 0.0;
        for (int q = 0; q < lc.nt; ++q) a += cf[q] * lc.t[q].v[i];
        out[i] = a;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// out[i] = sum_q sign_q(i) v[bin_q(i)] / sqrt(zeta)  (S^T v of the stream's
// embedding: 0 S_A, 1 S_L), i < m
template <int Z>
__global__ __launch_bounds__(kBlock) void k_sketch_transpose(const double* __restrict__ v, int s,
                                                            int64_t m, uint64_t seed, int stream,
                                                            int identity, double scale,
                                                            double* __restrict__ out,
                                                            int staged) {
    // v staged in LDS when it fits (staged), else read through the caches
    extern __shared__ double lds[];
    if (staged)
        for (int i = threadIdx.x; i < s; i += kBlock) lds[i] = v[i];
    __syncthreads();
    const double* vs = staged ? lds : v;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        double a;
        if (identity) {
            a = vs[i];
        } else {
            int bin[Z];
            double sg[Z];
            sketch_column<Z>(seed, stream, i, s, bin, sg);
            a = 0.0;
#pragma unroll
            for (int q = 0; q < Z; ++q) a += sg[q] * vs[bin[q]];
            a *= scale;
        }
        out[i] = a;
    }
}

// dst[perm[i] + j n] = W[i + j n] * cs[j] (perm null: the identity)
__global__ __launch_bounds__(kBlock) void k_scaled_W(const double* __restrict__ W,
                                                    const double* __restrict__ cs, int64_t n,
                                                    int d, double* __restrict__ dst,
                                                    const int32_t* __restrict__ perm) {
    const int64_t total = n * (int64_t)d;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t j = k / n, i = k - j * n;
        dst[(perm ? (int64_t)perm[i] : i) + j * n] = W[k] * cs[j];
    }
}

// ---------------------------------------------------------------------------
// internal order of the unknowns (a caller's permutation, e.g. along a
// space-filling curve of the image): order[i] = the caller's unknown at
// internal position i.  The columns of A and L are relabelled once at create
// (the values stay the caller's), so the transposes, W, H W and x are kept in
// the internal order; only the outputs (x_k, W) and the backward's input map
// back.
// ---------------------------------------------------------------------------

// inv[order[i]] = i; flag gets 1 if order is not a permutation of [0, n)
__global__ __launch_bounds__(kBlock) void k_invert_order(const int32_t* __restrict__ order,
                                                        int64_t n, int32_t* __restrict__ inv,
                                                        int* flag) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t o = order[i];
        if (o < 0 || (int64_t)o >= n || atomicCAS(&inv[o], -1, (int32_t)i) != -1)
            atomicOr(flag, 1);
    }
}

// col2[k] = inv[col[k]]
__global__ __launch_bounds__(kBlock) void k_relabel(const int32_t* __restrict__ col, int64_t nnz,
                                                   const int32_t* __restrict__ inv,
                                                   int32_t* __restrict__ col2) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock)
        col2[k] = inv[col[k]];
}

// out[i] = in[perm[i]] (the caller's order into the internal one)
__global__ __launch_bounds__(kBlock) void k_gather_perm(const double* __restrict__ in,
                                                       const int32_t* __restrict__ perm,
                                                       int64_t n, double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        out[i] = in[perm[i]];
}

// ---------------------------------------------------------------------------
// CSR transpose (stable: entries of a transposed row keep increasing order)
// ---------------------------------------------------------------------------

// rowid[k] = row of entry k, iota[k] = k; sixteen lanes per row write its
// entries contiguously
__global__ __launch_bounds__(kBlock) void k_row_ids(const int32_t* __restrict__ rowptr,
                                                   int64_t rows, int32_t* __restrict__ rowid,
                                                   int32_t* __restrict__ iota) {
    constexpr int V = 16;
    const int g = threadIdx.x % V;
    for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / V; r < rows;
         r += (int64_t)gridDim.x * (kBlock / V)) {
        const int b = rowptr[r], e = rowptr[r + 1];
        for (int k = b + g; k < e; k += V) {
            rowid[k] = (int32_t)r;
            iota[k] = k;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_transpose(
    const int32_t* __restrict__ keys, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ rowid, const T* __restrict__ val, int64_t nnz, int64_t cols,
    int32_t* __restrict__ rowptrT, int32_t* __restrict__ colT, T* __restrict__ valT) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        const int32_t e = perm[k];
        colT[k] = rowid[e];
        valT[k] = val[e];
        const int32_t c = keys[k];
        const int32_t prev = k == 0 ? -1 : keys[k - 1];
        for (int32_t q = prev + 1; q <= c; ++q) rowptrT[q] = (int32_t)k;
        if (k == nnz - 1)
            for (int64_t q = (int64_t)c + 1; q <= cols; ++q) rowptrT[q] = (int32_t)nnz;
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ===========================================================================
// launchers
// ===========================================================================

void launch_to_f64(const void* src, int vdt, double* dst, int64_t n, double* part, int nb,
                   hipStream_t st) {
    if (vdt == 0)
        hipLaunchKernelGGL(k_to_f64<float>, dim3(nb), dim3(kBlock), 0, st, (const float*)src, dst,
                           n, part);
    else
        hipLaunchKernelGGL(k_to_f64<double>, dim3(nb), dim3(kBlock), 0, st, (const double*)src,
                           dst, n, part);
}

void launch_sum_parts(const double* part, int nb, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, st, part, nb, out);
}

static int rows_blocks(const Csr& M) {
    const int per = kBlock / M.lanes;
    return (int)((M.rows + per - 1) / per);
}

int forward_blocks(const State& S, bool with_L, int* nbA_out) {
    const int nbA = rows_blocks(S.A);
    const int nbL = with_L ? rows_blocks(S.L) : 0;
    if (nbA_out) *nbA_out = nbA;
    return nbA + nbL;
}

void launch_forward(const State& S, const double* x, const double* b, double* u, double* t,
                    bool with_L, double* upart, double* tpart, hipStream_t st) {
    int nbA = 0;
    const int nb = forward_blocks(S, with_L, &nbA);
    if (S.vdt == 0)
        hipLaunchKernelGGL(k_forward<float>, dim3(nb), dim3(kBlock), 0, st, S.A, S.L, nbA, x, b,
                           u, t, upart, tpart);
    else
        hipLaunchKernelGGL(k_forward<double>, dim3(nb), dim3(kBlock), 0, st, S.A, S.L, nbA, x, b,
                           u, t, upart, tpart);
}

// Workgroups of the H W adjoint of a single problem when it runs beside the
// append chain: the chain's small launches find free wave slots only while the
// adjoint holds fewer than all of them, so its grid is a few workgroups per
// compute unit (grid-stride over the rows; 3 measured best on the dynamic CT
// workload among 2 to 8, 16% more expansions per second than 8).  A batch keeps
// the full grid: there the adjoint products of all problems are most of an
// expansion and the appends are one-workgroup launches.
constexpr int kSideAdjoint_WgPerCu = 3;

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return 256;
    return cus;
}

static int side_adjoint_blocks(const State& S, int cus) {
    const int per = kBlock / S.At.lanes;
    const int64_t groups = (S.n + per - 1) / per;
    const int64_t cap = (int64_t)kSideAdjoint_WgPerCu * cus;
    return (int)(groups < cap ? groups : cap);
}

int adjoint_blocks(const State& S) {
    const int per = kBlock / S.At.lanes;
    const int64_t nb = (S.n + per - 1) / per;
    return (int)(nb < 2048 ? nb : 2048);   // grid-stride beyond: fewer norm partials
}

void launch_adjoint(const State& S, const double* u, const double* t, bool with_L, double mu,
                    double* dst, double* part, hipStream_t st) {
    const int nb = adjoint_blocks(S);
    if (S.vdt == 0)
        hipLaunchKernelGGL(k_adjoint<float>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt,
                           with_L ? 1 : 0, mu, u, t, dst, S.n, part);
    else
        hipLaunchKernelGGL(k_adjoint<double>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt,
                           with_L ? 1 : 0, mu, u, t, dst, S.n, part);
}

// LDS bytes of the scatter for sketch size s: as many copies of the bins as fit
// in kScatterLdsBytes (at most one per wave), at least one
int scatter_ranges(int s) { return (s + kScatterRange - 1) / kScatterRange; }

size_t scatter_lds_bytes(int s) {
    const int R = scatter_ranges(s);
    s = (s + R - 1) / R;   // the sketch rows of one range
    int copies = kScatterLdsBytes / (8 * s);
    if (copies > kSketchWaves) copies = kSketchWaves;
    if (copies < 1) copies = 1;
    return (size_t)copies * s * sizeof(double);
}

void launch_scatter(const State& S, const double* zA, const double* zL, hipStream_t st) {
    const size_t shm = scatter_lds_bytes(S.s);
    const int nbL = zL ? S.nbL : 0;
    const int nb = (S.nbA + nbL) * scatter_ranges(S.s);
#define SGKS_SC(Zv)                                                                             \
    hipLaunchKernelGGL((k_scatter<Zv>), dim3(nb), dim3(kSketchBlock), shm, st, zA, S.m, zL, S.p, \
                       S.nbA, nbL, S.s, S.seed, S.sketch_mode, S.patA, S.patL, S.binA, S.binL, \
                       (int)(shm / sizeof(double)))
    switch (S.zeta) {
        case 2: SGKS_SC(2); break;
        case 4: SGKS_SC(4); break;
        case 16: SGKS_SC(16); break;
        default: SGKS_SC(8); break;
    }
#undef SGKS_SC
}

int srtt_chunks(int64_t h, int* blocks) {
    const int64_t nb = (h + kSrttBlockRows - 1) / kSrttBlockRows;
    *blocks = (int)nb;
    return (int)(nb < kSrttMaxChunks ? nb : kSrttMaxChunks);
}

int srtt_pad(int s) { return ((s + kSrttFT - 1) / kSrttFT) * kSrttFT; }

void launch_srtt_tables(const State& S, hipStream_t st) {
    const int spad = srtt_pad(S.s);
    const int64_t ne = (int64_t)spad * kSrttB;
    const dim3 grid((unsigned)((ne + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_srtt_tables, grid, dim3(kBlock), 0, st, S.rowsA, S.m, S.s, spad,
                       (double*)S.srtTA);
    hipLaunchKernelGGL(k_srtt_tables, grid, dim3(kBlock), 0, st, S.rowsL, S.p, S.s, spad,
                       (double*)S.srtTL);
}

void launch_srtt(const State& S, const double* zA, const double* zL, hipStream_t st) {
    const int nft = (S.s + kSrttFT - 1) / kSrttFT;
    const int nbL = zL ? S.nbL : 0;
    hipLaunchKernelGGL(k_srtt, dim3((S.nbA + nbL) * nft), dim3(kBlock), 0, st, S, zA, zL, nbL);
}

void srtt_rows_host(int64_t h, int s, uint64_t seed, int stream, int32_t* rows) {
    auto mix = [](uint64_t z) {
        z ^= z >> 30;
        z *= 0xBF58476D1CE4E5B9ull;
        z ^= z >> 27;
        z *= 0x94D049BB133111EBull;
        z ^= z >> 31;
        return z;
    };
    const uint64_t gam = 0x9E3779B97F4A7C15ull;
    const uint64_t kr = mix(seed + gam * (uint64_t)(stream + 1));
    std::vector<char> seen((size_t)h, 0);
    uint64_t c = 0;
    for (int j = 0; j < s;) {
        const uint64_t z = mix(kr + gam * (c + 1));
        ++c;
        const int64_t r = (int64_t)(((z >> 32) * (uint64_t)h) >> 32);
        if (!seen[r]) {
            seen[r] = 1;
            rows[j++] = (int32_t)r;
        }
    }
}

int scatter_blocks(int64_t rows, int tiles_per_wave) {
    const int64_t tiles = (rows + 63) / 64;
    const int64_t per = (int64_t)tiles_per_wave * kSketchWaves;
    int64_t nb = (tiles + per - 1) / per;
    if (nb < 1) nb = 1;
    if (nb > kMaxSketchBlocks) nb = kMaxSketchBlocks;
    return (int)nb;
}

void launch_make_pattern(int16_t* pat, int64_t rows, int s, int zeta, uint64_t seed, int stream,
                         hipStream_t st) {
    const int nb = grid_for(rows, kBlock, 4096);
#define SGKS_MP(Zv) \
    hipLaunchKernelGGL((k_make_pattern<Zv>), dim3(nb), dim3(kBlock), 0, st, pat, rows, s, seed, stream)
    switch (zeta) {
        case 2: SGKS_MP(2); break;
        case 4: SGKS_MP(4); break;
        case 16: SGKS_MP(16); break;
        default: SGKS_MP(8); break;
    }
#undef SGKS_MP
}

// z = A w, L w of basis column col into the u, t buffers, then their sketch bins
void launch_sketch_column(const State& S, int col, hipStream_t st) {
    launch_forward(S, S.W + (int64_t)col * S.n, nullptr, S.u, S.t, true, nullptr, nullptr, st);
    if (S.sketch_mode == kSketchSrtt)
        launch_srtt(S, S.u, S.t, st);
    else
        launch_scatter(S, S.u, S.t, st);
}

int gemv_blocks(const State& S) { return grid_for(S.n, kBlock, 4096); }

// workgroups of the gradient kernel (one partial sum of ||r||^2 each)
int gradient_blocks(const State& S) { return grid_for(S.n, kBlock, 2048); }

// adjoint workgroups (kAp1Threads threads) beside the compact side appends
int hw_blocks(const State& S) {
    return grid_for(S.n * (int64_t)S.At.lanes, kAp1Threads, 1024);
}

void launch_gemv(const State& S, const double* coef, double* out, const double* base,
                 int ncols_fixed, hipStream_t st) {
    SGKS_LAUNCH(k_gemv, dim3(gemv_blocks(S)), dim3(kBlock), 0, st, S.W, S.cs, coef, S.d,
                       ncols_fixed, S.n, base, out, (const int32_t*)nullptr);
}

void launch_solution(const State& S, double* out, hipStream_t st) {
    SGKS_LAUNCH(k_gemv, dim3(gemv_blocks(S)), dim3(kBlock), 0, st, S.W, S.cs, S.y, S.d, -1, S.n,
                (const double*)nullptr, out, S.perm);
}

int order_setup(const int32_t* order, int64_t n, int32_t* inv, int* flag, const Csr& A,
                int32_t* colA, const Csr& L, int32_t* colL, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, inv, n,
                       -1);
    hipLaunchKernelGGL(k_invert_order, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st,
                       order, n, inv, flag);
    if (A.nnz > 0)
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(A.nnz, kBlock, 16384)), dim3(kBlock), 0, st,
                           A.col, A.nnz, (const int32_t*)inv, colA);
    if (L.nnz > 0)
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(L.nnz, kBlock, 16384)), dim3(kBlock), 0, st,
                           L.col, L.nnz, (const int32_t*)inv, colL);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

void launch_gather_perm(const double* in, const int32_t* perm, int64_t n, double* out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_gather_perm, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, in,
                       perm, n, out);
}

void launch_gemvt(const State& S, const double* v, int ncols_fixed, hipStream_t st) {
    const size_t shm = (size_t)S.gt_rows * sizeof(double);
    hipLaunchKernelGGL(k_gemvt, dim3(S.ngt), dim3(kBlock), shm, st, S.W, S.cs, v, S.d,
                       ncols_fixed, S.n, S.gt_rows, S.gpart, S.dmax);
}

void launch_reduce_gpart(const State& S, int ncols_fixed, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(kBlock), 0, st, S.gpart, S.ngt, S.dmax, S.d,
                       ncols_fixed, out);
}

void launch_set_scale(const State& S, int col, bool store_r0, hipStream_t st) {
    hipLaunchKernelGGL(k_set_scale, dim3(1), dim3(kBlock), 0, st, S.norm_part, S.n_norm_part,
                       S.cs, col, store_r0 ? 1 : 0, S.scal, S.status);
}

int max_append_groups() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return kMaxAppendGroups;   // no device (a size query on the host): the largest choice
    return cus > 0 ? cus : 1;
}

// G = 1 selects the compact append (one workgroup per side, the second to
// finish also takes the stacked factor); G > 1 the chain of G-workgroup kernels.
bool append_groups_ok(int s, int dmax, int G) {
    if (G == 1) return s <= kMaxS && dmax <= kMaxD;
    return G >= 2 && G <= kMaxAppendGroups && (s + G - 1) / G <= kAppendMaxSlab &&
           (dmax + G - 1) / G <= kAppendMaxSlab;
}

int choose_append_groups(int s, int dmax, int cap, int64_t nnz) {
    const int64_t compact_max = nnz <= kFuseHWMaxNnz ? kCompactAppendMax : kCompactAppendMaxSep;
    if ((int64_t)s * dmax <= compact_max && s <= kMaxS) return 1;
    int G = (s + 31) / 32;
    if (G < 4) G = 4;
    while ((s + G - 1) / G > kAppendMaxSlab || (dmax + G - 1) / G > kAppendMaxSlab) ++G;
    if (G > kMaxAppendGroups) G = kMaxAppendGroups;
    if (G > cap) G = cap;
    return G;
}

void launch_cb(const State& S, hipStream_t st) {
    const double scale = S.sketch_mode == kSketchSparseSign ? 1.0 / sqrt((double)S.zeta) : 1.0;
    hipLaunchKernelGGL(k_cb, dim3(1), dim3(kBlock), 0, st, S.binA, S.nbA, S.s, scale, S.cb,
                       S.scal);
}

void launch_reduce_bins_probe(const double* bins, int nb, int s, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_bins_probe, dim3(1), dim3(kAp1Threads), 0, st, bins, nb, s, out);
}

void launch_residual_small(const State& S, double* out2, hipStream_t st) {
    hipLaunchKernelGGL(k_residual_small, dim3(1), dim3(kBlock), 0, st, S, out2);
}

void launch_backward_small(const State& S, double* v_out, double* gmu_out, hipStream_t st) {
    hipLaunchKernelGGL(k_backward_small, dim3(1), dim3(kBlock), 0, st, S, v_out, gmu_out);
}

void launch_sketch_transpose(const State& S, const double* v, double* out, hipStream_t st) {
    launch_sketch_transpose_side(S, 0, v, out, st);
}

void launch_sketch_transpose_side(const State& S, int side, const double* v, double* out,
                                  hipStream_t st) {
    const int64_t h = side ? S.p : S.m;
    if (S.sketch_mode == kSketchSrtt) {
        // one side's Q tiles (the kernel's first nbA workgroups take S_A, the rest S_L)
        const int per = 16 * kSrttTQ;
        const int nb = (int)(((h + kSrttB - 1) / kSrttB + per - 1) / per);
        hipLaunchKernelGGL(k_srtt_transpose_mfma, dim3(nb), dim3(kBlock), 0, st, v, v, S.s,
                           srtt_pad(S.s), S.m, S.p, S.rowsA, S.rowsL, S.srtTA, S.srtTL, S.seed,
                           side ? 0 : nb, out, out);
        return;
    }
    const int nb = grid_for(h, kBlock, 4096);
    const int staged = (size_t)S.s * sizeof(double) <= (size_t)kScatterLdsBytes ? 1 : 0;
    const size_t shm = staged ? (size_t)S.s * sizeof(double) : 0;
    const double scale = 1.0 / sqrt((double)S.zeta);
    const int ident = S.sketch_mode == 1 ? 1 : 0;
#define SGKS_ST(Zv)                                                                        \
    hipLaunchKernelGGL((k_sketch_transpose<Zv>), dim3(nb), dim3(kBlock), shm, st, v, S.s, \
                       h, S.seed, side, ident, scale, out, staged)
    switch (S.zeta) {
        case 2: SGKS_ST(2); break;
        case 4: SGKS_ST(4); break;
        case 16: SGKS_ST(16); break;
        default: SGKS_ST(8); break;
    }
#undef SGKS_ST
}

void launch_record_y(const State* Sdev, int np, hipStream_t st) {
    SGKS_LAUNCH(k_record_y, dim3(np), dim3(kBlock), 0, st, Sdev);
}

void launch_rev_small(const State& S, const Rev& R, int ell, int k, int j, int c, int c_done,
                      int fin, hipStream_t st) {
    hipLaunchKernelGGL(k_rev_small, dim3(1), dim3(kRevThreads), 0, st, S, R, ell, k, j, c,
                       c_done, fin);
}

void launch_rev_mu(const State& S, const Rev& R, int ell, int k, hipStream_t st) {
    hipLaunchKernelGGL(k_rev_mu, dim3(k + 1), dim3(kBlock), 0, st, S, R, ell);
    hipLaunchKernelGGL(k_rev_mu_sum, dim3(1), dim3(kBlock), 0, st, R, k);
}

void launch_rev_svec(const State& S, const Rev& R, int dk, hipStream_t st) {
    const int nbs = (S.s + 63) / 64;
    hipLaunchKernelGGL(k_rev_svec, dim3(2 * nbs), dim3(kBlock), 0, st, S, R, dk, nbs);
}

void launch_rev_kap(const State& S, const Rev& R, int ell, int k, hipStream_t st) {
    const int64_t tot = (int64_t)(ell + k) * (k + 1);
    hipLaunchKernelGGL(k_rev_kap, dim3(grid_for(tot, kBlock, 1024)), dim3(kBlock), 0, st, S, R,
                       ell, k);
}

void launch_rev_tgemv(const State& S, const Rev& R, int c, int i0, int ncols, hipStream_t st) {
    launch_gemv_plain(S, R.E + (int64_t)i0 * S.n, R.kap + (int64_t)c * R.kld + i0, ncols,
                      nullptr, R.tv, st);
}

void launch_rev_forward(const State& S, const Rev& R, const double* wc, hipStream_t st) {
    int nbA = 0;
    const int nb = forward_blocks(S, true, &nbA);
    const bool pat = S.sketch_mode == kSketchSparseSign && S.patA && S.patL;
    if (S.sketch_mode == kSketchSrtt) {
        // both sides' transposes in one grid (the S_A side alone fills few compute units)
        const int per = 16 * kSrttTQ;
        const int nbA2 = (int)(((S.m + kSrttB - 1) / kSrttB + per - 1) / per);
        const int nbL2 = (int)(((S.p + kSrttB - 1) / kSrttB + per - 1) / per);
        hipLaunchKernelGGL(k_srtt_transpose_mfma, dim3(nbA2 + nbL2), dim3(kBlock), 0, st,
                           (const double*)R.zA, (const double*)R.zL, S.s, srtt_pad(S.s), S.m,
                           S.p, S.rowsA, S.rowsL, S.srtTA, S.srtTL, S.seed, nbA2, R.bA, R.bL);
    } else if (!pat) {   // identity: the transposes in launches of their own
        launch_sketch_transpose_side(S, 0, R.zA, R.bA, st);
        launch_sketch_transpose_side(S, 1, R.zL, R.bL, st);
    }
    const double zs = 1.0 / sqrt((double)S.zeta);
#define SGKS_RF(Tv, Zv)                                                                      \
    hipLaunchKernelGGL((k_rev_forward<Tv, Zv>), dim3(nb), dim3(kBlock), 0, st, S.A, S.L, nbA, \
                       (const double*)R.tv, (const double*)R.bA, (const double*)R.bL,         \
                       (const double*)R.zA, (const double*)R.zL, S.patA, S.patL, zs, wc, S.u, \
                       S.t, R.ldot)
#define SGKS_RF_Z(Tv)                                  \
    if (!pat) {                                        \
        SGKS_RF(Tv, 0);                                \
    } else {                                           \
        switch (S.zeta) {                              \
            case 2: SGKS_RF(Tv, 2); break;             \
            case 4: SGKS_RF(Tv, 4); break;             \
            case 16: SGKS_RF(Tv, 16); break;           \
            default: SGKS_RF(Tv, 8); break;            \
        }                                              \
    }
    if (S.vdt == 0) {
        SGKS_RF_Z(float)
    } else {
        SGKS_RF_Z(double)
    }
#undef SGKS_RF_Z
#undef SGKS_RF
}

void launch_rev_adjoint(const State& S, const Rev& R, const double* gx, const double* scale,
                        double* dst, hipStream_t st) {
    const int nb = adjoint_blocks(S);
    if (S.vdt == 0)
        hipLaunchKernelGGL(k_rev_adjoint<float>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt, S.mu,
                           (const double*)S.u, (const double*)S.t, S.n, gx,
                           (const double*)(R.rs + 1), scale, dst);
    else
        hipLaunchKernelGGL(k_rev_adjoint<double>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt, S.mu,
                           (const double*)S.u, (const double*)S.t, S.n, gx,
                           (const double*)(R.rs + 1), scale, dst);
}

void launch_gemvt_mat(const State& S, const double* M, const double* v, int ncols, hipStream_t st) {
    const size_t shm = (size_t)S.gt_rows * sizeof(double);
    hipLaunchKernelGGL(k_gemvt, dim3(S.ngt), dim3(kBlock), shm, st, M, (const double*)S.cs, v,
                       (const int*)S.d, ncols, S.n, S.gt_rows, S.gpart, S.dmax);
}

void launch_lincomb(const LinComb& lc, int64_t n, double* out, bool accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, lc, n, out,
                       accumulate ? 1 : 0);
}

void launch_gemv_plain(const State& S, const double* M, const double* coef, int ncols,
                       const double* base, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_gemv, dim3(gemv_blocks(S)), dim3(kBlock), 0, st, M, (const double*)nullptr,
                       coef, (const int*)S.d, ncols, S.n, base, out, (const int32_t*)nullptr);
}

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, p, n, v);
}

void launch_scaled_W_cols(const State& S, int col0, int ncols, double* dst, hipStream_t st) {
    if (ncols <= 0) return;
    const int nb = grid_for(S.n * (int64_t)ncols, kBlock, 8192);
    hipLaunchKernelGGL(k_scaled_W, dim3(nb), dim3(kBlock), 0, st, S.W + (int64_t)col0 * S.n,
                       S.cs + col0, S.n, ncols, dst, S.perm);
}

int launch_copy_scaled_W(const State& S, double* dst, hipStream_t st) {
    int dh = 0;
    if (hipMemcpyAsync(&dh, S.d, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    if (dh <= 0) return 0;
    const int nb = grid_for(S.n * (int64_t)dh, kBlock, 8192);
    hipLaunchKernelGGL(k_scaled_W, dim3(nb), dim3(kBlock), 0, st, S.W, S.cs, S.n, dh, dst, S.perm);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// plans: one launch per step for every problem of a set
// ---------------------------------------------------------------------------

static void tab_set(BTab& t, int np, const int* counts) {
    t.np = np;
    t.pref[0] = 0;
    for (int q = 0; q < np; ++q) t.pref[q + 1] = t.pref[q] + counts[q];
    for (int q = np + 1; q <= kMaxBatch; ++q) t.pref[q] = t.pref[np];
}

static int tab_total(const BTab& t) { return t.pref[t.np]; }

int plan_build(Plan& P, const State* host, const State* dev, int np, const int* groups) {
    if (np < 1 || np > kMaxBatch) return -1;
    P.SS = dev;
    P.host = host;
    P.np = np;
    P.method = host[0].method;
    P.vdt = host[0].vdt;
    P.zeta = host[0].zeta;
    P.passes = host[0].passes;
    P.sketch_mode = host[0].sketch_mode;
    P.max_s = 0;
    P.max_gt_rows = 0;
    P.gradient_form = host[0].gradient_form;
    P.record_y = host[0].yh != nullptr ? 1 : 0;
    int fwd[kMaxBatch], adj[kMaxBatch], sc[kMaxBatch], gv[kMaxBatch], gt[kMaxBatch],
        ap[kMaxBatch], apf[kMaxBatch], ap1s[kMaxBatch], one[kMaxBatch],
        gr[kMaxBatch], ap1h[kMaxBatch], ahs[kMaxBatch];
    int64_t nnz_total = 0;
    for (int q = 0; q < np; ++q) nnz_total += host[q].A.nnz + host[q].L.nnz;
    const int cus = np == 1 ? device_cus() : 0;
    P.fuse_hw = nnz_total <= kFuseHWMaxNnz ? 1 : 0;
    for (int q = 0; q < np; ++q) {
        const State& S = host[q];
        if (S.vdt != P.vdt || S.zeta != P.zeta || S.passes != P.passes ||
            S.sketch_mode != P.sketch_mode || S.gradient_form != P.gradient_form ||
            S.method != P.method || (S.method != 0 && np != 1))
            return -1;
        if (!append_groups_ok(S.s, S.dmax, groups[q])) return -1;
        fwd[q] = forward_blocks(S, true, nullptr);
        adj[q] = adjoint_blocks(S);
        sc[q] = S.sketch_mode == kSketchSrtt
                    ? (S.nbA + S.nbL) * ((S.s + kSrttFT - 1) / kSrttFT)
                    : (S.nbA + S.nbL) * scatter_ranges(S.s);
        gv[q] = gemv_blocks(S);
        gr[q] = gradient_blocks(S);
        gt[q] = S.ngt;
        const bool compact = groups[q] == 1;
        ap[q] = compact ? 0 : groups[q];
        apf[q] = compact ? 0 : 1;
        ap1s[q] = compact ? 2 : 0;
        const bool hw = S.gradient_form == 0;
        ap1h[q] = compact ? 2 + (hw && P.fuse_hw ? hw_blocks(S) : 0) : 0;
        ahs[q] = (hw && !(compact && P.fuse_hw))
                     ? (np == 1 ? side_adjoint_blocks(S, cus) : adjoint_blocks(S))
                     : 0;
        one[q] = 1;
        P.max_s = S.s > P.max_s ? S.s : P.max_s;
        P.max_gt_rows = S.gt_rows > P.max_gt_rows ? S.gt_rows : P.max_gt_rows;
    }
    tab_set(P.fwd, np, fwd);
    tab_set(P.adj, np, adj);
    tab_set(P.sc, np, sc);
    tab_set(P.gemv, np, gv);
    tab_set(P.grad, np, gr);
    tab_set(P.gemvt, np, gt);
    tab_set(P.ap, np, ap);
    tab_set(P.ap_fix, np, apf);
    tab_set(P.ap1_side, np, ap1s);
    tab_set(P.ap1_side_hw, np, ap1h);
    tab_set(P.adj_hw_sep, np, ahs);
    tab_set(P.one, np, one);
    return 0;
}

void plan_gemv(const Plan& P, hipStream_t st) {
    SGKS_LAUNCH(kb_gemv, dim3(tab_total(P.gemv)), dim3(kBlock), 0, st, P.SS, P.gemv);
}

// Batched plans take the masked row form (see row_dot).
void plan_forward(const Plan& P, bool newcol, hipStream_t st) {
    const dim3 grid(tab_total(P.fwd));
    const bool m = P.np > 1;
    if (P.vdt == 0) {
        auto* k = m ? &kb_forward<float, true> : &kb_forward<float, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.fwd, newcol ? 1 : 0);
    } else {
        auto* k = m ? &kb_forward<double, true> : &kb_forward<double, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.fwd, newcol ? 1 : 0);
    }
}

void plan_adjoint(const Plan& P, int dst_kind, hipStream_t st) {
    const dim3 grid(tab_total(P.adj));
    const bool m = P.np > 1;
    if (P.vdt == 0) {
        auto* k = m ? &kb_adjoint<float, true> : &kb_adjoint<float, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.adj, dst_kind);
    } else {
        auto* k = m ? &kb_adjoint<double, true> : &kb_adjoint<double, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.adj, dst_kind);
    }
}

void plan_gradient(const Plan& P, bool to_rtmp, hipStream_t st) {
    SGKS_LAUNCH(kb_gradient, dim3(tab_total(P.grad)), dim3(kBlock), 0, st, P.SS, P.grad,
                       to_rtmp ? 1 : 0);
}

void plan_scatter(const Plan& P, hipStream_t st) {
    if (P.sketch_mode == kSketchSrtt) {
        SGKS_LAUNCH(kb_srtt, dim3(tab_total(P.sc)), dim3(kBlock), 0, st, P.SS, P.sc);
        return;
    }
    const size_t shm = scatter_lds_bytes(P.max_s);
    const dim3 grid(tab_total(P.sc));
#define SGKS_SC(Zv) \
    SGKS_LAUNCH((kb_scatter<Zv>), grid, dim3(kSketchBlock), shm, st, P.SS, P.sc, \
                (int)(shm / sizeof(double)))
    switch (P.zeta) {
        case 2: SGKS_SC(2); break;
        case 4: SGKS_SC(4); break;
        case 16: SGKS_SC(16); break;
        default: SGKS_SC(8); break;
    }
#undef SGKS_SC
}

bool plan_has_hw_separate(const Plan& P) {
    return P.gradient_form == 0 && tab_total(P.adj_hw_sep) > 0;
}

void plan_hw_separate(const Plan& P, hipStream_t st) {
    if (!plan_has_hw_separate(P)) return;
    const dim3 grid(tab_total(P.adj_hw_sep));
    const bool m = P.np > 1;
    if (P.vdt == 0) {
        auto* k = m ? &kb_adjoint<float, true> : &kb_adjoint<float, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.adj_hw_sep, kDstHW);
    } else {
        auto* k = m ? &kb_adjoint<double, true> : &kb_adjoint<double, false>;
        SGKS_LAUNCH(k, grid, dim3(kBlock), 0, st, P.SS, P.adj_hw_sep, kDstHW);
    }
}

int plan_append(const Plan& P, bool scale_from_norm, bool with_hw, hipStream_t st) {
    with_hw = with_hw && P.gradient_form == 0;
    if (tab_total(P.ap1_side) > 0) {
        const int sfn = scale_from_norm ? 1 : 0;
        if (!with_hw || !P.fuse_hw)
            SGKS_LAUNCH(k_ap1_side, dim3(tab_total(P.ap1_side)), dim3(kAp1Threads), 0, st,
                               P.SS, P.ap1_side, sfn);
        else if (P.vdt == 0)
            SGKS_LAUNCH(k_ap1_side_hw<float>, dim3(tab_total(P.ap1_side_hw)),
                               dim3(kAp1Threads), 0, st, P.SS, P.ap1_side_hw, sfn);
        else
            SGKS_LAUNCH(k_ap1_side_hw<double>, dim3(tab_total(P.ap1_side_hw)),
                               dim3(kAp1Threads), 0, st, P.SS, P.ap1_side_hw, sfn);
    }
    if (tab_total(P.ap) > 0) {
        const dim3 grid(tab_total(P.ap)), block(kAppendThreads);
        SGKS_LAUNCH(k_ap_q0, grid, block, 0, st, P.SS, P.ap, scale_from_norm ? 1 : 0);
        for (int pass = 1; pass < P.passes; ++pass)
            SGKS_LAUNCH(k_ap_qp, grid, block, 0, st, P.SS, P.ap, pass);
        SGKS_LAUNCH(k_ap_qf, grid, block, 0, st, P.SS, P.ap);
        for (int u = 1; u < P.passes; ++u)
            SGKS_LAUNCH(k_ap_u, grid, block, 0, st, P.SS, P.ap, u, 0);
        SGKS_LAUNCH(k_ap_u, grid, block, 0, st, P.SS, P.ap, P.passes, 1);
        SGKS_LAUNCH(k_ap_commit, grid, block, 0, st, P.SS, P.ap);
        SGKS_LAUNCH(k_yfix, dim3(tab_total(P.ap_fix)), dim3(1024), 0, st, P.SS,
                           P.ap_fix);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

void plan_stack_only(const Plan& P, hipStream_t st) {
    SGKS_LAUNCH(k_stack_only, dim3(P.np), dim3(kAp1Threads), 0, st, P.SS, P.one);
}

void plan_gemvt(const Plan& P, hipStream_t st) {
    const size_t shm = (size_t)P.max_gt_rows * sizeof(double);
    SGKS_LAUNCH(kb_gemvt, dim3(tab_total(P.gemvt)), dim3(kBlock), shm, st, P.SS, P.gemvt);
}

void plan_refine(const Plan& P, hipStream_t st) {
    SGKS_LAUNCH(k_refine, dim3(P.np), dim3(kRefineThreads), 0, st, P.SS, P.one);
}

void plan_mcol(const Plan& P, hipStream_t st) {
    const size_t shm = (size_t)P.max_gt_rows * sizeof(double);
    SGKS_LAUNCH(kb_mcol, dim3(tab_total(P.gemvt)), dim3(kBlock), shm, st, P.SS, P.gemvt);
}

void plan_mrefine(const Plan& P, int steps, hipStream_t st) {
    SGKS_LAUNCH(k_mrefine, dim3(P.np), dim3(kRefineThreads), 0, st, P.SS, P.one, steps);
}

// bytes of scratch the transpose of M needs (four nnz-long int32 arrays and the
// radix sort's storage; host-side size query only)
size_t transpose_scratch_bytes(const Csr& M) {
    if (M.nnz == 0) return 0;
    int bits = 1;
    while ((int64_t(1) << bits) < M.cols) ++bits;
    size_t tmp_bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, M.col, (int32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr,
                                           (int)M.nnz, 0, bits, (hipStream_t)0) != hipSuccess)
        tmp_bytes = (size_t)M.nnz * 16;   // generous when the query fails
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    return 4 * up((size_t)M.nnz * 4) + up(tmp_bytes);
}

int transpose_csr(const Csr& M, int vdt, int32_t* rowptrT, int32_t* colT, void* valT,
                  void* scratch, size_t scratch_bytes, hipStream_t st) {
    const int64_t nnz = M.nnz;
    if (nnz == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(M.cols + 1, kBlock, 4096)), dim3(kBlock), 0,
                           st, rowptrT, M.cols + 1, 0);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    int bits = 1;
    while ((int64_t(1) << bits) < M.cols) ++bits;
    // sort storage (size query only: nothing is read or launched)
    size_t tmp_bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, M.col, (int32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)nnz,
                                           0, bits, st) != hipSuccess)
        return -1;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t a4 = up((size_t)nnz * 4);
    const size_t need = 4 * a4 + up(tmp_bytes);
    char* base = (char*)scratch;
    const bool own = !(scratch && scratch_bytes >= need);
    if (own && hipMalloc((void**)&base, need) != hipSuccess) return -1;
    int32_t* rowid = (int32_t*)base;
    int32_t* iota = (int32_t*)(base + a4);
    int32_t* keys = (int32_t*)(base + 2 * a4);
    int32_t* perm = (int32_t*)(base + 3 * a4);
    void* tmp = base + 4 * a4;
    int rc = 0;
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(M.rows * 16, kBlock, 8192)), dim3(kBlock), 0, st,
                       M.rowptr, M.rows, rowid, iota);
    if (hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, M.col, keys, iota, perm, (int)nnz, 0,
                                           bits, st) != hipSuccess)
        rc = -1;
    if (!rc) {
        const int nb = grid_for(nnz, kBlock, 16384);
        if (vdt == 0)
            hipLaunchKernelGGL(k_gather_transpose<float>, dim3(nb), dim3(kBlock), 0, st, keys,
                               perm, rowid, (const float*)M.val, nnz, M.cols, rowptrT, colT,
                               (float*)valT);
        else
            hipLaunchKernelGGL(k_gather_transpose<double>, dim3(nb), dim3(kBlock), 0, st, keys,
                               perm, rowid, (const double*)M.val, nnz, M.cols, rowptrT, colT,
                               (double*)valT);
        if (hipGetLastError() != hipSuccess) rc = -1;
    }
    if (own) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(base);
    }
    return rc;
}

}  // namespace sgks
