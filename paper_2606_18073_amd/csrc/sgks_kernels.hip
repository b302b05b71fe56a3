// HIP kernels of the sGKS hot path for gfx950 (CDNA4, wave64).
//
// Bulk kernels are bandwidth bound (sparse and dense matrix-vector products,
// O(1) flop per byte): CSR rows are processed by groups of `lanes` lanes of a
// wavefront with a power-of-two group width, FP64 accumulation, and shuffle
// reductions inside the group.  The sparse-sign sketch rides inside the SpMV:
// each wave keeps a private copy of the s sketch bins in LDS, the row pattern
// of the embedding is regenerated from its counter-based hash, and partial
// bins are merged in a fixed order, so results are reproducible run to run.
// The small FP64 steps (rank-one QR appends, the stacked projected factor and
// the projected solve) run in one cooperative launch of a few workgroups that
// each own a slab of rows and meet at a bounded-spin grid barrier.
#include <hipcub/hipcub.hpp>

#include "sgks_internal.h"

namespace sgks {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int V>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = V / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum over a block of blockDim.x (multiple of 64) threads; every thread gets
// the same total (the per-wave sums are added in wave order).
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    __syncthreads();
    return t;
}

template <typename T>
__device__ __forceinline__ double ldv(const void* p, int64_t k) {
    return (double)((const T*)p)[k];
}

// Dot product of one CSR row with x by the V lanes of a group (lane g of V).
template <int V, typename T>
__device__ __forceinline__ double row_dot(const Csr& M, const double* __restrict__ x, int64_t row,
                                          int g) {
    const int32_t* __restrict__ ci = M.col;
    const T* __restrict__ va = (const T*)M.val;
    const int beg = M.rowptr[row], end = M.rowptr[row + 1];
    double acc = 0.0;
    int k = beg + g;
    for (; k + V < end; k += 2 * V) {
        acc += (double)va[k] * x[ci[k]];
        acc += (double)va[k + V] * x[ci[k + V]];
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
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) a += part[i];
    const double t = block_sum(a, red);
    if (threadIdx.x == 0) out[0] = t;
}

// ---------------------------------------------------------------------------
// forward products: u = A x - b (optional b), t = L x
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_forward(Csr A, Csr L, int nbA,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ u, double* __restrict__ t,
                                                   double* upart, double* tpart) {
    __shared__ double red[kWaves];
    const bool isA = (int)blockIdx.x < nbA;
    const Csr M = isA ? A : L;
    const int blk = isA ? (int)blockIdx.x : (int)blockIdx.x - nbA;
    double* out = isA ? u : t;
    const double* sub = isA ? b : nullptr;
    double* part = isA ? upart : tpart;
    double sq = 0.0;
    SGKS_LANES_SWITCH(M.lanes, {
        const int64_t row = (int64_t)blk * (kBlock / V) + threadIdx.x / V;
        const int g = threadIdx.x % V;
        if (row < M.rows) {
            double v = row_dot<V, T>(M, x, row, g);
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

// ---------------------------------------------------------------------------
// adjoint products: r = A^T u + mu L^T t, written to dst (or basis column d),
// with per-block partial sums of r^2
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint(Csr At, Csr Lt, int withL, double mu,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ t,
                                                   double* dst_fixed, double* W, const int* dptr,
                                                   int64_t n, double* part, const int* status) {
    __shared__ double red[kWaves];
    if (status && *status != 0) return;
    double* dst = dst_fixed ? dst_fixed : W + (int64_t)(*dptr) * n;
    double sq = 0.0;
    SGKS_LANES_SWITCH(At.lanes, {
        const int64_t row = (int64_t)blockIdx.x * (kBlock / V) + threadIdx.x / V;
        const int g = threadIdx.x % V;
        if (row < n) {
            double v = row_dot<V, T>(At, u, row, g);
            if (withL) v += mu * row_dot<V, T>(Lt, t, row, g);
            if (g == 0) {
                dst[row] = v;
                sq = v * v;
            }
        }
    })
    const double tot = block_sum(sq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// fused SpMV + sparse-sign sketch:  bins_A += S_A (A x),  bins_L += S_L (L x)
// (or of a vector directly).  Blocks [0, nbA) take A rows, the rest L rows.
// Each wave handles tiles of 64 rows: first the 64 row products (groups of V
// lanes, V passes, each lane collecting the value of "its" row), then every
// lane regenerates the pattern of its row and adds its value into the wave's
// private bins.  Raw bins (no 1/sqrt(zeta), no column scale) per block.
// ---------------------------------------------------------------------------

template <typename T, int Z>
__global__ __launch_bounds__(kBlock) void k_sketch(Csr A, Csr L, int nbA, int nbL,
                                                  const double* xfixed, const double* W,
                                                  const int* dptr, int64_t n, int col,
                                                  int vec_mode, int s, uint64_t seed,
                                                  int identity, double* binA, double* binL,
                                                  const int* status) {
    extern __shared__ double sm[];
    if (status && *status != 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kWaves * s; i += kBlock) sm[i] = 0.0;
    __syncthreads();
    double* bins = sm + wave * s;
    const bool isA = (int)blockIdx.x < nbA;
    const Csr M = isA ? A : L;
    const int blk = isA ? (int)blockIdx.x : (int)blockIdx.x - nbA;
    const int nblk = isA ? nbA : nbL;
    const int stream = isA ? 0 : 1;
    const double* x = xfixed ? xfixed : W + (int64_t)(col >= 0 ? col : *dptr) * n;
    const int64_t ntiles = (M.rows + 63) / 64;
    for (int64_t tile = (int64_t)blk * kWaves + wave; tile < ntiles;
         tile += (int64_t)nblk * kWaves) {
        const int64_t row0 = tile * 64;
        double z = 0.0;
        if (vec_mode) {
            if (row0 + lane < M.rows) z = x[row0 + lane];
        } else {
            SGKS_LANES_SWITCH(M.lanes, {
                constexpr int GP = 64 / V;   // rows per pass
                const int g = lane % V;
                for (int pass = 0; pass < V; ++pass) {
                    const int64_t row = row0 + pass * GP + lane / V;
                    double v = 0.0;
                    if (row < M.rows) v = row_dot<V, T>(M, x, row, g);
                    const double tv = __shfl(v, (lane % GP) * V);
                    if (lane / GP == pass) z = tv;
                }
            })
        }
        const int64_t i = row0 + lane;
        if (i < M.rows) {
            if (identity) {
                atomicAdd(&bins[i], z);
            } else {
                int bin[Z];
                double sg[Z];
                sketch_column<Z>(seed, stream, i, s, bin, sg);
#pragma unroll
                for (int q = 0; q < Z; ++q) atomicAdd(&bins[bin[q]], sg[q] * z);
            }
        }
    }
    __syncthreads();
    double* out = (isA ? binA : binL) + (int64_t)blk * s;
    for (int j = threadIdx.x; j < s; j += kBlock) {
        double a = 0.0;
        for (int w = 0; w < kWaves; ++w) a += sm[w * s + j];
        out[j] = a;
    }
}

// ---------------------------------------------------------------------------
// dense basis products
// ---------------------------------------------------------------------------

// out = [base -] sum_j W[:, j] * cs[j] * coef[j], j < d
__global__ __launch_bounds__(kBlock) void k_gemv(const double* __restrict__ W,
                                                const double* __restrict__ cs,
                                                const double* __restrict__ coef, const int* dptr,
                                                int ncols_fixed, int64_t n,
                                                const double* __restrict__ base,
                                                double* __restrict__ out) {
    __shared__ double yt[kMaxD];
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    for (int j = threadIdx.x; j < d; j += kBlock) yt[j] = cs[j] * coef[j];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double* w = W + i;
        double acc = 0.0;
        int j = 0;
        for (; j + 4 <= d; j += 4) {
            const double w0 = w[(int64_t)j * n], w1 = w[(int64_t)(j + 1) * n];
            const double w2 = w[(int64_t)(j + 2) * n], w3 = w[(int64_t)(j + 3) * n];
            acc += w0 * yt[j];
            acc += w1 * yt[j + 1];
            acc += w2 * yt[j + 2];
            acc += w3 * yt[j + 3];
        }
        for (; j < d; ++j) acc += w[(int64_t)j * n] * yt[j];
        out[i] = base ? base[i] - acc : acc;
    }
}

// part[blk * ld + j] = cs[j] * sum_{i in block rows} W[i, j] v[i], j < d
__global__ __launch_bounds__(kBlock) void k_gemvt(const double* __restrict__ W,
                                                 const double* __restrict__ cs,
                                                 const double* __restrict__ v, const int* dptr,
                                                 int ncols_fixed, int64_t n, int rows_per_block,
                                                 double* __restrict__ part, int ld) {
    extern __shared__ double vs[];
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int nr = (int)min((int64_t)rows_per_block, n - r0);
    for (int i = threadIdx.x; i < nr; i += kBlock) vs[i] = v[r0 + i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < d; j += kWaves) {
        const double* wc = W + (int64_t)j * n + r0;
        double acc = 0.0;
        for (int i = lane; i < nr; i += 64) acc += wc[i] * vs[i];
        acc = wave_sum(acc);
        if (lane == 0) part[(int64_t)blockIdx.x * ld + j] = acc * cs[j];
    }
}

// out[j] = sum_b part[b * ld + j], j < d
__global__ __launch_bounds__(kBlock) void k_reduce_cols(const double* __restrict__ part, int nb,
                                                       int ld, const int* dptr, int ncols_fixed,
                                                       double* __restrict__ out) {
    const int d = ncols_fixed >= 0 ? ncols_fixed : *dptr;
    for (int j = threadIdx.x; j < d; j += kBlock) {
        double a = 0.0;
        for (int b = 0; b < nb; ++b) a += part[(int64_t)b * ld + j];
        out[j] = a;
    }
}

// cs[col] = 1 / ||v|| from the norm partials; optionally scal[0] = ||v||.
__global__ __launch_bounds__(kBlock) void k_set_scale(const double* part, int nb, double* cs,
                                                     int col, int store_r0, double* scal,
                                                     int* status) {
    __shared__ double red[kWaves];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) a += part[i];
    const double t = block_sum(a, red);
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
        double a = 0.0;
        for (int b = 0; b < nb; ++b) a += bins[(int64_t)b * s + i];
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

__device__ bool grid_sync(unsigned* bar, int G) {
    if (G <= 1) {
        __syncthreads();
        return true;
    }
    __shared__ int ok_sh;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        if (arrived == (unsigned)G - 1u) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 22)) {
                    ok = 0;
                    break;
                }
            }
        }
        ok_sh = ok;
    }
    __syncthreads();
    __threadfence();
    return ok_sh != 0;
}

struct AppendSh {
    double aS[kMaxS];
    double lS[kMaxS];
    double pA[kMaxD];
    double pL[kMaxD];
    double cA[kMaxD];
    double cL[kMaxD];
    double cu[2 * kMaxD];
    double red[kAppendThreads / 64];
    double sc[8];
};

__global__ __launch_bounds__(kAppendThreads) void k_append(State S, int scale_from_norm, int G) {
    __shared__ AppendSh sh;
    const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nw = kAppendThreads / 64;
    if (*S.status != 0) return;
    const int d = *S.d;
    const int s = S.s, dmax = S.dmax, ld2 = 2 * dmax;
    const int CW = 2 * dmax + 8;
    double* coop = S.coop;

    // ---- column scale (breakdown test on ||r||, identical in every workgroup)
    double scale;
    if (scale_from_norm) {
        double a = 0.0;
        for (int i = tid; i < S.n_norm_part; i += kAppendThreads) a += S.norm_part[i];
        const double nr2 = block_sum(a, sh.red);
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

    // ---- this workgroup's slab of sketch rows; reduce the partial bins
    const int lo = (int)((int64_t)s * g / G), hi = (int)((int64_t)s * (g + 1) / G);
    const int ns = hi - lo;
    const double bscale = S.sketch_mode == 1 ? scale : scale / sqrt((double)S.zeta);
    double na2 = 0.0, nl2 = 0.0;
    for (int i = tid; i < ns; i += kAppendThreads) {
        double a = 0.0, l = 0.0;
        for (int b = 0; b < S.nbA; ++b) a += S.binA[(int64_t)b * s + lo + i];
        for (int b = 0; b < S.nbL; ++b) l += S.binL[(int64_t)b * s + lo + i];
        a *= bscale;
        l *= bscale;
        sh.aS[i] = a;
        sh.lS[i] = l;
        na2 += a * a;
        nl2 += l * l;
    }
    for (int j = tid; j < d; j += kAppendThreads) {
        sh.pA[j] = 0.0;
        sh.pL[j] = 0.0;
    }
    na2 = block_sum(na2, sh.red);
    nl2 = block_sum(nl2, sh.red);

    // ---- projections (CGS when passes = 1, CGS2 when 2)
    double naTot = 0.0, nlTot = 0.0;
    int region = 0;
    for (int pass = 0; pass < S.passes; ++pass, ++region) {
        double* mine = coop + ((int64_t)region * G + g) * CW;
        for (int j = wave; j < d; j += nw) {
            const double* qa = S.QA + (int64_t)j * s + lo;
            const double* ql = S.QL + (int64_t)j * s + lo;
            double ea = 0.0, el = 0.0;
            for (int i = lane; i < ns; i += 64) {
                ea += qa[i] * sh.aS[i];
                el += ql[i] * sh.lS[i];
            }
            ea = wave_sum(ea);
            el = wave_sum(el);
            if (lane == 0) {
                mine[j] = ea;
                mine[dmax + j] = el;
            }
        }
        if (pass == 0 && tid == 0) {
            mine[2 * dmax] = na2;
            mine[2 * dmax + 1] = nl2;
        }
        if (!grid_sync(S.bar, G)) {
            if (tid == 0) *S.status = kStatusDevice;
            return;
        }
        const double* all = coop + (int64_t)region * G * CW;
        for (int j = tid; j < d; j += kAppendThreads) {
            double ca = 0.0, cl = 0.0;
            for (int q = 0; q < G; ++q) {
                ca += all[(int64_t)q * CW + j];
                cl += all[(int64_t)q * CW + dmax + j];
            }
            sh.cA[j] = ca;
            sh.cL[j] = cl;
            sh.pA[j] += ca;
            sh.pL[j] += cl;
        }
        if (pass == 0) {
            for (int q = 0; q < G; ++q) {
                naTot += all[(int64_t)q * CW + 2 * dmax];
                nlTot += all[(int64_t)q * CW + 2 * dmax + 1];
            }
        }
        __syncthreads();
        for (int i = tid; i < ns; i += kAppendThreads) {
            double ea = 0.0, el = 0.0;
            for (int j = 0; j < d; ++j) {
                ea += S.QA[(int64_t)j * s + lo + i] * sh.cA[j];
                el += S.QL[(int64_t)j * s + lo + i] * sh.cL[j];
            }
            sh.aS[i] -= ea;
            sh.lS[i] -= el;
        }
        __syncthreads();
    }

    // ---- norms of the projected columns and the new d_A entry
    double ra = 0.0, rl = 0.0, dl = 0.0;
    for (int i = tid; i < ns; i += kAppendThreads) {
        ra += sh.aS[i] * sh.aS[i];
        rl += sh.lS[i] * sh.lS[i];
        dl += sh.aS[i] * S.cb[lo + i];
    }
    ra = block_sum(ra, sh.red);
    rl = block_sum(rl, sh.red);
    dl = block_sum(dl, sh.red);
    {
        double* mine = coop + ((int64_t)region * G + g) * CW;
        if (tid == 0) {
            mine[0] = ra;
            mine[1] = rl;
            mine[2] = dl;
        }
        if (!grid_sync(S.bar, G)) {
            if (tid == 0) *S.status = kStatusDevice;
            return;
        }
        const double* all = coop + (int64_t)region * G * CW;
        ra = rl = dl = 0.0;
        for (int q = 0; q < G; ++q) {
            ra += all[(int64_t)q * CW + 0];
            rl += all[(int64_t)q * CW + 1];
            dl += all[(int64_t)q * CW + 2];
        }
        ++region;
    }
    double rhoA = sqrt(ra), rhoL = sqrt(rl);
    const bool degA = !(rhoA > 1e-14 * sqrt(naTot));
    const bool degL = !(rhoL > 1e-14 * sqrt(nlTot));
    if (degA) rhoA = 0.0;
    if (degL) rhoL = 0.0;
    const double qsA = degA ? 0.0 : 1.0 / rhoA, qsL = degL ? 0.0 : 1.0 / rhoL;
    const double dAnew = degA ? 0.0 : dl / rhoA;
    for (int i = tid; i < ns; i += kAppendThreads) {
        S.QA[(int64_t)d * s + lo + i] = sh.aS[i] * qsA;
        S.QL[(int64_t)d * s + lo + i] = sh.lS[i] * qsL;
    }
    if (g == 0) {
        for (int j = tid; j < d; j += kAppendThreads) {
            S.RA[(int64_t)d * dmax + j] = sh.pA[j];
            S.RL[(int64_t)d * dmax + j] = sh.pL[j];
        }
        if (tid == 0) {
            S.RA[(int64_t)d * dmax + d] = rhoA;
            S.RL[(int64_t)d * dmax + d] = rhoL;
            S.dA[d] = dAnew;
            if (degA || degL) *S.degenerate += (int)degA + (int)degL;
        }
    }

    // ---- stacked factor: append c = [p_A, rho_A ; sqrt(mu) p_L, sqrt(mu) rho_L]
    // to U (orthonormal columns) with the same projections; rows of U pair with
    // rows 0..d of R_A (physical rows 0..d) and of R_L (rows dmax..dmax+d).
    const int nrow = d + 1;
    const int ulo = (int)((int64_t)nrow * g / G), uhi = (int)((int64_t)nrow * (g + 1) / G);
    const int nu = uhi - ulo;
    double* cuA = sh.cu;
    double* cuL = sh.cu + kMaxD;
    for (int i = tid; i < nu; i += kAppendThreads) {
        const int r = ulo + i;
        cuA[i] = r < d ? sh.pA[r] : rhoA;
        cuL[i] = S.sqrt_mu * (r < d ? sh.pL[r] : rhoL);
    }
    __syncthreads();
    double* gtmp = sh.cA;   // free after the Q projections
    double* gacc = sh.cL;
    for (int j = tid; j < d; j += kAppendThreads) gacc[j] = 0.0;
    for (int pass = 0; pass < S.passes; ++pass, ++region) {
        double* mine = coop + ((int64_t)region * G + g) * CW;
        for (int j = wave; j < d; j += nw) {
            const double* uc = S.U + (int64_t)j * ld2;
            double e = 0.0;
            for (int i = lane; i < nu; i += 64)
                e += uc[ulo + i] * cuA[i] + uc[dmax + ulo + i] * cuL[i];
            e = wave_sum(e);
            if (lane == 0) mine[j] = e;
        }
        if (!grid_sync(S.bar, G)) {
            if (tid == 0) *S.status = kStatusDevice;
            return;
        }
        const double* all = coop + (int64_t)region * G * CW;
        for (int j = tid; j < d; j += kAppendThreads) {
            double c = 0.0;
            for (int q = 0; q < G; ++q) c += all[(int64_t)q * CW + j];
            gtmp[j] = c;
            gacc[j] += c;
        }
        __syncthreads();
        for (int i = tid; i < nu; i += kAppendThreads) {
            double ea = 0.0, el = 0.0;
            for (int j = 0; j < d; ++j) {
                const double* uc = S.U + (int64_t)j * ld2;
                ea += uc[ulo + i] * gtmp[j];
                el += uc[dmax + ulo + i] * gtmp[j];
            }
            cuA[i] -= ea;
            cuL[i] -= el;
        }
        __syncthreads();
    }
    double gam2 = 0.0, hnum = 0.0;
    for (int i = tid; i < nu; i += kAppendThreads) {
        const int r = ulo + i;
        gam2 += cuA[i] * cuA[i] + cuL[i] * cuL[i];
        hnum += cuA[i] * (r < d ? S.dA[r] : dAnew);
    }
    gam2 = block_sum(gam2, sh.red);
    hnum = block_sum(hnum, sh.red);
    {
        double* mine = coop + ((int64_t)region * G + g) * CW;
        if (tid == 0) {
            mine[0] = gam2;
            mine[1] = hnum;
        }
        if (!grid_sync(S.bar, G)) {
            if (tid == 0) *S.status = kStatusDevice;
            return;
        }
        const double* all = coop + (int64_t)region * G * CW;
        gam2 = hnum = 0.0;
        for (int q = 0; q < G; ++q) {
            gam2 += all[(int64_t)q * CW + 0];
            hnum += all[(int64_t)q * CW + 1];
        }
    }
    const double gam = sqrt(gam2);
    if (!(gam < INFINITY)) {
        if (g == 0 && tid == 0) *S.status = kStatusNonfinite;
        return;
    }
    {
        // the new stacked column must keep more than 1e-14 of its norm after
        // projection, else the expansion adds nothing: stop (breakdown) without
        // appending (identical decision in every workgroup)
        double c2 = rhoA * rhoA + S.mu * rhoL * rhoL;
        for (int j = 0; j < d; ++j) c2 += sh.pA[j] * sh.pA[j] + S.mu * sh.pL[j] * sh.pL[j];
        if (!(gam > 1e-14 * sqrt(c2))) {
            if (g == 0 && tid == 0) *S.status = kStatusBreakdown;
            return;
        }
    }
    const double hnew = hnum / gam;
    for (int i = tid; i < nu; i += kAppendThreads) {
        S.U[(int64_t)d * ld2 + ulo + i] = cuA[i] / gam;
        S.U[(int64_t)d * ld2 + dmax + ulo + i] = cuL[i] / gam;
    }
    if (g == 0) {
        for (int j = tid; j < d; j += kAppendThreads) S.G[(int64_t)d * dmax + j] = gacc[j];
        if (tid == 0) {
            S.G[(int64_t)d * dmax + d] = gam;
            S.h[d] = hnew;
        }
    }

    // ---- G^{-1} gains column [-G^{-1} g / gam ; 1 / gam]; y = G^{-1} h.
    // Rows [ylo, yhi) of this workgroup only need their own rows of G^{-1}.
    // (S.G is reused below as storage of the inverse: column j of the inverse
    // lives in Ginv = S.G + dmax*dmax.)
    double* Ginv = S.G + (int64_t)dmax * dmax;
    const int ylo = ulo, yhi = uhi;
    for (int r = ylo + tid; r < yhi; r += kAppendThreads) {
        double nc, yr = 0.0;
        if (r < d) {
            double a = 0.0;
            for (int j = r; j < d; ++j) {
                const double gi = Ginv[(int64_t)j * dmax + r];
                a += gi * gacc[j];
                yr += gi * S.h[j];
            }
            nc = -a / gam;
        } else {
            nc = 1.0 / gam;
        }
        yr += nc * hnew;
        Ginv[(int64_t)d * dmax + r] = nc;
        S.y[r] = yr;
        S.yprev[r] = yr;
    }
    if (g == 0 && tid == 0) *S.d = d + 1;
}

// ---------------------------------------------------------------------------
// iterative refinement step (heavy ball): g = W^T r from partials,
// delta = G^{-1} G^{-T} g, y <- y - alpha delta + beta (y - y_prev)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_refine(State S) {
    __shared__ double gv[kMaxD];
    __shared__ double tv[kMaxD];
    if (*S.status != 0) return;
    const int d = *S.d;
    const int dmax = S.dmax;
    const double* Ginv = S.G + (int64_t)dmax * dmax;
    for (int j = threadIdx.x; j < d; j += kBlock) {
        double a = 0.0;
        for (int b = 0; b < S.ngt; ++b) a += S.gpart[(int64_t)b * dmax + j];
        gv[j] = a;
    }
    __syncthreads();
    // t = G^{-T} g : t_j = sum_{i <= j} Ginv[i, j] g_i
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < d; j += kWaves) {
        double a = 0.0;
        for (int i = lane; i <= j; i += 64) a += Ginv[(int64_t)j * dmax + i] * gv[i];
        a = wave_sum(a);
        if (lane == 0) tv[j] = a;
    }
    __syncthreads();
    const double eta2 = fmin((double)d / (double)S.s, 0.999);
    const double alpha = (1.0 - eta2) * (1.0 - eta2), beta = eta2;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        double a = 0.0;
        for (int j = i; j < d; ++j) a += Ginv[(int64_t)j * dmax + i] * tv[j];
        const double yi = S.y[i], yp = S.yprev[i];
        S.y[i] = yi - alpha * a + beta * (yi - yp);
        S.yprev[i] = yi;
    }
}

// ---------------------------------------------------------------------------
// sketched residual from the small factors:
// out2 = ||R_A y - d_A||^2 + ||S_A b||^2 - ||d_A||^2 + mu ||R_L y||^2
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_residual_small(State S, double* out2) {
    __shared__ double red[kWaves];
    const int d = *S.d, dmax = S.dmax;
    double ea = 0.0, el = 0.0, dd = 0.0;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        double a = 0.0, l = 0.0;
        for (int j = i; j < d; ++j) {
            a += S.RA[(int64_t)j * dmax + i] * S.y[j];
            l += S.RL[(int64_t)j * dmax + i] * S.y[j];
        }
        const double e = a - S.dA[i];
        ea += e * e;
        el += l * l;
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
    __shared__ double red[kWaves];
    const int d = *S.d, dmax = S.dmax;
    const double* Ginv = S.G + (int64_t)dmax * dmax;
    for (int j = threadIdx.x; j < d; j += kBlock) {
        double a = 0.0;
        for (int b = 0; b < S.ngt; ++b) a += S.gpart[(int64_t)b * dmax + j];
        gv[j] = a;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < d; j += kWaves) {
        double a = 0.0;
        for (int i = lane; i <= j; i += 64) a += Ginv[(int64_t)j * dmax + i] * gv[i];
        a = wave_sum(a);
        if (lane == 0) tv[j] = a;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += kBlock) {
        double a = 0.0;
        for (int j = i; j < d; ++j) a += Ginv[(int64_t)j * dmax + i] * tv[j];
        zv[i] = a;
    }
    __syncthreads();
    // tv <- R_A z, gv <- (R_L z) * (R_L y) terms
    double prod = 0.0;
    for (int i = threadIdx.x; i < d; i += kBlock) {
        double a = 0.0, lz = 0.0, ly = 0.0;
        for (int j = i; j < d; ++j) {
            a += S.RA[(int64_t)j * dmax + i] * zv[j];
            lz += S.RL[(int64_t)j * dmax + i] * zv[j];
            ly += S.RL[(int64_t)j * dmax + i] * S.y[j];
        }
        tv[i] = a;
        prod += lz * ly;
    }
    prod = block_sum(prod, red);   // contains __syncthreads
    for (int r = threadIdx.x; r < S.s; r += kBlock) {
        double a = 0.0;
        for (int j = 0; j < d; ++j) a += S.QA[(int64_t)j * S.s + r] * tv[j];
        v_out[r] = a;
    }
    if (threadIdx.x == 0) gmu_out[0] = -prod;
}

// out[i] = sum_q sign_q(i) v[bin_q(i)] / sqrt(zeta)  (S_A^T v), i < m
template <int Z>
__global__ __launch_bounds__(kBlock) void k_sketch_transpose(const double* __restrict__ v, int s,
                                                            int64_t m, uint64_t seed,
                                                            int identity, double scale,
                                                            double* __restrict__ out) {
    extern __shared__ double vs[];
    for (int i = threadIdx.x; i < s; i += kBlock) vs[i] = v[i];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        double a;
        if (identity) {
            a = vs[i];
        } else {
            int bin[Z];
            double sg[Z];
            sketch_column<Z>(seed, 0, i, s, bin, sg);
            a = 0.0;
#pragma unroll
            for (int q = 0; q < Z; ++q) a += sg[q] * vs[bin[q]];
            a *= scale;
        }
        out[i] = a;
    }
}

// dst[i + j n] = W[i + j n] * cs[j]
__global__ __launch_bounds__(kBlock) void k_scaled_W(const double* __restrict__ W,
                                                    const double* __restrict__ cs, int64_t n,
                                                    int d, double* __restrict__ dst) {
    const int64_t total = n * (int64_t)d;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * kBlock)
        dst[k] = W[k] * cs[k / n];
}

// ---------------------------------------------------------------------------
// CSR transpose (stable: entries of a transposed row keep increasing order)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_row_ids(const int32_t* __restrict__ rowptr,
                                                   int64_t rows, int32_t* __restrict__ rowid,
                                                   int32_t* __restrict__ iota) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * kBlock) {
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            rowid[k] = (int32_t)i;
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

static int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

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
                    bool with_L, double* upart, double* tpart, int nbF, hipStream_t st) {
    int nbA = 0;
    const int nb = forward_blocks(S, with_L, &nbA);
    (void)nbF;
    if (S.vdt == 0)
        hipLaunchKernelGGL(k_forward<float>, dim3(nb), dim3(kBlock), 0, st, S.A, S.L, nbA, x, b,
                           u, t, upart, tpart);
    else
        hipLaunchKernelGGL(k_forward<double>, dim3(nb), dim3(kBlock), 0, st, S.A, S.L, nbA, x, b,
                           u, t, upart, tpart);
}

int adjoint_blocks(const State& S) {
    const int per = kBlock / S.At.lanes;
    return (int)((S.n + per - 1) / per);
}

void launch_adjoint(const State& S, const double* u, const double* t, bool with_L, double mu,
                    double* dst_fixed, bool dst_is_basis_column, double* part, hipStream_t st) {
    const int nb = adjoint_blocks(S);
    const int* status = dst_is_basis_column ? S.status : nullptr;
    if (S.vdt == 0)
        hipLaunchKernelGGL(k_adjoint<float>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt,
                           with_L ? 1 : 0, mu, u, t, dst_fixed, S.W, S.d, S.n, part, status);
    else
        hipLaunchKernelGGL(k_adjoint<double>, dim3(nb), dim3(kBlock), 0, st, S.At, S.Lt,
                           with_L ? 1 : 0, mu, u, t, dst_fixed, S.W, S.d, S.n, part, status);
}

template <typename T>
static void launch_sketch_t(const State& S, int col, bool vec_mode, const double* vec,
                            hipStream_t st) {
    const size_t shm = (size_t)kWaves * S.s * sizeof(double);
    const int nb = S.nbA + (vec_mode ? 0 : S.nbL);
    const int nbL = vec_mode ? 0 : S.nbL;
    const int* status = (col < 0) ? S.status : nullptr;
#define SGKS_SK(Zv)                                                                           \
    hipLaunchKernelGGL((k_sketch<T, Zv>), dim3(nb), dim3(kBlock), shm, st, S.A, S.L, S.nbA,   \
                       nbL, vec, S.W, S.d, S.n, col, vec_mode ? 1 : 0, S.s, S.seed,           \
                       S.sketch_mode, S.binA, S.binL, status)
    switch (S.zeta) {
        case 2: SGKS_SK(2); break;
        case 4: SGKS_SK(4); break;
        case 16: SGKS_SK(16); break;
        default: SGKS_SK(8); break;
    }
#undef SGKS_SK
}

void launch_sketch(const State& S, int col, bool vec_mode, const double* vec, hipStream_t st) {
    if (S.vdt == 0)
        launch_sketch_t<float>(S, col, vec_mode, vec, st);
    else
        launch_sketch_t<double>(S, col, vec_mode, vec, st);
}

void launch_gemv(const State& S, const double* coef, bool coef_from_cs, double* out,
                 const double* base, int ncols_fixed, hipStream_t st) {
    (void)coef_from_cs;
    const int nb = grid_for(S.n, kBlock, 4096);
    hipLaunchKernelGGL(k_gemv, dim3(nb), dim3(kBlock), 0, st, S.W, S.cs, coef, S.d, ncols_fixed,
                       S.n, base, out);
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
    int dev = 0;
    hipGetDevice(&dev);
    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 1;
}

int launch_append(const State& S, bool scale_from_norm, int groups, hipStream_t st) {
    int sfn = scale_from_norm ? 1 : 0;
    int G = groups;
    State Sc = S;
    if (G <= 1) {
        hipLaunchKernelGGL(k_append, dim3(1), dim3(kAppendThreads), 0, st, Sc, sfn, 1);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    void* args[] = {&Sc, &sfn, &G};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_append, dim3(G),
                                              dim3(kAppendThreads), args, 0, st);
    return e == hipSuccess ? 0 : -1;
}

void launch_refine(const State& S, hipStream_t st) {
    hipLaunchKernelGGL(k_refine, dim3(1), dim3(kBlock), 0, st, S);
}

void launch_cb(const State& S, hipStream_t st) {
    const double scale = S.sketch_mode == 1 ? 1.0 : 1.0 / sqrt((double)S.zeta);
    hipLaunchKernelGGL(k_cb, dim3(1), dim3(kBlock), 0, st, S.binA, S.nbA, S.s, scale, S.cb,
                       S.scal);
}

void launch_residual_small(const State& S, double* out2, hipStream_t st) {
    hipLaunchKernelGGL(k_residual_small, dim3(1), dim3(kBlock), 0, st, S, out2);
}

void launch_backward_small(const State& S, double* v_out, double* gmu_out, hipStream_t st) {
    hipLaunchKernelGGL(k_backward_small, dim3(1), dim3(kBlock), 0, st, S, v_out, gmu_out);
}

void launch_sketch_transpose(const State& S, const double* v, double* out, hipStream_t st) {
    const int nb = grid_for(S.m, kBlock, 4096);
    const size_t shm = (size_t)S.s * sizeof(double);
    const double scale = 1.0 / sqrt((double)S.zeta);
    const int ident = S.sketch_mode == 1 ? 1 : 0;
#define SGKS_ST(Zv)                                                                        \
    hipLaunchKernelGGL((k_sketch_transpose<Zv>), dim3(nb), dim3(kBlock), shm, st, v, S.s, \
                       S.m, S.seed, ident, scale, out)
    switch (S.zeta) {
        case 2: SGKS_ST(2); break;
        case 4: SGKS_ST(4); break;
        case 16: SGKS_ST(16); break;
        default: SGKS_ST(8); break;
    }
#undef SGKS_ST
}

void launch_copy_scaled_W(const State& S, double* dst, hipStream_t st) {
    const int d = 0;
    (void)d;
    int dh = 0;
    hipMemcpyAsync(&dh, S.d, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (dh <= 0) return;
    const int nb = grid_for(S.n * (int64_t)dh, kBlock, 8192);
    hipLaunchKernelGGL(k_scaled_W, dim3(nb), dim3(kBlock), 0, st, S.W, S.cs, S.n, dh, dst);
}

int transpose_csr(const Csr& M, int vdt, int32_t* rowptrT, int32_t* colT, void* valT,
                  hipStream_t st) {
    const int64_t nnz = M.nnz;
    if (nnz == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(M.cols + 1, kBlock, 4096)), dim3(kBlock), 0,
                           st, rowptrT, M.cols + 1, 0);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    int32_t *rowid = nullptr, *iota = nullptr, *keys = nullptr, *perm = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    int rc = 0;
    if (hipMalloc(&rowid, nnz * 4) != hipSuccess || hipMalloc(&iota, nnz * 4) != hipSuccess ||
        hipMalloc(&keys, nnz * 4) != hipSuccess || hipMalloc(&perm, nnz * 4) != hipSuccess) {
        rc = -1;
    }
    int bits = 1;
    while ((int64_t(1) << bits) < M.cols) ++bits;
    if (!rc) {
        hipLaunchKernelGGL(k_row_ids, dim3(grid_for(M.rows, kBlock, 8192)), dim3(kBlock), 0, st,
                           M.rowptr, M.rows, rowid, iota);
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, M.col, keys, iota, perm,
                                               (int)nnz, 0, bits, st) != hipSuccess ||
            hipMalloc(&tmp, tmp_bytes) != hipSuccess)
            rc = -1;
    }
    if (!rc && hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, M.col, keys, iota, perm,
                                                  (int)nnz, 0, bits, st) != hipSuccess)
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
    hipStreamSynchronize(st);
    hipFree(rowid);
    hipFree(iota);
    hipFree(keys);
    hipFree(perm);
    hipFree(tmp);
    return rc;
}

}  // namespace sgks
