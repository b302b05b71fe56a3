// Internal declarations shared by the host runtime (sgks_api.hip) and the
// kernels (sgks_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgks {

// Kernel timing while profiling.  A timer set on the enqueueing thread hands
// every launch of the iteration path an event pair; that launch then goes
// through hipExtLaunchKernelGGL, whose events take the begin and end
// timestamps of the kernel's own execution (the dispatch gap before it is not
// included, as in a kernel trace).
struct LaunchTimer {
    virtual bool pair(hipEvent_t* begin, hipEvent_t* end) = 0;

protected:
    ~LaunchTimer() = default;
};
extern thread_local LaunchTimer* tl_launch_timer;

#define SGKS_LAUNCH(K, G, B, SH, ST, ...)                                               \
    do {                                                                                \
        hipEvent_t sgks_e0_, sgks_e1_;                                                  \
        if (::sgks::tl_launch_timer && ::sgks::tl_launch_timer->pair(&sgks_e0_, &sgks_e1_)) \
            hipExtLaunchKernelGGL(K, G, B, SH, ST, sgks_e0_, sgks_e1_, 0, __VA_ARGS__);  \
        else                                                                            \
            hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                           \
    } while (0)

constexpr int kBlock = 256;         // threads per block of the bulk kernels
constexpr int kWaves = kBlock / 64; // waves per block
constexpr int kMaxS = 1024;         // largest sketch size of the one-workgroup append (LDS vectors)
constexpr int kMaxSketch = 16384;   // largest sketch size (the multi-workgroup append)
// LDS of the sketch scatter: wave-private copies of the s bins while they fit in
// 64 KiB (8 copies up to s = 1024), fewer, shared by several waves, beyond; one
// copy of s doubles needs s * 8 bytes of one workgroup's LDS
constexpr int kScatterLdsBytes = 64 * 1024;
// sketch rows of one scatter range: beyond, the rows are split into ranges, each
// scatter workgroup taking one range of its tiles' bins (the tiles are read once
// per range)
constexpr int kScatterRange = kScatterLdsBytes / 8;
constexpr int kMaxD = 512;          // largest basis dimension
constexpr int kAppendThreads = 512; // threads per workgroup of the append chain kernels
constexpr int kMaxAppendGroups = 256; // workgroups of the append kernels
constexpr int kAppendMaxSlab = 64;    // sketch rows per append workgroup
constexpr int kSketchBlock = 512;   // threads per block of the sketch kernel
constexpr int kSketchWaves = kSketchBlock / 64;
constexpr int kMaxSketchBlocks = 256; // per operator
constexpr int kMaxBatch = 64;       // problems of one batched launch
// total nonzeros of A and L (over a plan's problems) up to which the adjoint
// products that add the H W column run inside the compact side launch: short
// enough to hide behind the latency-bound appends; beyond, they run in a launch
// of their own at full occupancy
constexpr int64_t kFuseHWMaxNnz = 12000000;
// s * dmax up to which the compact append (one workgroup per side) is chosen;
// beyond, the bandwidth of one compute unit makes the multi-workgroup chain
// faster.  With the H W adjoint in a launch of its own (larger operators) the
// chain, which overlaps that launch, wins earlier: measured at s * dmax =
// 91,800 (CT, 256 x 256) the chain is 4% faster per expansion, at 41,200
// (deblurring, H W inside the compact launch) the compact append 1.5x.
constexpr int64_t kCompactAppendMax = 120000;
constexpr int64_t kCompactAppendMaxSep = 60000;

// sketch kinds inside the library: the public ones, and none (GKS)
constexpr int kSketchSparseSign = 0, kSketchIdentity = 1, kSketchSrtt = 2, kSketchNone = 3;
// SRTT sketch: output frequencies per workgroup (one per thread), rows per chunk
constexpr int kSrttThreads = 256;
constexpr int kSrttMaxChunks = 32;   // SRTT ranges per side (partial bins): 32 and 16 measured
                                     // best (dynamic CT: 342 and 337 us per sketch; 128: 392, 8: 398)

// Device status word values (mirrors the public codes).
constexpr int kStatusOk = 0;
constexpr int kStatusBreakdown = 1;
constexpr int kStatusNonfinite = -7;
constexpr int kStatusDevice = -9;

// A CSR operator as the kernels see it.  vdt: 0 = float values, 1 = double.
struct Csr {
    int64_t rows;
    int64_t cols;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* col;
    const void* val;
    int lanes;      // lanes of a wavefront that share one row (1..64, power of 2)
};

// Everything the iteration kernels read or write.  Column-major layouts.
struct State {
    int64_t m, n, p;
    int s;           // sketch rows
    int dmax;        // capacity of the basis
    int zeta;
    int passes;      // projections per QR append (1 or 2)
    int sketch_mode; // kSketchSparseSign, kSketchIdentity, kSketchSrtt or kSketchNone
    int vdt;         // value dtype of A, L
    int gradient_form; // 0: r from the maintained H W; 1: r = A^T (A x - b) + mu L^T L x directly
    uint64_t seed;
    double mu;
    double sqrt_mu;

    Csr A, At, L, Lt;

    const int32_t* perm; // internal order of the unknowns: perm[i] = caller's index (null: same)
    const double* b;   // m
    double* x;         // n
    double* u;         // m
    double* t;         // p
    double* rtmp;      // n (refinement gradient, adjoint input)
    double* W;         // n x dmax, column j = r_j (unnormalised), scaled by cs[j]
    double* HW;        // n x dmax, column j = (A^T A + mu L^T L) W[:, j] (maintained gradient form)
    double* cs;        // dmax column scales (1 / ||column||)

    double* QA;        // s x dmax
    double* RA;        // dmax x dmax
    double* QL;        // s x dmax
    double* RL;        // dmax x dmax
    // FP32 copies of Q_A, Q_L, kept by the one-workgroup append for the first of
    // two projections (whose coefficients only need to be approximate: the
    // FP64 second projection measures and removes what the first one left)
    float* QA32;
    float* QL32;
    double* U;         // (2 dmax) x dmax: rows [0,dmax) pair with R_A, rows [dmax,2dmax) with R_L
    double* G;         // dmax x dmax R factor of [R_A; sqrt(mu) R_L], then G^{-1}; both row-major
    double* h;         // dmax, U^T [d_A; 0]
    double* dA;        // dmax
    double* cb;        // s, S_A b
    double* y;         // dmax
    double* yprev;     // dmax

    double* norm_part; // partial sums of ||r||^2 (one per block of the adjoint kernel)
    int n_norm_part;
    double* binA;      // nbA x s partial sketch bins of the A column (one per block)
    double* binL;      // nbL x s partial sketch bins of the L column
    int nbA, nbL;
    // sparse-sign pattern of S_A (m x zeta) and S_L (p x zeta), computed once
    // from the hash: entry i*zeta + q = +-(row + 1) (sign of the entry), 0 if none
    const int16_t* patA;
    const int16_t* patL;
    // SRTT: the s frequencies D selects on each side (draw order); the cosine and
    // sine tables of each side (2 x spad x 256, spad = s rounded up to 16); the
    // blocks of 4096 image rows (srA of m, srL of p), split into the nbA, nbL
    // ranges whose partial sums are the partial bins
    const int32_t* rowsA;
    const int32_t* rowsL;
    const double* srtTA;
    const double* srtTL;
    int srA, srL;
    double* wa;        // s: working sketched A column of the append
    double* wl;        // s: working sketched L column
    double* wu;        // 2 dmax: working column of the stacked factor
    double* pacc;      // 4 dmax: running sums of the Q projection coefficients, final sums
    double* gacc;      // dmax: running sum of the U projection coefficients
    double* gpart;     // ngt x (dmax + 1) partial W^T v sums
    double* Mnt;       // dmax x dmax row-major W^T H W, raw columns (maintained form with
                       // refinement; else null)
    double* cnt;       // dmax: W[:, i]^T A^T b, raw columns (with Mnt)
    int ngt;
    int gt_rows;       // rows per block of the W^T v kernel
    double* yh;        // (dmax + 1) x dmax: row d = y of the projected solve with d columns
                       // (recorded for the total-derivative adjoint; else null)
    double* coop;      // partial vectors of the append kernels (regions x (2 dmax + 8) x G)
    double* scal;      // scalars: [0] ||A^T b||, [1] ||S_A b||^2, [2..] scratch
    int* d;            // current number of basis columns
    int* status;       // device status word
    int* degenerate;   // count of numerically absent QR columns
    unsigned* sync;    // side appends finished this expansion (0 between launches)

    // GKS (Alg. 1) only: the basis W is orthonormal (columns scaled by cs), the
    // QR factors are of the unsketched A W and L W
    int method;        // 0 sGKS, 1 GKS
    double* QAt;       // m x dmax, Q of A W
    double* QLt;       // p x dmax, Q of L W
    double* wat;       // m: working column of the A-side append
    double* wlt;       // p: working column of the L-side append
    double* tpA;       // ntA x dmax partial column dots over the A-side row slabs
    double* tpL;       // ntL x dmax partial column dots over the L-side row slabs
    double* tsq;       // 8 x (ntA + ntL) partial sums of the appends (norms, w . b)
    double* gco;       // 6 dmax: projection coefficients (V pass 0, 1; A, L pass 0, 1 ...)
    double* vsq;       // 2 x 2048 partial sums of ||v||^2 after each V projection pass
    int ntA, ntL;      // row slabs of the A-side and L-side appends
    int trA, trL;      // rows per slab
};

// Buffers of the total-derivative adjoint (reverse sweep over the expansions).
// Column-major n-vectors; e_j is the adjoint of the gradient r_j.
struct Rev {
    double* uh;     // (dmax + 1) x dmax: row d = u of the adjoint solve with d columns
    double* E;      // n x max_iters: e_j, j < k
    double* vbar;   // n x ell: adjoints of the (unit) initial columns
    double* tv;     // n: sum_i (y_i)_c e_i of the current column c
    double* zb;     // n: scratch of the initial-basis reverse
    double* pb;     // n
    double* zh;     // n
    double* bA;     // m: S_A^T of zA
    double* bL;     // p: S_L^T of zL
    double* zA;     // s: Q_A R_A C[:, c] - S_A b ubar_c
    double* zL;     // s: Q_L R_L C[:, c]
    double* ldot;   // nldot workgroup partials of (L w_c) . (L t)
    double* ubar;   // dmax: sum of the u of every solve (zero padded)
    double* vA;     // dmax: R_A C[:, c]
    double* vL;     // dmax: R_L C[:, c]
    double* dz;     // dmax: coefficient vectors of the initial-basis reverse
    double* dp;     // dmax
    double* kap;    // d_max x kld: row c = (y_i)_c, i <= k (the coefficients of tv for column c)
    int kld;        // max_iters + 1
    double* ones;   // max_iters
    double* rs;     // 16 scalars: [0] d loss / d mu, [1] (y_k)_c, [2] ubar_c
    double* mupart; // max_iters + 1: (B_L u_j) . (B_L y_j) of each solve
    int nldot;
};

// Block table of one batched launch: problem q owns the workgroups
// [pref[q], pref[q + 1]) of the grid, q < np.  Passed by value.
struct BTab {
    int np;
    int pref[kMaxBatch + 1];
};

// Launch plan of the iteration over a set of problems whose States live in
// device memory (SS[q]).  Options that select kernel instantiations (value
// dtype, zeta, projection passes) are common to the set.
struct Plan {
    const State* SS;
    const State* host;   // host copy of problem 0's State (the GKS launchers read its shapes)
    int np;
    int method;         // 0 sGKS, 1 GKS (one problem)
    int vdt, zeta, passes, sketch_mode, gradient_form;
    int max_s;          // largest sketch size (LDS bins of the scatter)
    int max_gt_rows;    // largest row slab of the W^T v kernel
    BTab fwd;           // k_forward: A rows then L rows
    BTab adj;           // adjoint products
    BTab sc;            // scatter: S_A blocks then S_L blocks
    BTab gemv;          // x = W y
    BTab grad;          // gradient from H W
    BTab gemvt;         // W^T v partials
    BTab ap;            // append chain workgroups (problems with more than one append group)
    BTab ap_fix;        // one workgroup per chain problem (k_yfix)
    BTab ap1_side;      // compact append: two workgroups per problem (one append group)
    BTab ap1_side_hw;   // compact append with the H W column: 2 + hw_blocks per problem
    BTab adj_hw_sep;    // H W column in a launch of its own (adjoint workgroups)
    int fuse_hw;        // H W column inside the compact side launch (small total nnz)
    int record_y;       // the problems keep the y history (keep_history, common to the set)
    BTab one;           // one workgroup per problem
};

// ----- launchers (sgks_kernels.hip) -----------------------------------------
void launch_to_f64(const void* src, int vdt, double* dst, int64_t n, double* part, int nb,
                   hipStream_t st);
void launch_sum_parts(const double* part, int nb, double* out, hipStream_t st);
void launch_forward(const State& S, const double* x, const double* b, double* u, double* t,
                    bool with_L, double* upart, double* tpart, hipStream_t st);
int forward_blocks(const State& S, bool with_L, int* nbA_out);
void launch_adjoint(const State& S, const double* u, const double* t, bool with_L, double mu,
                    double* dst, double* part, hipStream_t st);
int adjoint_blocks(const State& S);
void launch_sketch_column(const State& S, int col, hipStream_t st);
void launch_scatter(const State& S, const double* zA, const double* zL, hipStream_t st);
void launch_gemv(const State& S, const double* coef, double* out, const double* base,
                 int ncols_fixed, hipStream_t st);
int gemv_blocks(const State& S);
int gradient_blocks(const State& S);
int hw_blocks(const State& S);
void launch_gemvt(const State& S, const double* v, int ncols_fixed, hipStream_t st);
void launch_reduce_gpart(const State& S, int ncols_fixed, double* out, hipStream_t st);
void launch_set_scale(const State& S, int col, bool store_r0, hipStream_t st);
int choose_append_groups(int s, int dmax, int cap, int64_t nnz);
bool append_groups_ok(int s, int dmax, int G);
void launch_cb(const State& S, hipStream_t st);
void launch_residual_small(const State& S, double* out2, hipStream_t st);
void launch_backward_small(const State& S, double* v_out, double* gmu_out, hipStream_t st);
void launch_sketch_transpose(const State& S, const double* v, double* out, hipStream_t st);
// S^T v of one side's embedding (0: S_A, m outputs; 1: S_L, p outputs)
void launch_sketch_transpose_side(const State& S, int side, const double* v, double* out,
                                  hipStream_t st);
// ----- total-derivative adjoint (reverse sweep) ----------------------------
// row d of yh = y for each of the np problems of a device State array
void launch_record_y(const State* Sdev, int np, hipStream_t st);
// one-workgroup step: j >= 0 the adjoint solve of the projected problem with
// ell + j columns (from the W^T partials in gpart); c >= 0 the small data of
// column c; c_done >= 0 adds the L partials of column c_done to d loss / d mu;
// fin: R_A ubar for the S_A b term
void launch_rev_small(const State& S, const Rev& R, int ell, int k, int j, int c, int c_done,
                      int fin, hipStream_t st);
void launch_rev_svec(const State& S, const Rev& R, int dk, hipStream_t st);
// d loss / d mu -= sum_j (B_L u_j) . (B_L y_j) over the k + 1 solves (after the sweep)
void launch_rev_mu(const State& S, const Rev& R, int ell, int k, hipStream_t st);
// kap row c = (y_i)_c from the y history, c < ell + k, i <= k
void launch_rev_kap(const State& S, const Rev& R, int ell, int k, hipStream_t st);
// tv = E[:, i0 : i0 + ncols] (row c of kap)[i0 : i0 + ncols]
void launch_rev_tgemv(const State& S, const Rev& R, int c, int i0, int ncols, hipStream_t st);
// u = A tv - S_A^T zA, t = L tv - S_L^T zL, partials of (L wc) . (L tv)
void launch_rev_forward(const State& S, const Rev& R, const double* wc, hipStream_t st);
// dst = scale (A^T u + mu L^T t + rs[1] gx)   (scale null: 1)
void launch_rev_adjoint(const State& S, const Rev& R, const double* gx, const double* scale,
                        double* dst, hipStream_t st);
// partials of M[:, :ncols]^T v scaled by cs into gpart (ld dmax)
void launch_gemvt_mat(const State& S, const double* M, const double* v, int ncols, hipStream_t st);
// out (+)= sum_t h_t f(d1_t) f(d2_t) v_t, f(d) = *d (1 / *d where inv), f(null) = 1
struct LinTerm {
    const double* v;
    double h;
    const double* d1;
    const double* d2;
    int inv1;
};
struct LinComb {
    LinTerm t[4];
    int nt;
};
void launch_lincomb(const LinComb& lc, int64_t n, double* out, bool accumulate, hipStream_t st);
// out = base - M[:, :ncols] coef (no column scale), M with n rows
void launch_gemv_plain(const State& S, const double* M, const double* coef, int ncols,
                       const double* base, double* out, hipStream_t st);
void launch_fill(double* p, int64_t n, double v, hipStream_t st);
int launch_copy_scaled_W(const State& S, double* dst, hipStream_t st);  // 0 or -1
// x_k = W y into out in the caller's order of the unknowns
void launch_solution(const State& S, double* out, hipStream_t st);
// inverse of a caller's order (flag: 1 if it is not a permutation) and the
// relabelled column indices of A and L
int order_setup(const int32_t* order, int64_t n, int32_t* inv, int* flag, const Csr& A,
                int32_t* colA, const Csr& L, int32_t* colL, hipStream_t st);
// out[i] = in[perm[i]]
void launch_gather_perm(const double* in, const int32_t* perm, int64_t n, double* out,
                        hipStream_t st);
// columns [col0, col0 + ncols) of W scaled by cs into dst (n x ncols, column-major)
void launch_scaled_W_cols(const State& S, int col0, int ncols, double* dst, hipStream_t st);
// one workgroup reducing nb x s partial bins as a side append does (autotuning)
void launch_reduce_bins_probe(const double* bins, int nb, int s, double* out, hipStream_t st);
void launch_make_pattern(int16_t* pat, int64_t rows, int s, int zeta, uint64_t seed, int stream,
                         hipStream_t st);
int scatter_blocks(int64_t rows, int tiles_per_wave);
size_t scatter_lds_bytes(int s);
// SRTT: the blocks of 4096 of h rows (into *blocks) and the ranges of blocks
// (at most kSrttMaxChunks) whose sums are the partial bins
int srtt_chunks(int64_t h, int* blocks);
int srtt_pad(int s);
void launch_srtt_tables(const State& S, hipStream_t st);
// partial SRTT sketches of zA (m rows, S_A) and, if zL, zL (p rows, S_L) into the
// partial bins, scaled by sqrt(h/s) c_k (the append adds the chunks)
void launch_srtt(const State& S, const double* zA, const double* zL, hipStream_t st);
// the s frequencies an SRTT selects among h rows (host, draw order)
void srtt_rows_host(int64_t h, int s, uint64_t seed, int stream, int32_t* rows);
int scatter_ranges(int s);
size_t transpose_scratch_bytes(const Csr& M);
// scratch (device, scratch_bytes) serves the sort when large enough; else the
// scratch is allocated and freed around the sort
int transpose_csr(const Csr& M, int vdt, int32_t* rowptrT, int32_t* colT, void* valT,
                  void* scratch, size_t scratch_bytes, hipStream_t st);
int max_append_groups();

// plan from the host copies of the States (same order as SS)
int plan_build(Plan& P, const State* host, const State* dev, int np, const int* groups);
// one iteration step of every problem of the plan
void plan_gemv(const Plan& P, hipStream_t st);                 // x = W y
void plan_forward(const Plan& P, bool newcol, hipStream_t st); // u = A x - b, t = L x / A w, L w
// r = A^T u + mu L^T t into the new basis column (0), the refinement gradient
// (1) or column d of H W (2)
void plan_adjoint(const Plan& P, int dst_kind, hipStream_t st);
void plan_gradient(const Plan& P, bool to_rtmp, hipStream_t st);  // r from H W
void plan_scatter(const Plan& P, hipStream_t st);              // sketch bins of (u, t)
// with_hw (maintained gradient form): also add column d of H W from (u, t) in
// the compact side launch (when the plan fuses it there)
int plan_append(const Plan& P, bool scale_from_norm, bool with_hw, hipStream_t st);
// column d of H W from (u, t) = (A w, L w) in a launch of its own, for the
// problems whose H W column is not fused into the compact side launch
bool plan_has_hw_separate(const Plan& P);
void plan_hw_separate(const Plan& P, hipStream_t st);
void plan_gemvt(const Plan& P, hipStream_t st);                // W^T rtmp partials
void plan_mcol(const Plan& P, hipStream_t st);                 // new column of W^T H W
void plan_mrefine(const Plan& P, int steps, hipStream_t st);   // store it, refinement steps
// the stacked step alone, after the unsketched QR appends of GKS
void plan_stack_only(const Plan& P, hipStream_t st);

// ----- GKS (Alg. 1, sgks_gks.hip), one problem -----------------------------
// projection of the new basis column (the gradient, in W column d) on the
// orthonormal columns before it: pass 0, then pass 1 when the loss ratio
// ||V^T v|| / ||v|| is at least kGksTau; then the column scale and breakdown test
constexpr double kGksTau = 1e-10;
void gks_project(const State& S, const State* Sdev, hipStream_t st);
// rank-one appends of A v and L v (in u, t, unnormalised) to the QR factors of
// A V and L V, d_A gains q^T b; then the stacked step (plan_stack_only)
void gks_append(const State& S, const State* Sdev, hipStream_t st);
int gks_tall_blocks(int64_t rows, int* rows_per_block);
void plan_refine(const Plan& P, hipStream_t st);

}  // namespace sgks
