/*
 * sgks.h - C ABI of the sketched generalized Krylov subspace (sGKS) solver for
 * MI355X (gfx950).
 *
 * Problem (general-form Tikhonov, eq:tik of Palitta & Pasha):
 *     min_x ||A x - b||^2 + mu ||L x||^2,   A: m x n, L: p x n, mu > 0.
 * Method (Alg. 2, Sec. 3): x_k = W_k y_k where W_k = [W_0, w_1, ..., w_k] is NOT
 * orthonormalised; w_j = r_j / ||r_j|| with r_j the Tikhonov gradient
 * A^T(A x - b) + mu L^T L x (eq: gradient); y_k solves the sketched projected
 * problem (eq:projected_sketched_bis)
 *     min_y || [R_A; sqrt(mu) R_L] y - [Q_A^T S_A b; 0] ||
 * with Q_A R_A = S_A A W_k and Q_L R_L = S_L L W_k kept by rank-one column
 * appends (eq:updqr, eq:dA_update).  S_A (s x m) and S_L (s x p) are seeded
 * sparse-sign embeddings (Sec. 2.2 allows any oblivious embedding): column j
 * has zeta entries +-1/sqrt(zeta) in distinct rows drawn from SplitMix64,
 * key(stream, j) = mix64(seed + g (2j + stream + 1)), draw c = mix64(key + g (c+1)),
 * row = ((draw >> 32) * s) >> 32, sign = -1 if draw is odd; stream 0 is S_A,
 * stream 1 is S_L; a draw whose row repeats an earlier slot is skipped.
 * W_0 is an orthonormal basis of K_ell(A^T A, A^T b) (Sec. 2.1, ell = 3 in Sec. 4).
 *
 * Memory and ownership.  Every pointer named "device" is HIP device memory.
 * The operator arrays (CSR of A and L) and b are borrowed: the caller keeps
 * them alive and unmodified until sgks_destroy.  The context allocates its own
 * device workspace (transposes of A and L, the basis W, the small factors) in
 * sgks_create and frees it in sgks_destroy.  All work is enqueued on the
 * stream given in the options; calls documented as synchronising wait for it.
 * A context is not thread safe.
 *
 * Precision.  A, L and b are stored in SGKS_F32 or SGKS_F64.  The basis W,
 * the iterate x, the residual vectors and every accumulation are FP64; the
 * small factors (Q, R, the stacked factor G) and the projected solve are FP64.
 *
 * Return codes: 0 = OK; SGKS_BREAKDOWN (> 0, informational) = the expansion
 * stopped because ||r|| <= 1e-14 ||A^T b|| (invariant subspace) or because the
 * new column of [R_A; sqrt(mu) R_L] is numerically dependent on the previous
 * ones (kept below 1e-14 of its norm by the projections); the column is not
 * appended, the solution stays valid and fewer iterations were done.
 * Negative values are errors.
 */
#ifndef SGKS_H
#define SGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGKS_OK 0
#define SGKS_BREAKDOWN 1
#define SGKS_ERR_INVALID_ARG (-1)     /* null pointer, bad option value            */
#define SGKS_ERR_SHAPE (-2)           /* A.cols != L.cols, bad CSR sizes           */
#define SGKS_ERR_BAD_MU (-3)          /* mu <= 0 or not finite                     */
#define SGKS_ERR_SKETCH_SIZE (-4)     /* s < ell + max_iters, zeta > s, s > 16384,
                                         or s doubles beyond one workgroup's LDS     */
#define SGKS_ERR_CAPACITY (-5)        /* iterate would exceed ell + max_iters      */
#define SGKS_ERR_ZERO_RHS (-6)        /* b = 0 or A^T b = 0                        */
#define SGKS_ERR_NONFINITE (-7)       /* NaN/Inf in b or in a computed vector      */
#define SGKS_ERR_HIP (-8)             /* a HIP runtime call failed                 */
#define SGKS_ERR_DEVICE (-9)          /* device-side failure reported by a kernel  */
#define SGKS_ERR_INITIAL_SPACE (-10)  /* K_ell(A^T A, A^T b) has dimension < ell,
                                         or its sketched columns are dependent     */

/* storage type of the operator values and of b */
#define SGKS_F32 0
#define SGKS_F64 1

/* sketch kinds: the sparse-sign embedding; identities (sGKS_0 of Prop. 1,
 * meant for small checks: then s must equal max(m, p) and both sketches are
 * the identity on the first m (resp. p) rows); or the subsampled randomised
 * trigonometric transform of eq:sketching_trig, S = sqrt(h/s) D F E with F the
 * orthonormal DCT-II of length h (h = m for S_A, p for S_L), E Rademacher signs
 * (sign i = -1 if mix64(mix64(seed + g (stream + 3)) + g (i + 1)) is odd) and
 * D s distinct rows (draws mix64(mix64(seed + g (stream + 1)) + g (c + 1)),
 * row ((draw >> 32) h) >> 32, repeats skipped, outputs in draw order); needs
 * s <= min(m, p); zeta is not used.  Its s outputs are evaluated directly, h s
 * FP64 terms per image. */
#define SGKS_SKETCH_SPARSE_SIGN 0
#define SGKS_SKETCH_IDENTITY 1
#define SGKS_SKETCH_SRTT 2

/* Gradient forms (the same vector, two associations; eq: gradient).  DIRECT:
 * x = W y, u = A x - b, t = L x, r = A^T u + mu L^T t (two SpMVs and a GEMV per
 * expansion and per refinement step).  MAINTAINED: the context keeps
 * H W = (A^T A + mu L^T L) W column by column (the new column's A w and L w are
 * formed for its sketch anyway, one adjoint SpMV adds its H w) and evaluates
 * r = (H W) y - A^T b with one GEMV (A^T b is the first, unnormalised basis
 * column).  It saves an SpMV pass per expansion and both SpMVs of every
 * refinement step, for n * (ell + max_iters) more doubles of device memory. */
#define SGKS_GRADIENT_MAINTAINED 0
#define SGKS_GRADIENT_DIRECT 1

/* Methods.  SGKS (default): sketched GKS, Alg. 2 -- the basis W is not
 * reorthogonalised and the projected problem is the sketched one of
 * eq:projected_sketched_bis.  GKS: Alg. 1, the baseline sGKS is measured against
 * -- each new direction is projected on the orthonormal basis V by the projector
 * of eq:single_mgs, a second time when the loss ratio of eq:loss_criterion is at
 * least 1e-10, and normalised; the QR factors are those of the unsketched A V
 * (m x d) and L V (p x d), extended by eq:updqr with d_A = Q_A^T b
 * (eq:dA_update), and y solves eq:projected_withQR.  With GKS sketch_rows,
 * seed, zeta and sketch_mode are not used, refine_steps must be 0, and
 * sgks_backward and batches are not available (SGKS_ERR_INVALID_ARG). */
#define SGKS_METHOD_SGKS 0
#define SGKS_METHOD_GKS 1

/* CSR matrix with int32 indices; column indices sorted within each row.  All
 * three arrays are device pointers; val holds nnz values of the options'
 * value_dtype. */
typedef struct {
    int64_t rows, cols, nnz;
    const int32_t *rowptr;   /* rows + 1 entries, rowptr[0] = 0, rowptr[rows] = nnz */
    const int32_t *colind;   /* nnz entries in [0, cols)                            */
    const void *val;         /* nnz entries                                        */
} sgks_csr;

typedef struct {
    int32_t ell;             /* initial Krylov dimension, >= 1 (default 3)                    */
    int32_t max_iters;       /* capacity: at most ell + max_iters basis columns (default 200) */
    int32_t zeta;            /* nonzeros per sketch column: 2, 4, 8 or 16 (default 8)         */
    int32_t value_dtype;     /* SGKS_F32 or SGKS_F64 (default SGKS_F64)                       */
    int32_t refine_steps;    /* iterative-refinement steps after every projected solve (0)    */
    int32_t qr_passes;       /* 2 = project twice (CGS2, default), 1 = single projection       */
    int32_t sketch_mode;     /* SGKS_SKETCH_SPARSE_SIGN (default) or SGKS_SKETCH_IDENTITY     */
    int32_t lanes_A;         /* lanes per row for A-row SpMVs; 0 = choose from nnz/row          */
    int32_t lanes_At;        /* lanes per row for A^T rows; 0 = choose                          */
    int32_t append_groups;   /* QR append: 1 = compact (one launch, one workgroup per sketch
                                side; the second to finish also updates the stacked factor),
                                2..256 = chain of kernels on that many workgroups (slabs of
                                <= 64 sketch rows); 0 = choose by s * dmax                     */
    int32_t graph;           /* 0 = sgks_iterate / sgks_batch_iterate launch kernel by kernel
                                (default: the faster of the two on MI355X), 1 = replay captured
                                HIP graphs of 1 and 8 expansions.  Profiling
                                (sgks_profile_enable) always launches kernel by kernel          */
    int32_t gradient_form;   /* SGKS_GRADIENT_MAINTAINED (default) or SGKS_GRADIENT_DIRECT:
                                how the gradient r = A^T (A x - b) + mu L^T L x is evaluated
                                each expansion (see below)                                      */
    int32_t autotune;        /* 1 = time the lanes-per-row choices of the SpMVs and the tiles
                                per wave of the sketch scatter at create and keep the fastest
                                (cached per operator shape in the process); 0 = choose from
                                nnz/row and a fixed tile count (default)                        */
    int32_t method;          /* SGKS_METHOD_SGKS (default) or SGKS_METHOD_GKS (see above)      */
    int32_t keep_history;    /* 1 = record y after every projected solve, and hold the buffers
                                of sgks_backward_total (about 3 dmax^2 + n (max_iters + ell + 4)
                                + m + p + 2 s doubles more, dmax = ell + max_iters); needs method SGKS, the
                                maintained gradient form and refine_steps = 0, else
                                SGKS_ERR_INVALID_ARG at create; in a batch every problem
                                keeps its history.  0 = off (default)                          */
    const int32_t *order;    /* NULL (default) or device array of n int32: a permutation of the
                                unknowns the context works in internally, order[i] = the
                                caller's unknown at internal position i (e.g. pixels along a
                                space-filling curve, so that the rows of A and L gather nearby
                                entries).  The columns of A and L are relabelled once at create
                                (4 (nnz(A) + nnz(L)) more bytes of device memory; the values
                                stay the caller's); results are unchanged up to rounding order,
                                and every output (x_k, W) and input (grad_x) is in the caller's
                                order.  SGKS_ERR_INVALID_ARG at create if it is not a
                                permutation of [0, n).  Borrowed until sgks_destroy.          */
    void *stream;            /* hipStream_t the work is enqueued on (NULL = default stream)   */
    void *workspace;         /* NULL: the context allocates its device memory (one hipMalloc in
                                sgks_create, freed by sgks_destroy).  Else device memory of
                                workspace_bytes >= sgks_workspace_bytes(...), 256-byte aligned,
                                owned by the caller and used for every array of the context
                                (no device allocation in sgks_create or afterwards, except the
                                temporary of sgks_copy_state(W)); keep it alive until
                                sgks_destroy.  sgks_batch_create takes one workspace for the
                                whole batch (sgks_batch_workspace_bytes).                      */
    size_t workspace_bytes;
} sgks_options;

typedef struct sgks_ctx sgks_ctx;

/* Fill *opt with the defaults listed above. */
void sgks_default_options(sgks_options *opt);

/* Device bytes a context with these arguments uses (host only, no device
 * work); 0 if the arguments are invalid.  Independent of the values, the
 * seed, the stream and the autotuner's choices. */
size_t sgks_workspace_bytes(const sgks_csr *A, const sgks_csr *L, int32_t sketch_rows,
                            const sgks_options *opt);

/* Check the arguments of sgks_create without touching the device (host only).
 * Returns the code sgks_create would return for an argument error, or 0. */
int sgks_validate(const sgks_csr *A, const sgks_csr *L, const void *b, double mu,
                  int32_t sketch_rows, const sgks_options *opt);

/* Set up a solve (Alg. 2 before its loop): build A^T and L^T, the sketch of
 * b, the initial basis W_0 (K_ell(A^T A, A^T b), orthonormal), the QR factors
 * of S_A A W_0 and S_L L W_0 and y_0.  b: device, m values of value_dtype.
 * sketch_rows = s (s_A = s_L = s); seed selects the sketches.
 * Synchronises the stream.  On success *out receives a new context. */
int sgks_create(const sgks_csr *A, const sgks_csr *L, const void *b, double mu,
                int32_t sketch_rows, uint64_t seed, const sgks_options *opt,
                sgks_ctx **out);

/* Run k more expansions (the loop body of Alg. 2): x = W y; r = gradient;
 * append r/||r||; sketch and QR-append the new column; solve for y;
 * refine_steps refinement steps.  Asynchronous; resumable: iterate(a) then
 * iterate(b) equals iterate(a + b).  Returns SGKS_ERR_CAPACITY if the
 * basis would exceed ell + max_iters columns. */
int sgks_iterate(sgks_ctx *ctx, int32_t k);

/* The iterate x_k = W_k y_k that Alg. 2 returns (its last line, with the basis
 * of the expansions done so far): n FP64 values into the device buffer x_dev
 * (caller-owned, n doubles).  Asynchronous on the context's stream; returns
 * SGKS_ERR_INVALID_ARG for a null pointer. */
int sgks_solution(sgks_ctx *ctx, double *x_dev);

/* Residual norms at the current iterate x = W y.  true_norm is the square root
 * of the Tikhonov functional of eq:tik, sqrt(||A x - b||^2 + mu ||L x||^2),
 * from one pass of A and L over x.  sketched_norm is the square root of the
 * sketched functional of eq:tik_new_sketched, sqrt(||S_A(A x - b)||^2 +
 * mu ||S_L L x||^2), computed in O(d^2) from the small factors alone
 * (S_A A W = Q_A R_A, S_L L W = Q_L R_L, d_A = Q_A^T S_A b, eq:updqr and
 * eq:dA_update): ||R_A y - d_A||^2 + ||S_A b||^2 - ||d_A||^2 + mu ||R_L y||^2.
 * Host doubles; either pointer may be NULL.  Synchronises the stream. */
int sgks_residual_norm(sgks_ctx *ctx, double *true_norm, double *sketched_norm);

/* Synchronising.  *iters_done = expansions done so far; returns the status
 * word (0, SGKS_BREAKDOWN or a negative device error). */
int sgks_status(sgks_ctx *ctx, int32_t *iters_done);

/* Frozen-basis adjoint of the final projected solve (not in the paper): with
 * W, Q_A, R_A, R_L held fixed, x = W H^{-1} R_A^T Q_A^T S_A b where
 * H = R_A^T R_A + mu R_L^T R_L.  Given grad_x (device, n FP64) writes
 * grad_b = S_A^T Q_A R_A z with z = H^{-1} W^T grad_x (device, m FP64) and
 * *grad_mu = -(R_L z).(R_L y) (host).  Synchronising.  Returns
 * SGKS_ERR_INVALID_ARG, before any device work, for a context created with
 * refine_steps > 0: its x is the refined solve, whose derivative this adjoint
 * is not. */
int sgks_backward(sgks_ctx *ctx, const double *grad_x, double *grad_b, double *grad_mu);

/* Total-derivative adjoint (not in the paper): the gradient of loss(x_k) with
 * respect to b and mu through the whole sGKS map of Alg. 2 -- the initial
 * Krylov basis K_ell(A^T A, A^T b) (Sec. 2.1), every gradient column of
 * eq: gradient appended since, the sketched products S_A A W and S_L L W
 * (eq:updqr) and every projected solve (eq:projected_sketched_bis, with
 * d_A = Q_A^T S_A b of eq:dA_update) -- in exact arithmetic, where the solve
 * with d columns is y = N^{-1} (S_A A W)^T S_A b, N = (S_A A W)^T S_A A W +
 * mu (S_L L W)^T S_L L W.  Reverse sweep over the expansions done so far
 * (a breakdown ends them early), with W, H W and the factors resident on the
 * device: per basis column one product of A, A^T, L and L^T, two sketch
 * transposes and two dense passes over at most d stored n-vectors.  Given
 * grad_x (device, n FP64, the caller's order) writes grad_b (device, m FP64)
 * and *grad_mu (host, may be NULL).  Needs a context created with
 * keep_history = 1 (else SGKS_ERR_INVALID_ARG, before any device work).
 * Accuracy: every solve is inverted through N = G^T G, so rounding errors grow
 * like eps kappa(G)^2 (G the final stacked factor [R_A; sqrt(mu) R_L] = U G,
 * whose leading blocks are the G_j); *err_est (host, may be NULL) receives
 * d eps kappa(G)^2, kappa from power iterations on G and G^{-1}, a pessimistic
 * bound on the relative rounding error.  The basis of Alg. 2 is never
 * reorthogonalised, so kappa grows with k; where the estimate is large (the
 * Python binding warns above 1e-3) the gradient is dominated by rounding; the
 * frozen adjoint (sgks_backward) loses accuracy far later.  Returns the
 * context's negative device status if it has one.
 * Synchronising; the context can iterate further afterwards. */
int sgks_backward_total(sgks_ctx *ctx, const double *grad_x, double *grad_b, double *grad_mu,
                        double *err_est);

/* Copy one piece of the solver state to host memory (synchronising), for
 * checks.  which: 0 W (n x d, column-major, columns scaled to unit norm),
 * 1 y (d), 2 Q_A (s x d; m x d with GKS), 3 R_A (d x d), 4 Q_L (s x d; p x d
 * with GKS), 5 R_L (d x d), 6 d_A (d), 7 G (d x d, R factor of
 * [R_A; sqrt(mu) R_L]), 8 S_A b (s; not with GKS).
 * count = number of doubles dst can take; returns the number written (>= 0)
 * or an error code. */
int64_t sgks_copy_state(sgks_ctx *ctx, int32_t which, double *dst, int64_t count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): sgks_copy_state
 * without its device temporary.  which, dst, count and the return value are as
 * for sgks_copy_state (same values, bit for bit).  For W (which = 0) the scaled
 * columns are staged through a static device array of
 * SGKS_NOALLOC_SCRATCH_BYTES held by the library on each GPU it runs on (until
 * the process ends), as many columns at a time as fit; returns
 * SGKS_ERR_CAPACITY if one column (8 n bytes) exceeds it.  The array is shared
 * by every call on that GPU: calls that overlap on one GPU (several threads or
 * contexts at once) race.  Allocates nothing; synchronises the stream. */
#define SGKS_NOALLOC_SCRATCH_BYTES (16u << 20)
int64_t sgks_copy_state_noalloc(sgks_ctx *ctx, int32_t which, double *dst, int64_t count);

/* Per-phase device timing (the per-component breakdown of Sec. 4): while
 * enabled, every kernel launch of sgks_iterate / sgks_solution is issued with
 * a pair of HIP events bound to that kernel, which hold the begin and end of
 * its execution (the dispatch gap before it is not counted, as in a kernel
 * trace); a phase's time is the sum over its kernels and its count the number
 * of kernels launched.  On a stream under capture the launches are recorded
 * without events and are not counted.  Phases: 0 x = W y, 1 forward products
 * (A x - b, L x), 2 adjoint products (A^T u + mu L^T t), 3 SpMV of the new
 * column (A w, L w), 4 QR appends + projected solve, 5 W^T v (refinement),
 * 6 refinement step, 7 sketch scatter of the new column.  sgks_profile_read
 * synchronises, writes the summed milliseconds and launch counts of the
 * SGKS_PHASES phases (either array may be NULL) and resets them. */
#define SGKS_PHASES 8
int sgks_profile_enable(sgks_ctx *ctx, int32_t on);
int sgks_profile_read(sgks_ctx *ctx, double *ms, int64_t *launches);

/* Current number of basis columns d (host-side view, no synchronisation). */
int32_t sgks_dim(const sgks_ctx *ctx);

/* Launch shapes in use (chosen at create, by the autotuner when enabled):
 * out[0], out[1] lanes of a wavefront per CSR row for the rows of A and of L
 * (forward products), out[2] for the rows of A^T and L^T (adjoint products),
 * powers of two in [1, 64] (64 / lanes rows share one wavefront); out[3],
 * out[4] workgroups of the sketch scatter over the m (S_A) and p (S_L)
 * entries; out[5] append groups (1 = compact append). */
int sgks_get_tuning(const sgks_ctx *ctx, int32_t out[6]);

/* Releases the context and its device memory (synchronises its stream).  A
 * context obtained from sgks_batch_get belongs to its batch: destroying it
 * here does nothing. */
void sgks_destroy(sgks_ctx *ctx);
const char *sgks_strerror(int code);

/* ------------------------------------------------------------------------
 * Batched solves (an extension, not in the paper): many independent problems
 * of uneven sizes advance together.  Each kernel launch of an expansion covers
 * every problem of the batch (its workgroups are split among the problems by
 * a block table), so the latency-bound small steps of different problems
 * overlap and the bulk steps of small problems fill the GPU together.
 * ------------------------------------------------------------------------ */

#define SGKS_MAX_BATCH 64

/* One problem of a batch: operators, right-hand side (device, value_dtype of
 * the options), mu > 0, sketch size s, seed and order of unknowns, as the
 * arguments and the order option of sgks_create (the options' order is not
 * used by batches). */
typedef struct {
    sgks_csr A, L;
    const void *b;
    double mu;
    int32_t sketch_rows;
    uint64_t seed;
    const int32_t *order;    /* the problem's internal order of unknowns, as sgks_options.order */
} sgks_problem;

typedef struct sgks_batch sgks_batch;

/* Device bytes of a batch of these problems and options (host only, no device
 * work): the contexts' arenas, each 256-byte aligned, then the device array of
 * the problems' States.  0 if an argument is invalid. */
size_t sgks_batch_workspace_bytes(int32_t count, const sgks_problem *problems,
                                  const sgks_options *opt);

/* Set up count (1..SGKS_MAX_BATCH) problems that share opt (value dtype,
 * zeta, ell, max_iters, refinement, QR passes, sketch kind, stream, graph and
 * autotune choices; lanes and append_groups must be 0).  Each problem is set
 * up as by sgks_create; the first failing problem's code is returned and
 * nothing is kept.  Device memory: with opt->workspace NULL the batch
 * allocates each context's arena and its States array; otherwise
 * opt->workspace (256-byte aligned, opt->workspace_bytes >=
 * sgks_batch_workspace_bytes) holds all of them, carved in problem order, and
 * nothing is allocated (SGKS_ERR_INVALID_ARG if it is too small or
 * misaligned).  Synchronises the stream. */
int sgks_batch_create(int32_t count, const sgks_problem *problems, const sgks_options *opt,
                      sgks_batch **out);

/* k more expansions of every problem (as sgks_iterate on each, with the same
 * results bit for bit).  A problem that stopped (breakdown) stays as it is
 * while the others go on.  Asynchronous; SGKS_ERR_CAPACITY if any problem
 * would exceed ell + max_iters columns. */
int sgks_batch_iterate(sgks_batch *batch, int32_t k);

/* Problem i of the batch as a context (borrowed, valid until
 * sgks_batch_destroy): sgks_solution, sgks_residual_norm, sgks_status,
 * sgks_backward, sgks_copy_state and sgks_iterate apply to it.  NULL if i is
 * out of range. */
sgks_ctx *sgks_batch_get(sgks_batch *batch, int32_t i);

/* Number of problems; 0 for NULL. */
int32_t sgks_batch_count(const sgks_batch *batch);

/* Per-phase timing of sgks_batch_iterate, as sgks_profile_enable / _read
 * (one event pair per kernel launch, each launch covering every problem). */
int sgks_batch_profile_enable(sgks_batch *batch, int32_t on);
int sgks_batch_profile_read(sgks_batch *batch, double *ms, int64_t *launches);

void sgks_batch_destroy(sgks_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* SGKS_H */
