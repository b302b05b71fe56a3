// Host runtime of the sGKS library: argument validation, workspace planning,
// set-up (Alg. 2 before its loop) and the enqueueing of the iteration
// kernels.  Exposes the C ABI declared in include/sgks.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "sgks.h"
#include "sgks_internal.h"

using sgks::Csr;
using sgks::State;

thread_local sgks::LaunchTimer* sgks::tl_launch_timer = nullptr;

// Staging memory of sgks_copy_state_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes its name to a
// kernel or a copy; it uses the device address hipGetSymbolAddress returns for
// the current device (kept per device below).
static __device__ __align__(256) double scratch[SGKS_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device
// with that device current.
int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SGKS_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SGKS_ERR_HIP;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SGKS_OK;
}

}  // namespace

namespace {

// Per-phase kernel timing: every launch made inside a phase gets an event
// pair bound to the kernel itself (sgks::LaunchTimer), so a phase's time is
// the summed execution time of its kernels and its count their number.
struct Profiler final : sgks::LaunchTimer {
    bool on = false;
    int phase = -1;                    // phase of the launches being enqueued
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> events;    // pairs (begin, end)
    std::vector<int> pair_phase;
    size_t pairs_used = 0;

    ~Profiler() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
    bool pair(hipEvent_t* begin, hipEvent_t* end) override {
        if (!on || phase < 0) return false;
        // a stream under capture records the launch untimed
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
            return false;
        if (pairs_used >= pair_phase.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return false;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return false;
            }
            events.push_back(a);
            events.push_back(b);
            pair_phase.push_back(0);
        }
        const size_t i = pairs_used++;
        pair_phase[i] = phase;
        *begin = events[2 * i];
        *end = events[2 * i + 1];
        return true;
    }
    int read(double* ms, int64_t* launches) {
        if (hipStreamSynchronize(st) != hipSuccess) return SGKS_ERR_HIP;
        double acc[SGKS_PHASES] = {0};
        int64_t cnt[SGKS_PHASES] = {0};
        for (size_t i = 0; i < pairs_used; ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, events[2 * i], events[2 * i + 1]) != hipSuccess)
                return SGKS_ERR_HIP;
            acc[pair_phase[i]] += t;
            cnt[pair_phase[i]] += 1;
        }
        pairs_used = 0;
        for (int p = 0; p < SGKS_PHASES; ++p) {
            if (ms) ms[p] = acc[p];
            if (launches) launches[p] = cnt[p];
        }
        return SGKS_OK;
    }
};

// Marks the launches enqueued in its scope as those of one phase when
// profiling (installs the profiler as this thread's launch timer).
struct Phase {
    Profiler* pr;
    sgks::LaunchTimer* prev = nullptr;
    Phase(Profiler* p, int phase) : pr(p && p->on ? p : nullptr) {
        if (!pr) return;
        pr->phase = phase;
        prev = sgks::tl_launch_timer;
        sgks::tl_launch_timer = pr;
    }
    ~Phase() {
        if (!pr) return;
        pr->phase = -1;
        sgks::tl_launch_timer = prev;
    }
};

// Refinement step of every problem of the plan: the gradient r(y) into rtmp,
// W^T r, y update (heavy ball).
// The refinement steps after an append (Sec. 3.1: the unsketched projected
// normal equations, preconditioned by the sketched factor).  Maintained form:
// the new column of W^T H W from the kept H W column, then all the steps on
// the d x d matrix in one launch (`steps` = 0 only stores the column).  Direct
// form: per step x = W y, u = A x - b, t = L x, r = A^T u + mu L^T t, W^T r and
// the heavy-ball update.
void enqueue_refinement(const sgks::Plan& P, int steps, Profiler* pr, hipStream_t st) {
    if (P.gradient_form == SGKS_GRADIENT_MAINTAINED) {
        { Phase ph(pr, 5); sgks::plan_mcol(P, st); }
        { Phase ph(pr, 6); sgks::plan_mrefine(P, steps, st); }
        return;
    }
    for (int r = 0; r < steps; ++r) {
        { Phase ph(pr, 0); sgks::plan_gemv(P, st); }
        { Phase ph(pr, 1); sgks::plan_forward(P, false, st); }
        { Phase ph(pr, 2); sgks::plan_adjoint(P, 1, st); }
        { Phase ph(pr, 5); sgks::plan_gemvt(P, st); }
        { Phase ph(pr, 6); sgks::plan_refine(P, st); }
    }
}

// One expansion of every problem of the plan (the loop body of Alg. 2): the
// gradient r at x = W y into the next basis column, A w and L w of that
// column, their sketches, the QR appends and the projected solve; then the
// refinement steps.  Maintained form: r = (H W) y - A^T b from the kept
// columns of H W = (A^T A + mu L^T L) W, whose new column is A^T (A w) +
// mu L^T (L w) from the images the sketch needs anyway.  Direct form:
// x = W y, u = A x - b, t = L x, r = A^T u + mu L^T t.
// A second stream of the caller's device (default priority) that takes the
// H W column's adjoint products while the caller's stream runs the sketch
// scatter and the QR appends of the same expansion: the two read the same
// images (A w, L w) and write disjoint memory, and the appends are latency
// bound (a few workgroups), so the bandwidth-bound adjoint fills the GPU
// beside them.  The caller's stream waits for it before the expansion ends.
struct SideStream {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    ~SideStream() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
    }
    bool ready() {
        if (side) return true;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) {
            side = nullptr;
            return false;
        }
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess)
            return false;
        return true;
    }
};

// One expansion of GKS (Alg. 1; one problem): the gradient into W column d,
// its projection on the orthonormal columns before it (the loss-ratio test of
// the second pass, the column scale), A v and L v, the H W column, the
// unsketched QR appends and the stacked step.
int enqueue_gks_iteration(const sgks::Plan& P, Profiler* pr, hipStream_t st) {
    const bool maintained = P.gradient_form == SGKS_GRADIENT_MAINTAINED;
    if (maintained) {
        Phase ph(pr, 0);
        sgks::plan_gradient(P, false, st);
    } else {
        { Phase ph(pr, 0); sgks::plan_gemv(P, st); }
        { Phase ph(pr, 1); sgks::plan_forward(P, false, st); }
        { Phase ph(pr, 2); sgks::plan_adjoint(P, 0, st); }
    }
    { Phase ph(pr, 5); sgks::gks_project(*P.host, P.SS, st); }
    { Phase ph(pr, 3); sgks::plan_forward(P, true, st); }
    if (maintained) {
        Phase ph(pr, 2);
        sgks::plan_adjoint(P, 2, st);   // column d of H W
    }
    {
        Phase ph(pr, 4);
        sgks::gks_append(*P.host, P.SS, st);
        sgks::plan_stack_only(P, st);
    }
    return hipGetLastError() == hipSuccess ? SGKS_OK : SGKS_ERR_HIP;
}

int enqueue_iteration(const sgks::Plan& P, int refine_steps, Profiler* pr, hipStream_t st,
                      SideStream* ss = nullptr) {
    if (P.method == SGKS_METHOD_GKS) return enqueue_gks_iteration(P, pr, st);
    const bool maintained = P.gradient_form == SGKS_GRADIENT_MAINTAINED;
    if (maintained) {
        Phase ph(pr, 0);
        sgks::plan_gradient(P, false, st);
    } else {
        { Phase ph(pr, 0); sgks::plan_gemv(P, st); }
        { Phase ph(pr, 1); sgks::plan_forward(P, false, st); }
        { Phase ph(pr, 2); sgks::plan_adjoint(P, 0, st); }
    }
    { Phase ph(pr, 3); sgks::plan_forward(P, true, st); }
    // maintained form: column d of H W from (A w, L w), in the compact append's
    // launch (beside the side appends, its column index recorded by the SpMV
    // above) or in a launch of its own, on the side stream when there is one
    const bool hw_sep = maintained && sgks::plan_has_hw_separate(P);
    const bool fork = hw_sep && ss;
    if (fork) {
        if (hipEventRecord(ss->fork, st) != hipSuccess ||
            hipStreamWaitEvent(ss->side, ss->fork, 0) != hipSuccess)
            return SGKS_ERR_HIP;
        { Phase ph(pr, 2); sgks::plan_hw_separate(P, ss->side); }
        if (hipEventRecord(ss->join, ss->side) != hipSuccess) return SGKS_ERR_HIP;
    } else if (hw_sep) {
        Phase ph(pr, 2);
        sgks::plan_hw_separate(P, st);
    }
    { Phase ph(pr, 7); sgks::plan_scatter(P, st); }
    {
        Phase ph(pr, 4);
        if (sgks::plan_append(P, true, maintained, st)) return SGKS_ERR_HIP;
    }
    if (fork && hipStreamWaitEvent(st, ss->join, 0) != hipSuccess) return SGKS_ERR_HIP;
    if (refine_steps > 0) enqueue_refinement(P, refine_steps, pr, st);
    // y of this solve, for the total-derivative adjoint
    if (P.record_y) sgks::launch_record_y(P.SS, P.np, st);
    return SGKS_OK;
}

// Captured HIP graphs of the expansion: one of a single expansion and one of
// kGraphChunk expansions.  The kernels take only device-resident state (the
// basis size d is read on the device), so one graph serves every expansion.
constexpr int kGraphChunk = 8;

// default 64-entry tiles per wave of the sketch scatter: fewer tiles give more
// workgroups (the scatter is bound by each compute unit's LDS atomics) but more
// partial bins for the append to reduce; 4 balances the two at the 2D
// deblurring sizes (m = 65,536, p = 131,072, s = 400)
constexpr int kScatterTilesPerWave = 4;

struct GraphCache {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};

    ~GraphCache() {
        for (hipGraphExec_t e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
    }
    int capture(const sgks::Plan& P, int refine_steps, int iters, hipGraphExec_t* out) {
        if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
            return SGKS_ERR_HIP;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) != hipSuccess)
            return SGKS_ERR_HIP;
        int rc = SGKS_OK;
        for (int i = 0; i < iters && rc == SGKS_OK; ++i)
            rc = enqueue_iteration(P, refine_steps, nullptr, cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cap, &g);
        if (e != hipSuccess || rc != SGKS_OK || !g) {
            if (g) (void)hipGraphDestroy(g);
            return SGKS_ERR_HIP;
        }
        const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        return ei == hipSuccess ? SGKS_OK : SGKS_ERR_HIP;
    }
};

// k expansions of every problem of the plan: graph replays, or kernel by
// kernel while profiling or when graphs are off.
int run_iterations(const sgks::Plan& P, int refine_steps, Profiler* pr, GraphCache* gc,
                   bool use_graph, hipStream_t st, int k, SideStream* ss) {
    if (!use_graph || (pr && pr->on)) {
        // no second stream while the caller's stream is being captured
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cst) != hipSuccess) return SGKS_ERR_HIP;
        SideStream* use = nullptr;
        if (cst == hipStreamCaptureStatusNone && sgks::plan_has_hw_separate(P) && ss &&
            ss->ready())
            use = ss;
        for (int it = 0; it < k; ++it) {
            const int rc = enqueue_iteration(P, refine_steps, pr, st, use);
            if (rc) return rc;
        }
        return hipGetLastError() == hipSuccess ? SGKS_OK : SGKS_ERR_HIP;
    }
    while (k > 0) {
        const int which = k >= kGraphChunk ? 1 : 0;
        if (!gc->exec[which]) {
            const int rc = gc->capture(P, refine_steps, which ? kGraphChunk : 1, &gc->exec[which]);
            if (rc) return rc;
        }
        if (hipGraphLaunch(gc->exec[which], st) != hipSuccess) return SGKS_ERR_HIP;
        k -= which ? kGraphChunk : 1;
    }
    return SGKS_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the lanes per CSR row: every power of two is timed on the
// operator itself (HIP events, best of a few launches); choices are cached
// per operator shape for the life of the process.
// ---------------------------------------------------------------------------

std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int64_t, int64_t, int64_t, int>, int> g_tune;

template <typename F>
float time_launches(hipStream_t st, F&& launch, int reps) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return INFINITY;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return INFINITY;
    }
    launch();   // warm-up
    float best = INFINITY;
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(a, st) != hipSuccess) break;
        launch();
        if (hipEventRecord(b, st) != hipSuccess) break;
        float ms = INFINITY;
        if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess &&
            ms < best)
            best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

// kind: 0 rows of A (forward), 1 rows of L (forward), 2 rows of A^T and L^T (adjoint)
int tune_one(const State& S, int kind, hipStream_t st) {
    const Csr& M = kind == 0 ? S.A : kind == 1 ? S.L : S.At;
    const auto key = std::make_tuple(kind, M.rows, M.cols, M.nnz,
                                     kind == 2 ? S.Lt.nnz : (int64_t)0, S.vdt);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    int best = M.lanes;
    float tbest = INFINITY;
    for (int lanes = 1; lanes <= 64; lanes *= 2) {
        State T = S;
        float ms;
        if (kind == 2) {
            T.At.lanes = lanes;
            ms = time_launches(st, [&] {
                sgks::launch_adjoint(T, S.u, S.t, true, S.mu, S.rtmp, S.norm_part, st);
            }, 5);
        } else {
            T.A = kind == 0 ? S.A : S.L;
            T.A.lanes = lanes;
            double* out = kind == 0 ? S.u : S.t;
            ms = time_launches(st, [&] {
                sgks::launch_forward(T, S.x, nullptr, out, nullptr, false, nullptr, nullptr, st);
            }, 5);
        }
        if (ms < tbest) {
            tbest = ms;
            best = lanes;
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

// tiles per wave of the sketch scatter: each count is timed as the scatter of
// both images plus the reduction of its partial bins as the append does it (one
// workgroup per side, both sides at once: the side with more partial bins sets
// the time).  Fewer, fuller workgroups leave fewer partial bins to reduce.
int tune_scatter(const State& S, hipStream_t st) {
    const auto key = std::make_tuple(3, S.m, S.p, (int64_t)S.s, (int64_t)S.zeta, S.vdt);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    int best = kScatterTilesPerWave;
    float tbest = INFINITY;
    for (int tpw = 1; tpw <= 16; tpw *= 2) {
        State T = S;
        T.nbA = sgks::scatter_blocks(S.m, tpw);
        T.nbL = sgks::scatter_blocks(S.p, tpw);
        const float ms = time_launches(st, [&] {
            sgks::launch_scatter(T, S.u, S.t, st);
            if (T.nbA >= T.nbL)
                sgks::launch_reduce_bins_probe(T.binA, T.nbA, S.s, S.cb, st);
            else
                sgks::launch_reduce_bins_probe(T.binL, T.nbL, S.s, S.cb, st);
        }, 5);
        if (ms < tbest) {
            tbest = ms;
            best = tpw;
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

}  // namespace

struct sgks_ctx {
    State S;
    State* Sdev;         // device copy of S (the kernels of the iteration read it)
    sgks::Plan plan;     // the iteration as a batch of one
    sgks_options opt;
    hipStream_t st;
    int device = 0;      // the device current at sgks_create
    int d_host;          // basis columns expected on the device (no breakdown)
    int groups;          // workgroups of the append kernels
    bool borrowed = false;   // owned by a batch
    GraphCache graphs;
    SideStream side;
    std::vector<void*> allocs;
    double* upart;       // partial sums of ||A x - b||^2
    double* tpart;       // partial sums of ||L x||^2
    int nbF_A, nbF_L;
    double* coefbuf;     // dmax scratch
    double* sbuf;        // s scratch
    double* init_norms;  // copy of the scalars after the initial basis (checked at the end of create)
    int16_t* patA = nullptr;
    int16_t* patL = nullptr;
    int32_t* colA2 = nullptr;   // columns of A and L in the internal order of the unknowns
    int32_t* colL2 = nullptr;
    int* order_flag = nullptr;  // set on the device if the order is not a permutation
    std::vector<int32_t> srtt_rows;   // the SRTT frequencies of both sides (host copy)
    void* sort_scratch = nullptr;   // transpose sort scratch when W (and HW) are too small
    size_t sort_bytes = 0;
    int32_t* At_rowptr;
    int32_t* At_col;
    void* At_val;
    int32_t* Lt_rowptr;
    int32_t* Lt_col;
    void* Lt_val;
    Profiler prof;
    sgks::Rev rv{};      // buffers of the total-derivative adjoint (keep_history)
};

namespace {

bool pow2_lanes(int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8 || v == 16 || v == 32 || v == 64; }

// lanes per CSR row: the largest power of two up to a sixth of the mean row
// length (measured on gfx950: 8 lanes for ~80 nonzeros per row, 32 for ~230)
int choose_lanes(int64_t nnz, int64_t rows) {
    if (rows <= 0) return 1;
    const double avg = (double)nnz / (double)rows;
    int v = 1;
    while (v < 64 && 2.0 * v <= avg / 6.0) v *= 2;
    return v;
}

// One device allocation carved into 256-byte aligned pieces: fewer runtime
// allocations at create, and the small state shares a few large pages.
struct Arena {
    struct Req {
        void** p;
        size_t off;
    };
    std::vector<Req> reqs;
    size_t total = 0;
    template <typename P>
    void add(P** p, size_t bytes) {
        reqs.push_back({(void**)p, total});
        total += (bytes + 255) / 256 * 256;
        if (bytes == 0) total += 256;
    }
    void place(char* base) {
        for (const Req& r : reqs) *r.p = base + r.off;
    }
    hipError_t commit(sgks_ctx* c) {
        char* base = nullptr;
        hipError_t e = hipMalloc((void**)&base, total);
        if (e != hipSuccess) return e;
        c->allocs.push_back(base);
        for (const Req& r : reqs) *r.p = base + r.off;
        return hipSuccess;
    }
};

int check_csr(const sgks_csr* M) {
    if (!M) return SGKS_ERR_INVALID_ARG;
    if (M->rows < 0 || M->cols <= 0 || M->nnz < 0) return SGKS_ERR_SHAPE;
    if (M->rows >= (int64_t(1) << 31) || M->cols >= (int64_t(1) << 31) ||
        M->nnz >= (int64_t(1) << 31))
        return SGKS_ERR_SHAPE;
    if (!M->rowptr) return SGKS_ERR_INVALID_ARG;
    if (M->nnz > 0 && (!M->colind || !M->val)) return SGKS_ERR_INVALID_ARG;
    return 0;
}

int sync_status(sgks_ctx* c) {
    int st = 0;
    if (hipMemcpyAsync(&st, c->S.status, sizeof(int), hipMemcpyDeviceToHost, c->st) != hipSuccess)
        return SGKS_ERR_HIP;
    if (hipStreamSynchronize(c->st) != hipSuccess) return SGKS_ERR_HIP;
    return st;
}

// partial sums of ||r||^2: one per workgroup of the kernel that forms r
int norm_parts(const State& T) {
    return T.gradient_form == SGKS_GRADIENT_MAINTAINED ? sgks::gradient_blocks(T)
                                                       : sgks::adjoint_blocks(T);
}

// Shapes and launch choices of a context from its arguments (validated
// already); host only, no device memory.
int plan_context(sgks_ctx* c, const sgks_csr* A, const sgks_csr* L, double mu, int32_t s,
                 uint64_t seed) {
    c->st = (hipStream_t)c->opt.stream;
    State& S = c->S;
    memset(&S, 0, sizeof(S));
    S.m = A->rows;
    S.n = A->cols;
    S.p = L->rows;
    S.method = c->opt.method;
    const bool gks = S.method == SGKS_METHOD_GKS;
    if (gks) s = 1;   // no sketch: the small sketch-sized arrays shrink to one row
    S.s = s;
    S.dmax = c->opt.ell + c->opt.max_iters;
    S.zeta = c->opt.zeta;
    S.passes = c->opt.qr_passes;
    S.sketch_mode = gks ? sgks::kSketchNone : c->opt.sketch_mode;
    S.vdt = c->opt.value_dtype;
    S.gradient_form = c->opt.gradient_form;
    S.seed = seed;
    S.mu = mu;
    S.sqrt_mu = sqrt(mu);
    const int dmax = S.dmax;

    S.A = Csr{A->rows, A->cols, A->nnz, A->rowptr, A->colind, A->val,
              c->opt.lanes_A ? c->opt.lanes_A : choose_lanes(A->nnz, A->rows)};
    S.L = Csr{L->rows, L->cols, L->nnz, L->rowptr, L->colind, L->val,
              choose_lanes(L->nnz, L->rows)};

    // transposes of A and L (explicit CSR, n rows): shapes now, arrays below
    S.At = Csr{S.n, S.m, S.A.nnz, nullptr, nullptr, nullptr,
               c->opt.lanes_At ? c->opt.lanes_At : choose_lanes(S.A.nnz, S.n)};
    S.Lt = Csr{S.n, S.p, S.L.nnz, nullptr, nullptr, nullptr, choose_lanes(S.L.nnz, S.n)};

    // scatter workgroups: kScatterTilesPerWave 64-entry tiles per wave (the
    // autotuner may choose another count; the partial bins are sized for one);
    // SRTT: blocks of 4096 rows in at most 128 ranges (the partial bins)
    if (S.sketch_mode == SGKS_SKETCH_SRTT) {
        S.nbA = sgks::srtt_chunks(S.m, &S.srA);
        S.nbL = sgks::srtt_chunks(S.p, &S.srL);
    } else {
        S.nbA = sgks::scatter_blocks(S.m, kScatterTilesPerWave);
        S.nbL = sgks::scatter_blocks(S.p, kScatterTilesPerWave);
    }
    S.n_norm_part = norm_parts(S);
    int nbFA = 0;
    const int nbF = sgks::forward_blocks(S, true, &nbFA);
    c->nbF_A = nbFA;
    c->nbF_L = nbF - nbFA;
    // W^T v partials: at most 512 blocks, rows per block a multiple of 64
    {
        int64_t rpb = (S.n + 511) / 512;
        rpb = ((rpb + 63) / 64) * 64;
        if (rpb < 128) rpb = 128;
        if (rpb > 4096) rpb = 4096;   // staged in LDS (32 KiB)
        S.gt_rows = (int)rpb;
        S.ngt = (int)((S.n + rpb - 1) / rpb);
    }
    if (gks) {
        S.ntA = sgks::gks_tall_blocks(S.m, &S.trA);
        S.ntL = sgks::gks_tall_blocks(S.p, &S.trL);
    }
    // cooperative append workgroups
    {
        const int cap = sgks::max_append_groups();
        int G = c->opt.append_groups;
        if (G == 0) G = sgks::choose_append_groups(s, dmax, cap, S.A.nnz + S.L.nnz);
        if (G > cap) G = cap;
        if (!sgks::append_groups_ok(s, dmax, G)) return SGKS_ERR_SKETCH_SIZE;
        c->groups = G;
    }

    return SGKS_OK;
}

// Device memory of a context: every piece registered with the arena (its
// pointers are filled in by the commit).  The transposes' sort scratch lives
// in W (and HW), unused until the transposes are built, or in a piece of its
// own when that is too small.
void layout_context(sgks_ctx* c, Arena& ar) {
    State& S = c->S;
    const int dmax = S.dmax, s = S.s;
    const size_t vsz = S.vdt == SGKS_F32 ? 4 : 8;
    const int nbA_max = sgks::scatter_blocks(S.m, 1), nbL_max = sgks::scatter_blocks(S.p, 1);
    const bool sparse = S.sketch_mode == SGKS_SKETCH_SPARSE_SIGN;
    const int regions = 2 * S.passes + 2;
    const int CW = 2 * dmax + 8;
    if (c->opt.order) {
        ar.add(&c->colA2, S.A.nnz * 4);
        ar.add(&c->colL2, S.L.nnz * 4);
        ar.add(&c->order_flag, 64);
    }
    ar.add(&c->At_rowptr, (S.n + 1) * 4);
    ar.add(&c->At_col, S.A.nnz * 4);
    ar.add((char**)&c->At_val, S.A.nnz * vsz);
    ar.add(&c->Lt_rowptr, (S.n + 1) * 4);
    ar.add(&c->Lt_col, S.L.nnz * 4);
    ar.add((char**)&c->Lt_val, S.L.nnz * vsz);
    ar.add((double**)&S.b, S.m * 8);
    ar.add(&S.x, S.n * 8);
    ar.add(&S.u, S.m * 8);
    ar.add(&S.t, S.p * 8);
    ar.add(&S.rtmp, S.n * 8);
    ar.add(&S.W, (size_t)S.n * dmax * 8);
    if (S.gradient_form == SGKS_GRADIENT_MAINTAINED) ar.add(&S.HW, (size_t)S.n * dmax * 8);
    // the small state, together
    ar.add(&S.cs, dmax * 8);
    ar.add(&S.QA, (size_t)s * dmax * 8);
    ar.add(&S.QL, (size_t)s * dmax * 8);
    ar.add(&S.QA32, (size_t)s * dmax * 4);
    ar.add(&S.QL32, (size_t)s * dmax * 4);
    ar.add(&S.RA, (size_t)dmax * dmax * 8);
    ar.add(&S.RL, (size_t)dmax * dmax * 8);
    ar.add(&S.U, (size_t)2 * dmax * dmax * 8);
    ar.add(&S.G, (size_t)2 * dmax * dmax * 8);   // G, then G^{-1}
    ar.add(&S.h, dmax * 8);
    ar.add(&S.dA, dmax * 8);
    ar.add(&S.cb, s * 8);
    ar.add(&S.y, dmax * 8);
    ar.add(&S.yprev, dmax * 8);
    ar.add(&S.norm_part, 2048 * 8);   // adjoint workgroups are capped at 2048
    ar.add(&S.binA, (size_t)nbA_max * s * 8);
    ar.add(&S.binL, (size_t)nbL_max * s * 8);
    if (sparse) {
        ar.add(&c->patA, (size_t)S.m * S.zeta * 2);
        ar.add(&c->patL, (size_t)S.p * S.zeta * 2);
    }
    if (S.sketch_mode == SGKS_SKETCH_SRTT) {
        ar.add((int32_t**)&S.rowsA, (size_t)s * 4);
        ar.add((int32_t**)&S.rowsL, (size_t)s * 4);
        ar.add((double**)&S.srtTA, (size_t)2 * sgks::srtt_pad(s) * 256 * 8);
        ar.add((double**)&S.srtTL, (size_t)2 * sgks::srtt_pad(s) * 256 * 8);
    }
    ar.add(&S.wa, s * 8);
    ar.add(&S.wl, s * 8);
    ar.add(&S.wu, 2 * dmax * 8);
    ar.add(&S.pacc, 4 * dmax * 8);
    ar.add(&S.gacc, dmax * 8);
    ar.add(&S.gpart, (size_t)S.ngt * (dmax + 1) * 8);
    if (S.gradient_form == SGKS_GRADIENT_MAINTAINED && c->opt.refine_steps > 0) {
        ar.add(&S.Mnt, (size_t)dmax * dmax * 8);
        ar.add(&S.cnt, dmax * 8);
    }
    if (c->opt.keep_history) ar.add(&S.yh, (size_t)(dmax + 1) * dmax * 8);
    ar.add(&S.coop, (size_t)regions * c->groups * CW * 8);
    ar.add(&S.scal, (16 + 2 * dmax) * 8);
    ar.add(&S.d, 64);
    ar.add(&S.status, 64);
    ar.add(&S.degenerate, 64);
    ar.add(&S.sync, 64);
    // forward workgroups for any lanes choice (at most four rows per workgroup fewer)
    ar.add(&c->upart, ((S.m + 3) / 4 + 1) * 8);
    ar.add(&c->tpart, ((S.p + 3) / 4 + 1) * 8);
    ar.add(&c->coefbuf, dmax * 8);
    ar.add(&c->sbuf, s * 8);
    ar.add(&c->init_norms, (16 + 2 * dmax) * 8);
    ar.add(&c->Sdev, sizeof(State));
    if (c->opt.keep_history) {
        sgks::Rev& R = c->rv;
        const int K = c->opt.max_iters;
        ar.add(&R.uh, (size_t)(dmax + 1) * dmax * 8);
        ar.add(&R.E, (size_t)S.n * (K > 0 ? K : 1) * 8);
        ar.add(&R.vbar, (size_t)S.n * c->opt.ell * 8);
        ar.add(&R.tv, S.n * 8);
        ar.add(&R.zb, S.n * 8);
        ar.add(&R.pb, S.n * 8);
        ar.add(&R.zh, S.n * 8);
        ar.add(&R.bA, S.m * 8);
        ar.add(&R.bL, S.p * 8);
        ar.add(&R.zA, (size_t)s * 8);
        ar.add(&R.zL, (size_t)s * 8);
        // L-row workgroups of the forward products for any lanes choice (the
        // autotuner may change them after the layout)
        ar.add(&R.ldot, (size_t)((S.p + 3) / 4 + 1) * 8);
        ar.add(&R.ubar, dmax * 8);
        ar.add(&R.vA, dmax * 8);
        ar.add(&R.vL, dmax * 8);
        ar.add(&R.dz, dmax * 8);
        ar.add(&R.dp, dmax * 8);
        R.kld = K + 1;
        ar.add(&R.kap, (size_t)dmax * (K + 1) * 8);
        ar.add(&R.ones, (size_t)(K > 0 ? K : 1) * 8);
        ar.add(&R.rs, 16 * 8);
        ar.add(&R.mupart, (size_t)(K + 1) * 8);
    }
    if (S.method == SGKS_METHOD_GKS) {
        ar.add(&S.QAt, (size_t)S.m * dmax * 8);
        ar.add(&S.QLt, (size_t)S.p * dmax * 8);
        ar.add(&S.wat, S.m * 8);
        ar.add(&S.wlt, S.p * 8);
        ar.add(&S.tpA, (size_t)S.ntA * dmax * 8);
        ar.add(&S.tpL, (size_t)S.ntL * dmax * 8);
        ar.add(&S.tsq, 5 * 4096 * 8);
        ar.add(&S.gco, 6 * dmax * 8);
        ar.add(&S.vsq, 2 * 2048 * 8);
    }
    const size_t wbytes = (size_t)S.n * dmax * 8 * (S.gradient_form == SGKS_GRADIENT_MAINTAINED ? 2 : 1);
    const size_t sort = std::max(sgks::transpose_scratch_bytes(S.A), sgks::transpose_scratch_bytes(S.L));
    c->sort_bytes = sort > wbytes ? sort : 0;
    if (c->sort_bytes) ar.add(&c->sort_scratch, c->sort_bytes);
}

// ||v||, via the conversion kernel run in place, into cs[col] = 1/||v||
void norm_to_scale(sgks_ctx* c, double* v, int col, bool store_r0) {
    State& S = c->S;
    sgks::launch_to_f64(v, 1, v, S.n, S.norm_part, S.n_norm_part, c->st);
    sgks::launch_set_scale(S, col, store_r0, c->st);
}

}  // namespace

extern "C" {

void sgks_default_options(sgks_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->ell = 3;
    o->max_iters = 200;
    o->zeta = 8;
    o->value_dtype = SGKS_F64;
    o->refine_steps = 0;
    o->qr_passes = 2;
    o->sketch_mode = SGKS_SKETCH_SPARSE_SIGN;
    o->lanes_A = 0;
    o->lanes_At = 0;
    o->append_groups = 0;
    o->graph = 0;
    o->autotune = 0;
    o->keep_history = 0;
    o->gradient_form = SGKS_GRADIENT_MAINTAINED;
    o->method = SGKS_METHOD_SGKS;
    o->order = nullptr;
    o->workspace = nullptr;
    o->workspace_bytes = 0;
    o->stream = nullptr;
}

int sgks_validate(const sgks_csr* A, const sgks_csr* L, const void* b, double mu,
                  int32_t s, const sgks_options* opt) {
    sgks_options o;
    if (opt)
        o = *opt;
    else
        sgks_default_options(&o);
    int rc = check_csr(A);
    if (rc) return rc;
    rc = check_csr(L);
    if (rc) return rc;
    if (!b) return SGKS_ERR_INVALID_ARG;
    if (A->rows <= 0 || L->rows <= 0) return SGKS_ERR_SHAPE;
    if (L->cols != A->cols) return SGKS_ERR_SHAPE;
    if (!(mu > 0.0) || !(mu < INFINITY)) return SGKS_ERR_BAD_MU;
    if (o.ell < 1 || o.max_iters < 0) return SGKS_ERR_INVALID_ARG;
    if ((int64_t)o.ell + o.max_iters > sgks::kMaxD) return SGKS_ERR_CAPACITY;
    if (o.zeta != 2 && o.zeta != 4 && o.zeta != 8 && o.zeta != 16) return SGKS_ERR_INVALID_ARG;
    if (o.value_dtype != SGKS_F32 && o.value_dtype != SGKS_F64) return SGKS_ERR_INVALID_ARG;
    if (o.qr_passes != 1 && o.qr_passes != 2) return SGKS_ERR_INVALID_ARG;
    if (o.refine_steps < 0) return SGKS_ERR_INVALID_ARG;
    if (o.sketch_mode != SGKS_SKETCH_SPARSE_SIGN && o.sketch_mode != SGKS_SKETCH_IDENTITY &&
        o.sketch_mode != SGKS_SKETCH_SRTT)
        return SGKS_ERR_INVALID_ARG;
    if (!pow2_lanes(o.lanes_A) || !pow2_lanes(o.lanes_At)) return SGKS_ERR_INVALID_ARG;
    if (o.append_groups < 0) return SGKS_ERR_INVALID_ARG;
    if ((o.graph != 0 && o.graph != 1) || (o.autotune != 0 && o.autotune != 1))
        return SGKS_ERR_INVALID_ARG;
    if (o.gradient_form != SGKS_GRADIENT_MAINTAINED && o.gradient_form != SGKS_GRADIENT_DIRECT)
        return SGKS_ERR_INVALID_ARG;
    if (o.method != SGKS_METHOD_SGKS && o.method != SGKS_METHOD_GKS) return SGKS_ERR_INVALID_ARG;
    if (o.keep_history != 0 && o.keep_history != 1) return SGKS_ERR_INVALID_ARG;
    // the total-derivative adjoint differentiates the unrefined sGKS map and reads H W
    if (o.keep_history && (o.method != SGKS_METHOD_SGKS || o.refine_steps != 0 ||
                           o.gradient_form != SGKS_GRADIENT_MAINTAINED))
        return SGKS_ERR_INVALID_ARG;
    if (o.method == SGKS_METHOD_GKS) return o.refine_steps == 0 ? 0 : SGKS_ERR_INVALID_ARG;
    if (s > sgks::kMaxSketch || s < 1) return SGKS_ERR_SKETCH_SIZE;
    if (o.sketch_mode == SGKS_SKETCH_SPARSE_SIGN) {
        if (s < o.ell + o.max_iters) return SGKS_ERR_SKETCH_SIZE;
        if (o.zeta > s) return SGKS_ERR_SKETCH_SIZE;
    } else if (o.sketch_mode == SGKS_SKETCH_SRTT) {
        // D keeps s distinct rows of each image
        if (s < o.ell + o.max_iters || (int64_t)s > A->rows || (int64_t)s > L->rows)
            return SGKS_ERR_SKETCH_SIZE;
    } else {
        if ((int64_t)s < A->rows || (int64_t)s < L->rows) return SGKS_ERR_SKETCH_SIZE;
    }
    return 0;
}

size_t sgks_workspace_bytes(const sgks_csr* A, const sgks_csr* L, int32_t s,
                            const sgks_options* opt) {
    // b is not read: any non-null pointer passes the validation
    if (sgks_validate(A, L, (const void*)A, 1.0, s, opt) != 0) return 0;
    sgks_ctx* c = new (std::nothrow) sgks_ctx();
    if (!c) return 0;
    if (opt)
        c->opt = *opt;
    else
        sgks_default_options(&c->opt);
    size_t total = 0;
    if (plan_context(c, A, L, 1.0, s, 0) == SGKS_OK) {
        Arena ar;
        layout_context(c, ar);
        total = ar.total;
    }
    delete c;
    return total;
}

int sgks_create(const sgks_csr* A, const sgks_csr* L, const void* b, double mu, int32_t s,
                uint64_t seed, const sgks_options* opt, sgks_ctx** out) {
    if (!out) return SGKS_ERR_INVALID_ARG;
    *out = nullptr;
    int rc = sgks_validate(A, L, b, mu, s, opt);
    if (rc) return rc;
    sgks_ctx* c = new (std::nothrow) sgks_ctx();
    if (!c) return SGKS_ERR_HIP;
    if (opt)
        c->opt = *opt;
    else
        sgks_default_options(&c->opt);
    rc = plan_context(c, A, L, mu, s, seed);
    if (rc) {
        sgks_destroy(c);
        return rc;
    }
    {
        // the device of the context, and (once per device) the address of its
        // copy of the static staging array
        void* sp = nullptr;
        if (hipGetDevice(&c->device) != hipSuccess || scratch_address(&sp) != SGKS_OK) {
            sgks_destroy(c);
            return SGKS_ERR_HIP;
        }
        // the sketch scatter holds at least one copy of the s bins in one workgroup's LDS
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
            hipSuccess) {
            sgks_destroy(c);
            return SGKS_ERR_HIP;
        }
        if (c->S.method == SGKS_METHOD_SGKS && sgks::scatter_lds_bytes(c->S.s) > (size_t)lds) {
            sgks_destroy(c);
            return SGKS_ERR_SKETCH_SIZE;
        }
    }
#define SGKS_TRY(expr)                      \
    do {                                    \
        if ((expr) != hipSuccess) {         \
            sgks_destroy(c);                \
            return SGKS_ERR_HIP;            \
        }                                   \
    } while (0)
    State& S = c->S;
    const int dmax = S.dmax;
    const bool sparse = S.sketch_mode == SGKS_SKETCH_SPARSE_SIGN;
    Arena ar;
    layout_context(c, ar);
    if (c->opt.workspace) {
        // caller-owned device memory: no allocation here
        if (c->opt.workspace_bytes < ar.total || ((uintptr_t)c->opt.workspace & 255)) {
            sgks_destroy(c);
            return SGKS_ERR_INVALID_ARG;
        }
        ar.place((char*)c->opt.workspace);
    } else {
        SGKS_TRY(ar.commit(c));
    }
    if (c->opt.order) {
        // internal order of the unknowns: relabel the columns of A and L (the
        // inverse permutation lives in x until the first iterate)
        SGKS_TRY(hipMemsetAsync(c->order_flag, 0, 64, c->st));
        if (sgks::order_setup(c->opt.order, S.n, (int32_t*)S.x, c->order_flag, S.A, c->colA2,
                              S.L, c->colL2, c->st)) {
            sgks_destroy(c);
            return SGKS_ERR_HIP;
        }
        S.A.col = c->colA2;
        S.L.col = c->colL2;
        S.perm = c->opt.order;
    }
    // sort scratch: W (and HW) before they are used, or its own piece
    void* sbase = c->sort_bytes ? c->sort_scratch : (void*)S.W;
    const size_t sbytes =
        c->sort_bytes ? c->sort_bytes : (size_t)S.n * dmax * 8 * (S.HW ? 2 : 1);
    if (sgks::transpose_csr(S.A, S.vdt, c->At_rowptr, c->At_col, c->At_val, sbase, sbytes,
                            c->st) ||
        sgks::transpose_csr(S.L, S.vdt, c->Lt_rowptr, c->Lt_col, c->Lt_val, sbase, sbytes,
                            c->st)) {
        sgks_destroy(c);
        return SGKS_ERR_HIP;
    }
    S.At.rowptr = c->At_rowptr;
    S.At.col = c->At_col;
    S.At.val = c->At_val;
    S.Lt.rowptr = c->Lt_rowptr;
    S.Lt.col = c->Lt_col;
    S.Lt.val = c->Lt_val;
    hipStream_t st = c->st;
    c->prof.st = st;
    if (sparse) {
        // the sparse-sign pattern, once, from the hash
        sgks::launch_make_pattern(c->patA, S.m, s, S.zeta, seed, 0, st);
        sgks::launch_make_pattern(c->patL, S.p, s, S.zeta, seed, 1, st);
        S.patA = c->patA;
        S.patL = c->patL;
    }
    if (S.sketch_mode == SGKS_SKETCH_SRTT) {
        // the frequencies D selects, drawn on the host
        c->srtt_rows.resize((size_t)2 * s);
        sgks::srtt_rows_host(S.m, s, seed, 0, c->srtt_rows.data());
        sgks::srtt_rows_host(S.p, s, seed, 1, c->srtt_rows.data() + s);
        SGKS_TRY(hipMemcpyAsync((void*)S.rowsA, c->srtt_rows.data(), (size_t)s * 4,
                                hipMemcpyHostToDevice, st));
        SGKS_TRY(hipMemcpyAsync((void*)S.rowsL, c->srtt_rows.data() + s, (size_t)s * 4,
                                hipMemcpyHostToDevice, st));
        sgks::launch_srtt_tables(S, st);   // the cosines and sines of the chunk rows
    }
    if (c->opt.autotune) {
        SGKS_TRY(hipMemsetAsync(S.x, 0, S.n * 8, st));
        SGKS_TRY(hipMemsetAsync(S.u, 0, S.m * 8, st));
        SGKS_TRY(hipMemsetAsync(S.t, 0, S.p * 8, st));
        if (!c->opt.lanes_A) S.A.lanes = tune_one(S, 0, st);
        S.L.lanes = tune_one(S, 1, st);
        if (!c->opt.lanes_At) S.At.lanes = tune_one(S, 2, st);
        S.Lt.lanes = S.At.lanes;
        if (sparse && S.s <= sgks::kMaxS) {   // the probe reduces bins as the compact append does
            const int tpw = tune_scatter(S, st);
            S.nbA = sgks::scatter_blocks(S.m, tpw);
            S.nbL = sgks::scatter_blocks(S.p, tpw);
        }
        SGKS_TRY(hipGetLastError());
        S.n_norm_part = norm_parts(S);
        int nbFA2 = 0;
        const int nbF2 = sgks::forward_blocks(S, true, &nbFA2);
        c->nbF_A = nbFA2;
        c->nbF_L = nbF2 - nbFA2;
    }
    // the kernels of the iteration read the State from device memory
    SGKS_TRY(hipMemcpyAsync(c->Sdev, &S, sizeof(State), hipMemcpyHostToDevice, st));
    if (sgks::plan_build(c->plan, &S, c->Sdev, 1, &c->groups)) {
        sgks_destroy(c);
        return SGKS_ERR_INVALID_ARG;
    }
    // the small state starts at zero: two contiguous runs of the arena (cs ..
    // yprev and wa .. sync, laid out in that order by layout_context;
    // the scratch pieces between them are written before they are read)
    {
        char* a0 = (char*)S.cs;
        char* a1 = (char*)(S.yprev + dmax);
        char* b0 = (char*)S.wa;
        char* b1 = (char*)S.sync + 64;
        if (!(a0 < a1 && b0 < b1 && (char*)S.QA > a0 && (char*)S.dA < a1 &&
              (char*)S.scal > b0 && (char*)S.d < b1)) {
            sgks_destroy(c);
            return SGKS_ERR_HIP;
        }
        SGKS_TRY(hipMemsetAsync(a0, 0, (size_t)(a1 - a0), st));
        SGKS_TRY(hipMemsetAsync(b0, 0, (size_t)(b1 - b0), st));
    }

    // b in FP64 and ||b||^2 (checked with everything else after the one
    // synchronisation at the end: a zero or non-finite b only makes the
    // set-up kernels compute zeros or NaNs)
    sgks::launch_to_f64(b, S.vdt, (double*)S.b, S.m, S.norm_part, S.n_norm_part, st);
    sgks::launch_sum_parts(S.norm_part, S.n_norm_part, S.scal + 2, st);

    const bool gks = S.method == SGKS_METHOD_GKS;
    if (gks) {
        // no sketch: scal[1] (the ||S_A b||^2 of the small-factor residual) is ||b||^2
        sgks::launch_sum_parts(S.norm_part, S.n_norm_part, S.scal + 1, st);
    } else {
        // c_b = S_A b
        if (S.sketch_mode == SGKS_SKETCH_SRTT)
            sgks::launch_srtt(S, S.b, nullptr, st);
        else
            sgks::launch_scatter(S, S.b, nullptr, st);
        sgks::launch_cb(S, st);
    }

    // initial basis: orthonormal basis of K_ell(A^T A, A^T b), CGS2 (stored
    // unnormalised with cs[j] = 1 / ||column||)
    sgks::launch_adjoint(S, S.b, nullptr, false, 0.0, S.W, S.norm_part, st);
    norm_to_scale(c, S.W, 0, true);   // partials of this context's norm layout
    for (int j = 1; j < c->opt.ell; ++j) {
        double* prev = S.W + (size_t)(j - 1) * S.n;
        double* col = S.W + (size_t)j * S.n;
        sgks::launch_forward(S, prev, nullptr, S.u, S.t, false, nullptr, nullptr, st);
        sgks::launch_adjoint(S, S.u, nullptr, false, 0.0, col, S.norm_part, st);
        // norm before the projections (to detect a Krylov space that stopped growing)
        sgks::launch_to_f64(col, 1, col, S.n, S.norm_part, S.n_norm_part, st);
        sgks::launch_sum_parts(S.norm_part, S.n_norm_part, S.scal + 16 + dmax + j, st);
        for (int pass = 0; pass < 2; ++pass) {
            sgks::launch_gemvt(S, col, j, st);
            sgks::launch_reduce_gpart(S, j, c->coefbuf, st);
            sgks::launch_gemv(S, c->coefbuf, col, col, j, st);
        }
        norm_to_scale(c, col, j, false);
    }
    // the initial norms, before the appends overwrite the scratch scalars
    SGKS_TRY(hipMemcpyAsync(c->init_norms, S.scal, (16 + 2 * dmax) * 8, hipMemcpyDeviceToDevice,
                            st));

    // sketch (sGKS) and QR-append the initial columns, then y_0
    for (int j = 0; j < c->opt.ell; ++j) {
        if (gks)
            sgks::launch_forward(S, S.W + (size_t)j * S.n, nullptr, S.u, S.t, true, nullptr,
                                 nullptr, st);
        else
            sgks::launch_sketch_column(S, j, st);
        if (S.HW)   // H W[:, j] = A^T (A w) + mu L^T (L w) from the images just formed
            sgks::launch_adjoint(S, S.u, S.t, true, S.mu, S.HW + (size_t)j * S.n, S.norm_part,
                                 st);
        if (gks) {
            sgks::gks_append(S, c->Sdev, st);
            sgks::plan_stack_only(c->plan, st);
        } else if (sgks::plan_append(c->plan, false, false, st)) {
            sgks_destroy(c);
            return SGKS_ERR_HIP;
        }
        // maintained form with refinement: column j of W^T H W (the refinement
        // steps after the last initial column)
        if (S.Mnt)
            enqueue_refinement(c->plan, j + 1 == c->opt.ell ? c->opt.refine_steps : 0, nullptr, st);
    }
    if (!S.Mnt && c->opt.refine_steps > 0)
        enqueue_refinement(c->plan, c->opt.refine_steps, nullptr, st);
    if (S.yh) {
        sgks::launch_record_y(c->Sdev, 1, st);
        if (c->opt.max_iters > 0) sgks::launch_fill(c->rv.ones, c->opt.max_iters, 1.0, st);
    }
    c->d_host = c->opt.ell;

    // the one synchronisation of the set-up: ||b||^2, the initial norms and the status
    std::vector<double> sc(16 + 2 * dmax, 0.0);
    int stw = 0;
    SGKS_TRY(hipMemcpyAsync(sc.data(), c->init_norms, sc.size() * 8, hipMemcpyDeviceToHost, st));
    SGKS_TRY(hipMemcpyAsync(&stw, S.status, sizeof(int), hipMemcpyDeviceToHost, st));
    int bad_order = 0;
    if (c->order_flag)
        SGKS_TRY(hipMemcpyAsync(&bad_order, c->order_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    SGKS_TRY(hipStreamSynchronize(st));
    if (bad_order) {
        sgks_destroy(c);
        return SGKS_ERR_INVALID_ARG;
    }
    int err = SGKS_OK;
    const double bn2 = sc[2], r0 = sc[0];
    if (!(bn2 < INFINITY))
        err = SGKS_ERR_NONFINITE;
    else if (!(bn2 > 0.0))
        err = SGKS_ERR_ZERO_RHS;
    else if (!(r0 < INFINITY))
        err = SGKS_ERR_NONFINITE;
    else if (!(r0 > 0.0))
        err = SGKS_ERR_ZERO_RHS;
    for (int j = 1; j < c->opt.ell && err == SGKS_OK; ++j) {
        // after / before the projections, squared norms vs norms
        const double after = sc[16 + j], before = sqrt(sc[16 + dmax + j]);
        if (!(after < INFINITY) || !(before < INFINITY))
            err = SGKS_ERR_NONFINITE;
        else if (!(after > 1e-12 * before))
            err = SGKS_ERR_INITIAL_SPACE;
    }
    if (err == SGKS_OK && stw != 0) err = stw == SGKS_BREAKDOWN ? SGKS_ERR_INITIAL_SPACE : stw;
    if (err != SGKS_OK) {
        sgks_destroy(c);
        return err;
    }
    *out = c;
    return SGKS_OK;
#undef SGKS_TRY
}

int sgks_iterate(sgks_ctx* c, int32_t k) {
    if (!c || k < 0) return SGKS_ERR_INVALID_ARG;
    if (c->d_host + k > c->S.dmax) return SGKS_ERR_CAPACITY;
    const int rc = run_iterations(c->plan, c->opt.refine_steps, &c->prof, &c->graphs,
                                  c->opt.graph != 0, c->st, k, &c->side);
    if (rc) return rc;
    c->d_host += k;
    return SGKS_OK;
}

int sgks_solution(sgks_ctx* c, double* x_dev) {
    if (!c || !x_dev) return SGKS_ERR_INVALID_ARG;
    Phase ph(&c->prof, 0);
    sgks::launch_solution(c->S, x_dev, c->st);
    return hipGetLastError() == hipSuccess ? SGKS_OK : SGKS_ERR_HIP;
}

int sgks_residual_norm(sgks_ctx* c, double* true_norm, double* sketched_norm) {
    if (!c) return SGKS_ERR_INVALID_ARG;
    State& S = c->S;
    hipStream_t st = c->st;
    sgks::launch_gemv(S, S.y, S.x, nullptr, -1, st);
    sgks::launch_forward(S, S.x, S.b, S.u, S.t, true, c->upart, c->tpart, st);
    sgks::launch_sum_parts(c->upart, c->nbF_A, S.scal + 8, st);
    sgks::launch_sum_parts(c->tpart, c->nbF_L, S.scal + 9, st);
    sgks::launch_residual_small(S, S.scal + 10, st);
    double v[3] = {0, 0, 0};
    if (hipMemcpyAsync(v, S.scal + 8, 24, hipMemcpyDeviceToHost, st) != hipSuccess)
        return SGKS_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SGKS_ERR_HIP;
    if (true_norm) *true_norm = sqrt(v[0] + S.mu * v[1]);
    if (sketched_norm) *sketched_norm = sqrt(v[2] > 0.0 ? v[2] : 0.0);
    return SGKS_OK;
}

int sgks_status(sgks_ctx* c, int32_t* iters_done) {
    if (!c) return SGKS_ERR_INVALID_ARG;
    int st = sync_status(c);
    int d = 0;
    if (hipMemcpy(&d, c->S.d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SGKS_ERR_HIP;
    if (iters_done) *iters_done = d - c->opt.ell;
    return st;
}

int sgks_backward(sgks_ctx* c, const double* grad_x, double* grad_b, double* grad_mu) {
    if (!c || !grad_x || !grad_b) return SGKS_ERR_INVALID_ARG;
    // the adjoint is that of the unrefined projected solve (y = G^{-1} h); a
    // refined y is another function of b and mu
    if (c->opt.refine_steps > 0 || c->S.method == SGKS_METHOD_GKS) return SGKS_ERR_INVALID_ARG;
    State& S = c->S;
    hipStream_t st = c->st;
    if (S.perm) {
        sgks::launch_gather_perm(grad_x, S.perm, S.n, S.rtmp, st);
        grad_x = S.rtmp;
    }
    sgks::launch_gemvt(S, grad_x, -1, st);
    sgks::launch_backward_small(S, c->sbuf, S.scal + 11, st);
    sgks::launch_sketch_transpose(S, c->sbuf, grad_b, st);
    double gm = 0.0;
    if (hipMemcpyAsync(&gm, S.scal + 11, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
        return SGKS_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SGKS_ERR_HIP;
    if (grad_mu) *grad_mu = gm;
    return SGKS_OK;
}

// ||M||_2 of an upper-triangular d x d row-major matrix (leading dimension ld) by
// power iteration on M^T M from a fixed start (a lower bound that converges to it)
static double tri_norm2(const std::vector<double>& M, int d, int ld) {
    std::vector<double> v(d, 1.0 / sqrt((double)d)), w(d), z(d);
    double lam = 0.0;
    for (int it = 0; it < 40; ++it) {
        for (int i = 0; i < d; ++i) {
            double a = 0.0;
            for (int j = i; j < d; ++j) a += M[(size_t)i * ld + j] * v[j];
            w[i] = a;
        }
        for (int j = 0; j < d; ++j) z[j] = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = i; j < d; ++j) z[j] += M[(size_t)i * ld + j] * w[i];
        double nz = 0.0;
        for (int j = 0; j < d; ++j) nz += z[j] * z[j];
        nz = sqrt(nz);
        if (!(nz > 0.0) || !(nz < INFINITY)) return nz;
        lam = nz;   // ||M^T M v|| with ||v|| = 1
        for (int j = 0; j < d; ++j) v[j] = z[j] / nz;
    }
    return sqrt(lam);
}

int sgks_backward_total(sgks_ctx* c, const double* grad_x, double* grad_b, double* grad_mu,
                        double* err_est) {
#define SGKS_HIP_OK(expr) \
    do { if ((expr) != hipSuccess) return SGKS_ERR_HIP; } while (0)
    if (!c || !grad_x || !grad_b) return SGKS_ERR_INVALID_ARG;
    State& S = c->S;
    if (!S.yh) return SGKS_ERR_INVALID_ARG;
    const int stw = sync_status(c);
    if (stw < 0) return stw;
    sgks::Rev R = c->rv;
    R.nldot = c->nbF_L;   // L-row workgroups of the forward products (final lanes)
    hipStream_t st = c->st;
    const int ell = c->opt.ell;
    int d = 0;
    SGKS_HIP_OK(hipMemcpyAsync(&d, S.d, sizeof(int), hipMemcpyDeviceToHost, st));
    SGKS_HIP_OK(hipStreamSynchronize(st));
    const int k = d - ell;   // expansions done (a breakdown stops them early)
    if (k < 0 || k > c->opt.max_iters) return SGKS_ERR_DEVICE;
    const int64_t n = S.n;
    if (S.perm) {
        sgks::launch_gather_perm(grad_x, S.perm, n, S.rtmp, st);
        grad_x = S.rtmp;
    }
    const int dmax = S.dmax;
    SGKS_HIP_OK(hipMemsetAsync(R.uh, 0, (size_t)(dmax + 1) * dmax * 8, st));
    SGKS_HIP_OK(hipMemsetAsync(R.ubar, 0, (size_t)dmax * 8, st));
    SGKS_HIP_OK(hipMemsetAsync(R.rs, 0, 16 * 8, st));

    // The coefficients of every column's sum over the stored e_i come from the y
    // history alone, so the next column's sum (bandwidth bound) runs on the second
    // stream beside this column's adjoint solve (one workgroup, latency bound).
    sgks::launch_rev_kap(S, R, ell, k, st);
    SideStream* ss = c->side.ready() ? &c->side : nullptr;
    bool pending = false;
    auto tgemv = [&](int c_) -> int {   // tv for column c_ (after the e_i it reads)
        const int i0 = c_ - ell + 1 > 0 ? c_ - ell + 1 : 0;
        if (!ss) {
            sgks::launch_rev_tgemv(S, R, c_, i0, k - i0, st);
            return SGKS_OK;
        }
        if (hipEventRecord(ss->fork, st) != hipSuccess ||
            hipStreamWaitEvent(ss->side, ss->fork, 0) != hipSuccess)
            return SGKS_ERR_HIP;
        sgks::launch_rev_tgemv(S, R, c_, i0, k - i0, ss->side);
        if (hipEventRecord(ss->join, ss->side) != hipSuccess) return SGKS_ERR_HIP;
        pending = true;
        return SGKS_OK;
    };
    auto join = [&]() -> int {
        if (pending) {
            if (hipStreamWaitEvent(st, ss->join, 0) != hipSuccess) return SGKS_ERR_HIP;
            pending = false;
        }
        return SGKS_OK;
    };
    // one column c: its adjoint, scaled by `scale`, into dst (its tv already formed)
    auto column = [&](int c_, const double* scale, double* dst) -> int {
        sgks::launch_rev_svec(S, R, d, st);                    // Q R C[:, c] (- S_A b ubar_c)
        if (join()) return SGKS_ERR_HIP;
        sgks::launch_rev_forward(S, R, S.W + (size_t)c_ * n, st);   // with S_A^T zA, S_L^T zL
        sgks::launch_rev_adjoint(S, R, grad_x, scale, dst, st);
        return SGKS_OK;
    };
    // the last solve: W_k^T grad_x, then the columns from the newest down
    sgks::launch_gemvt(S, grad_x, d, st);
    if (tgemv(d - 1)) return SGKS_ERR_HIP;
    sgks::launch_rev_small(S, R, ell, k, k, d - 1, -1, 0, st);
    for (int j = k - 1; j >= 0; --j) {
        const int cc = ell + j;   // made from the gradient r_j
        double* e = R.E + (size_t)j * n;
        if (column(cc, S.cs + cc, e)) return SGKS_ERR_HIP;   // e_j = adjoint / ||r_j||
        sgks::launch_gemvt_mat(S, S.HW, e, cc, st);   // W_j^T H e_j
        if (tgemv(cc - 1)) return SGKS_ERR_HIP;
        sgks::launch_rev_small(S, R, ell, k, j, cc - 1, cc, 0, st);
    }
    for (int cc = ell - 1; cc >= 0; --cc) {
        if (column(cc, nullptr, R.vbar + (size_t)cc * n)) return SGKS_ERR_HIP;
        if (cc > 0 && tgemv(cc - 1)) return SGKS_ERR_HIP;
        sgks::launch_rev_small(S, R, ell, k, -1, cc - 1, cc, cc == 0 ? 1 : 0, st);
    }
    if (join()) return SGKS_ERR_HIP;
    sgks::launch_rev_mu(S, R, ell, k, st);   // the solves' mu terms, off the column chain
    // the initial basis: v_i = p_i / ||p_i||, p_i = (I - V_i V_i^T) A^T A v_{i-1}
    // (raw columns: W[:, i] = p_i / cs[i - 1], cs[i] = 1 / ||W[:, i]||)
    for (int i = ell - 1; i >= 1; --i) {
        const double* wprev = S.W + (size_t)(i - 1) * n;
        sgks::launch_forward(S, wprev, nullptr, S.u, S.t, false, nullptr, nullptr, st);
        sgks::launch_adjoint(S, S.u, nullptr, false, 0.0, R.zb, nullptr, st);   // z (raw)
        sgks::launch_gemvt(S, R.zb, i, st);
        sgks::launch_reduce_gpart(S, i, R.dz, st);                             // V_i^T z
        sgks::LinComb lc{};
        lc.t[0] = sgks::LinTerm{R.vbar + (size_t)i * n, 1.0, S.cs + i, nullptr, 0};
        lc.nt = 1;
        sgks::launch_lincomb(lc, n, R.pb, false, st);                           // p^ (raw)
        sgks::launch_gemvt(S, R.pb, i, st);
        sgks::launch_reduce_gpart(S, i, R.dp, st);                             // V_i^T p^
        sgks::launch_gemv(S, R.dp, R.zh, R.pb, i, st);                         // z^ (raw)
        for (int l = 0; l < i; ++l) {
            sgks::LinComb u{};
            u.t[0] = sgks::LinTerm{R.pb, -1.0, R.dz + l, nullptr, 0};
            u.t[1] = sgks::LinTerm{R.zb, -1.0, R.dp + l, nullptr, 0};
            u.nt = 2;
            sgks::launch_lincomb(u, n, R.vbar + (size_t)l * n, true, st);
        }
        sgks::launch_forward(S, R.zh, nullptr, S.u, S.t, false, nullptr, nullptr, st);
        sgks::launch_adjoint(S, S.u, nullptr, false, 0.0, R.zb, nullptr, st);   // A^T A z^
        sgks::LinComb a{};
        a.t[0] = sgks::LinTerm{R.zb, 1.0, S.cs + (i - 1), nullptr, 1};
        a.nt = 1;
        sgks::launch_lincomb(a, n, R.vbar + (size_t)(i - 1) * n, true, st);
    }
    // d loss / d b = A (cs[0] vbar_0 - sum_j e_j) + S_A^T Q_A R_A ubar
    {
        sgks::LinComb v0{};
        v0.t[0] = sgks::LinTerm{R.vbar, 1.0, S.cs, nullptr, 0};
        v0.nt = 1;
        sgks::launch_lincomb(v0, n, R.zb, false, st);
        sgks::launch_gemv_plain(S, R.E, R.ones, k, R.zb, R.zh, st);
        sgks::launch_rev_svec(S, R, d, st);   // zA = -Q_A R_A ubar (set by the last small step)
        sgks::launch_sketch_transpose_side(S, 0, R.zA, R.bA, st);
        sgks::launch_forward(S, R.zh, R.bA, grad_b, S.t, false, nullptr, nullptr, st);
    }
    double gm = 0.0;
    SGKS_HIP_OK(hipGetLastError());
    SGKS_HIP_OK(hipMemcpyAsync(&gm, R.rs, 8, hipMemcpyDeviceToHost, st));
    if (err_est) {
        // d eps kappa(G)^2: the adjoint solves with N_j = G_j^T G_j
        std::vector<double> Gh((size_t)d * dmax), Gih((size_t)d * dmax);
        SGKS_HIP_OK(hipMemcpyAsync(Gh.data(), S.G, Gh.size() * 8, hipMemcpyDeviceToHost, st));
        SGKS_HIP_OK(hipMemcpyAsync(Gih.data(), S.G + (size_t)dmax * dmax, Gih.size() * 8,
                                   hipMemcpyDeviceToHost, st));
        SGKS_HIP_OK(hipStreamSynchronize(st));
        const double kap = tri_norm2(Gh, d, dmax) * tri_norm2(Gih, d, dmax);
        *err_est = (double)d * 0x1p-53 * kap * kap;
    }
    SGKS_HIP_OK(hipStreamSynchronize(st));
    if (grad_mu) *grad_mu = gm;
    return SGKS_OK;
#undef SGKS_HIP_OK
}

int64_t sgks_copy_state(sgks_ctx* c, int32_t which, double* dst, int64_t count) {
    if (!c || !dst) return SGKS_ERR_INVALID_ARG;
    State& S = c->S;
    hipStream_t st = c->st;
    if (hipStreamSynchronize(st) != hipSuccess) return SGKS_ERR_HIP;
    int d = 0;
    if (hipMemcpy(&d, S.d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SGKS_ERR_HIP;
    const int dmax = S.dmax;
    auto copy = [&](const double* src, int64_t n) -> int64_t {
        if (n > count) return SGKS_ERR_INVALID_ARG;
        if (n > 0 && hipMemcpy(dst, src, n * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return SGKS_ERR_HIP;
        return n;
    };
    auto copy2d = [&](const double* src, int64_t rows, int64_t cols, int64_t ld) -> int64_t {
        if (rows * cols > count) return SGKS_ERR_INVALID_ARG;
        if (rows * cols > 0 &&
            hipMemcpy2D(dst, rows * 8, src, ld * 8, rows * 8, cols, hipMemcpyDeviceToHost) !=
                hipSuccess)
            return SGKS_ERR_HIP;
        return rows * cols;
    };
    switch (which) {
        case 0: {
            const int64_t n = S.n * (int64_t)d;
            if (n > count) return SGKS_ERR_INVALID_ARG;
            double* tmp = nullptr;
            if (hipMalloc(&tmp, (n > 0 ? n : 1) * 8) != hipSuccess) return SGKS_ERR_HIP;
            if (sgks::launch_copy_scaled_W(S, tmp, st) != 0 ||
                hipStreamSynchronize(st) != hipSuccess) {
                (void)hipFree(tmp);
                return SGKS_ERR_HIP;
            }
            int64_t r = copy(tmp, n);
            (void)hipFree(tmp);
            return r;
        }
        case 1: return copy(S.y, d);
        case 2:
            return S.method == SGKS_METHOD_GKS ? copy2d(S.QAt, S.m, d, S.m)
                                               : copy2d(S.QA, S.s, d, S.s);
        case 3: return copy2d(S.RA, d, d, dmax);
        case 4:
            return S.method == SGKS_METHOD_GKS ? copy2d(S.QLt, S.p, d, S.p)
                                               : copy2d(S.QL, S.s, d, S.s);
        case 5: return copy2d(S.RL, d, d, dmax);
        case 6: return copy(S.dA, d);
        case 7: {   // G is stored row-major: copy then transpose on the host
            const int64_t r = copy2d(S.G, d, d, dmax);
            if (r < 0) return r;
            for (int i = 0; i < d; ++i)
                for (int j = i + 1; j < d; ++j) {
                    const double t = dst[i + (int64_t)j * d];
                    dst[i + (int64_t)j * d] = dst[j + (int64_t)i * d];
                    dst[j + (int64_t)i * d] = t;
                }
            return r;
        }
        case 8: return S.method == SGKS_METHOD_GKS ? SGKS_ERR_INVALID_ARG : copy(S.cb, S.s);
        default: return SGKS_ERR_INVALID_ARG;
    }
}

int64_t sgks_copy_state_noalloc(sgks_ctx* c, int32_t which, double* dst, int64_t count) {
    if (!c || !dst) return SGKS_ERR_INVALID_ARG;
    if (which != 0) return sgks_copy_state(c, which, dst, count);   // no temporary there
    State& S = c->S;
    hipStream_t st = c->st;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SGKS_ERR_HIP;
    if (cur != c->device && hipSetDevice(c->device) != hipSuccess) return SGKS_ERR_HIP;
    int64_t rc = 0;
    void* sp = nullptr;
    int d = 0;
    const size_t colbytes = (size_t)S.n * sizeof(double);
    if (colbytes > SGKS_NOALLOC_SCRATCH_BYTES) {
        rc = SGKS_ERR_CAPACITY;   // one column of W does not fit the staging array
    } else if (scratch_address(&sp) != SGKS_OK || hipStreamSynchronize(st) != hipSuccess ||
               hipMemcpy(&d, S.d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
        rc = SGKS_ERR_HIP;
    } else if ((int64_t)S.n * d > count) {
        rc = SGKS_ERR_INVALID_ARG;
    } else {
        // W scaled to unit columns, as many columns at a time as the array holds
        const int per = (int)(SGKS_NOALLOC_SCRATCH_BYTES / colbytes);
        for (int j0 = 0; j0 < d && rc == 0; j0 += per) {
            const int nc = std::min(per, d - j0);
            sgks::launch_scaled_W_cols(S, j0, nc, (double*)sp, st);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(dst + (int64_t)j0 * S.n, sp, (size_t)nc * colbytes,
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = SGKS_ERR_HIP;
        }
        if (rc == 0) rc = (int64_t)S.n * d;
    }
    if (cur != c->device) (void)hipSetDevice(cur);
    return rc;
}

int sgks_profile_enable(sgks_ctx* c, int32_t on) {
    if (!c) return SGKS_ERR_INVALID_ARG;
    c->prof.on = on != 0;
    return SGKS_OK;
}

int sgks_profile_read(sgks_ctx* c, double* ms, int64_t* launches) {
    if (!c) return SGKS_ERR_INVALID_ARG;
    return c->prof.read(ms, launches);
}

int32_t sgks_dim(const sgks_ctx* c) { return c ? c->d_host : 0; }

int sgks_get_tuning(const sgks_ctx* c, int32_t out[6]) {
    if (!c || !out) return SGKS_ERR_INVALID_ARG;
    out[0] = c->S.A.lanes;
    out[1] = c->S.L.lanes;
    out[2] = c->S.At.lanes;
    out[3] = c->S.nbA;
    out[4] = c->S.nbL;
    out[5] = c->groups;
    return SGKS_OK;
}

static void destroy_ctx(sgks_ctx* c) {
    (void)hipStreamSynchronize(c->st);
    for (void* p : c->allocs) (void)hipFree(p);
    delete c;
}

void sgks_destroy(sgks_ctx* c) {
    if (!c || c->borrowed) return;
    destroy_ctx(c);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

}  // extern "C"

struct sgks_batch {
    std::vector<sgks_ctx*> ctx;
    std::vector<State> host;    // host copies of the States (the plan points at them)
    State* Sdev = nullptr;      // device array of the problems' States
    bool own_sdev = false;      // allocated here (not in a caller's workspace)
    sgks::Plan plan;
    sgks_options opt;
    hipStream_t st = nullptr;
    Profiler prof;
    GraphCache graphs;
    SideStream side;
};

namespace {

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// arena bytes of each problem of a batch (0 if one is invalid)
bool batch_sizes(int32_t count, const sgks_problem* probs, const sgks_options& o,
                 std::vector<size_t>& sizes) {
    sizes.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        sgks_options oi = o;
        oi.workspace = nullptr;
        oi.workspace_bytes = 0;
        oi.order = probs[i].order;
        sizes[i] = sgks_workspace_bytes(&probs[i].A, &probs[i].L, probs[i].sketch_rows, &oi);
        if (!sizes[i]) return false;
    }
    return true;
}

}  // namespace

extern "C" {

size_t sgks_batch_workspace_bytes(int32_t count, const sgks_problem* probs,
                                  const sgks_options* opt) {
    if (count < 1 || count > sgks::kMaxBatch || !probs) return 0;
    sgks_options o;
    if (opt)
        o = *opt;
    else
        sgks_default_options(&o);
    std::vector<size_t> sizes;
    if (!batch_sizes(count, probs, o, sizes)) return 0;
    size_t total = 0;
    for (size_t v : sizes) total += round256(v);
    return total + round256(sizeof(State) * count);
}

int sgks_batch_create(int32_t count, const sgks_problem* probs, const sgks_options* opt,
                      sgks_batch** out) {
    if (!out) return SGKS_ERR_INVALID_ARG;
    *out = nullptr;
    if (count < 1 || count > sgks::kMaxBatch || !probs) return SGKS_ERR_INVALID_ARG;
    sgks_options o;
    if (opt)
        o = *opt;
    else
        sgks_default_options(&o);
    if (o.lanes_A || o.lanes_At || o.append_groups || o.method != SGKS_METHOD_SGKS)
        return SGKS_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        const int rc = sgks_validate(&probs[i].A, &probs[i].L, probs[i].b, probs[i].mu,
                                     probs[i].sketch_rows, &o);
        if (rc) return rc;
    }
    // a caller's workspace: the contexts' arenas in problem order, then the States
    std::vector<size_t> offs(count, 0), sizes;
    char* ws = (char*)o.workspace;
    size_t states_off = 0;
    if (ws) {
        if (((uintptr_t)ws & 255) || !batch_sizes(count, probs, o, sizes))
            return SGKS_ERR_INVALID_ARG;
        size_t off = 0;
        for (int i = 0; i < count; ++i) {
            offs[i] = off;
            off += round256(sizes[i]);
        }
        states_off = off;
        if (o.workspace_bytes < off + round256(sizeof(State) * count)) return SGKS_ERR_INVALID_ARG;
    }
    sgks_batch* B = new (std::nothrow) sgks_batch();
    if (!B) return SGKS_ERR_HIP;
    B->opt = o;
    B->st = (hipStream_t)o.stream;
    B->prof.st = B->st;
    auto fail = [&](int rc) {
        sgks_batch_destroy(B);
        return rc;
    };
    std::vector<State>& host = B->host;
    host.resize(count);
    std::vector<int> groups(count);
    for (int i = 0; i < count; ++i) {
        sgks_ctx* c = nullptr;
        sgks_options oi = o;
        oi.order = probs[i].order;
        if (ws) {
            oi.workspace = ws + offs[i];
            oi.workspace_bytes = round256(sizes[i]);
        }
        const int rc = sgks_create(&probs[i].A, &probs[i].L, probs[i].b, probs[i].mu,
                                   probs[i].sketch_rows, probs[i].seed, &oi, &c);
        if (rc) return fail(rc);
        c->borrowed = true;
        B->ctx.push_back(c);
        host[i] = c->S;
        groups[i] = c->groups;
    }
    if (ws) {
        B->Sdev = (State*)(ws + states_off);
    } else {
        if (hipMalloc((void**)&B->Sdev, sizeof(State) * count) != hipSuccess) {
            B->Sdev = nullptr;
            return fail(SGKS_ERR_HIP);
        }
        B->own_sdev = true;
    }
    if (hipMemcpyAsync(B->Sdev, host.data(), sizeof(State) * count, hipMemcpyHostToDevice,
                       B->st) != hipSuccess ||
        hipStreamSynchronize(B->st) != hipSuccess)
        return fail(SGKS_ERR_HIP);
    if (sgks::plan_build(B->plan, host.data(), B->Sdev, count, groups.data()))
        return fail(SGKS_ERR_INVALID_ARG);
    *out = B;
    return SGKS_OK;
}

int sgks_batch_iterate(sgks_batch* B, int32_t k) {
    if (!B || k < 0) return SGKS_ERR_INVALID_ARG;
    for (sgks_ctx* c : B->ctx)
        if (c->d_host + k > c->S.dmax) return SGKS_ERR_CAPACITY;
    const int rc = run_iterations(B->plan, B->opt.refine_steps, &B->prof, &B->graphs,
                                  B->opt.graph != 0, B->st, k, &B->side);
    if (rc) return rc;
    for (sgks_ctx* c : B->ctx) c->d_host += k;
    return SGKS_OK;
}

sgks_ctx* sgks_batch_get(sgks_batch* B, int32_t i) {
    if (!B || i < 0 || i >= (int32_t)B->ctx.size()) return nullptr;
    return B->ctx[i];
}

int32_t sgks_batch_count(const sgks_batch* B) { return B ? (int32_t)B->ctx.size() : 0; }

int sgks_batch_profile_enable(sgks_batch* B, int32_t on) {
    if (!B) return SGKS_ERR_INVALID_ARG;
    B->prof.on = on != 0;
    return SGKS_OK;
}

int sgks_batch_profile_read(sgks_batch* B, double* ms, int64_t* launches) {
    if (!B) return SGKS_ERR_INVALID_ARG;
    return B->prof.read(ms, launches);
}

void sgks_batch_destroy(sgks_batch* B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->st);
    for (sgks_ctx* c : B->ctx) destroy_ctx(c);
    if (B->Sdev && B->own_sdev) (void)hipFree(B->Sdev);
    delete B;
}

const char* sgks_strerror(int code) {
    switch (code) {
        case SGKS_OK: return "ok";
        case SGKS_BREAKDOWN: return "breakdown: the gradient vanished (invariant subspace)";
        case SGKS_ERR_INVALID_ARG: return "invalid argument";
        case SGKS_ERR_SHAPE: return "shape mismatch";
        case SGKS_ERR_BAD_MU: return "mu must be positive and finite";
        case SGKS_ERR_SKETCH_SIZE: return "sketch size out of range";
        case SGKS_ERR_CAPACITY: return "basis capacity exceeded";
        case SGKS_ERR_ZERO_RHS: return "b (or A^T b) is zero";
        case SGKS_ERR_NONFINITE: return "non-finite value";
        case SGKS_ERR_HIP: return "HIP runtime error";
        case SGKS_ERR_DEVICE: return "device-side failure";
        case SGKS_ERR_INITIAL_SPACE: return "initial Krylov space has dimension below ell";
        default: return "unknown error";
    }
}

}  // extern "C"
