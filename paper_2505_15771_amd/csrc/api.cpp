// C ABI of the HHO elasto-acoustic ERK engine (declared in include/hho.h): context
// lifetime, device buffers, state transfer, sources, loads, receivers and the
// explicit Runge-Kutta driver (Sec. 4.2, eq. ERK_compact / ex_solve, tableaux eq. ERK).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/hho.h"
#include "device.h"
#include "initial.h"
#include "internal.h"
#include "plan.h"

using namespace hho;

// Workspace of the discrete adjoint (allocated by the first hho_adjoint_step, grown on demand).
struct AdjWork {
    // adjoint arena, addressed by the kernels through one buffer resource like the forward one:
    // lambda, z (two stage buffers), the running sum of L^T mu, two trace buffers, and copies of
    // the link / face-coefficient / material arrays
    void *arena = nullptr;
    size_t arena_bytes = 0;
    void *lam = nullptr, *Z[2] = {nullptr, nullptr}, *acc = nullptr, *T[2] = {nullptr, nullptr};
    int32_t *link = nullptr;
    void *c0 = nullptr, *mat = nullptr;
    // forward data of one checkpoint segment: per (step, stage) slot the primal rows of Y_i
    // ([2N][LT]), k_i ([5N][LT]) and the primal face values of Y_i ([trace rows][LT]); two
    // segments' worth (store_slots each), so that the recompute of one segment overlaps the
    // adjoint stages of the next
    size_t slot_elems = 0, k_off = 0, f_off = 0;
    void *store[2] = {nullptr, nullptr};
    size_t store_slots = 0;
    // second stream (default priority) for the forward recompute, its events, and the clock that
    // the adjoint kernels read (only dt), apart from the forward clock the recompute advances
    hipStream_t aux = nullptr;
    hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
    Clock *aclock = nullptr;
    Clock h_aclock{};
    void *ckpt = nullptr;  // checkpoints U^{g * every} and U^N, [n + 1][5N][LT]
    // Captured graphs of one full checkpoint segment for store buffer b: the forward recompute with
    // stage stores (replayed on aux) and the adjoint stages (replayed on the context's stream).  Valid
    // while the key (segment length, steps, context version, buffers) is unchanged.
    hipGraphExec_t rec_graph[2] = {nullptr, nullptr}, adj_graph[2] = {nullptr, nullptr};
    int g_every = 0, g_steps = 0;
    double g_dt = 0.0;  // the adjoint stage coefficients dt b_i, dt a_{i+1,i} are launch arguments
    unsigned g_version = 0;
    const void *g_key[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t ckpt_states = 0;
    double *gacc = nullptr, *gm = nullptr, *grad = nullptr, *dobs = nullptr;
    size_t dobs_cap = 0;
    int32_t *ic_of_cell = nullptr;
};

// Captured step graphs: one of kGraphSteps steps and one of each smaller power of two, so that a
// call of any length replays graphs only (n = q kGraphSteps + the binary digits of the rest).
constexpr int kGraphSteps = 32;
constexpr int kNumGraphs = 6;  // 32, 16, 8, 4, 2, 1 steps
static_assert(kGraphSteps == 1 << (kNumGraphs - 1), "graph lengths are the powers of two up to kGraphSteps");

struct hho_ctx {
    Plan plan;
    int dtype = 0, stages = 4, record_energy = 0, device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;
    size_t rsize = 8;          // bytes per real
    long long LT = 0;          // lanes
    int rows = 0, trows = 0;   // state rows (5N), trace rows
    void *U = nullptr, *Y[2] = {nullptr, nullptr}, *acc = nullptr, *T[3] = {nullptr, nullptr, nullptr};
    int tcur = 0;
    bool traces_valid = false;
    void *arena = nullptr;  // state, stage, trace, link, c0 and mat arrays (one buffer resource)
    size_t arena_bytes = 0;
    int32_t *link = nullptr;
    void *c0 = nullptr, *mat = nullptr, *tab = nullptr;
    double *emat = nullptr;
    int32_t *ic_tab = nullptr;  // [n_ic] class table offset per internal cell
    // launch shapes (Plan::launches) and the one in use
    struct LaunchDev {
        GroupDev *groups = nullptr;
        int32_t *blk_group = nullptr;
        int n_blocks = 0, cpb = 0, lanes = 0;
    };
    std::vector<LaunchDev> launch;
    int shape = 0;
    int n_blocks() const { return launch[shape].n_blocks; }
    int max_blocks = 0;
    int64_t *map = nullptr;
    double *staging = nullptr;
    // point sources
    std::vector<SrcDev> h_src;
    int32_t *src_first = nullptr;
    SrcDev *src = nullptr;
    size_t src_cap = 0;
    // separable loads
    int nterms = 0;
    double omega[4] = {0, 0, 0, 0}, phase[4] = {0, 0, 0, 0};
    void *gload = nullptr;
    // receivers
    int nrec = 0;
    int rec_w = 2;  // values per receiver and step (3 in three dimensions: p, or v_x, v_y, v_z)
    int32_t *rec_first = nullptr;
    RecDev *rec = nullptr;
    double *rec_out = nullptr;
    size_t rec_cap = 0;
    int last_steps = 0;
    // energy; pinned host copies of the initial energies and of the recorded history, so that a
    // batch reads every context's energies with one synchronisation
    // energy partials: kGraphSteps slots of [max_blocks][S] (one per step, summed once per graph)
    double *e_part = nullptr, *e_hist = nullptr, *e_now = nullptr;
    size_t e_part_cap = 0;
    size_t e_hist_cap = 0;
    double *h_e0 = nullptr, *h_ehist = nullptr;
    size_t h_ehist_cap = 0;
    // device clocks (two, alternating by step parity) and the cached step graphs (kGraphSteps >> i
    // steps in gexec[i])
    Clock *clock = nullptr;
    Clock h_clock{};
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[kNumGraphs] = {};
    unsigned version = 1, graph_version = 0;  // graphs are valid when graph_version == version
    double cfl_dt = 0.0;                       // CFL-limited time step at factor 1
    // Stage outputs stored with the non-temporal cache policy (chosen by hho_autotune: faster
    // for some large working sets, slower when the stage data stays in the last-level cache).
    int nt_stores = 0;
    // per-shot multipliers of dt (hho_set_dt_scale), [S] on the device; used when dt_scaled
    double *dt_scale = nullptr;
    bool dt_scaled = false;
    void *cfl_save = nullptr;  // entry states of hho_cfl_search
    AdjWork adj;
};

struct hho_batch {
    std::vector<hho_ctx *> ctxs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipGraphExec_t gexec[kNumGraphs] = {};  // kGraphSteps >> i steps of every context in gexec[i]
    std::vector<unsigned> versions;  // context versions the graphs were captured with
    // timing events around the graph replays of the last hho_batch_erk_step (on the launch stream)
    hipEvent_t t_begin = nullptr, t_end = nullptr;
    float last_ms = 0.0f;
    std::string err;
};

namespace {

std::string g_setup_error;

#define HCK(call)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                \
            return e_ == hipErrorOutOfMemory ? HHO_ERR_OOM : HHO_ERR_DEVICE;             \
        }                                                                                \
    } while (0)

hho_status dalloc(hho_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        ctx->err = "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? HHO_ERR_OOM : HHO_ERR_DEVICE;
    }
    ctx->allocs.push_back(*p);
    e = hipMemsetAsync(*p, 0, bytes, ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
        return HHO_ERR_DEVICE;
    }
    return HHO_OK;
}

// free an allocation made by dalloc (null-safe)
void dfree(hho_ctx *ctx, void *p) {
    if (!p) return;
    auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
    if (it != ctx->allocs.end()) ctx->allocs.erase(it);
    (void)hipFree(p);
}

template <typename T>
hho_status upload(hho_ctx *ctx, T **dst, const std::vector<T> &src) {
    hho_status s = dalloc(ctx, (void **)dst, src.size() * sizeof(T));
    if (s != HHO_OK) return s;
    if (!src.empty()) HCK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    HCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

// copy host data into an existing device array
template <typename T>
hho_status copy_in(hho_ctx *ctx, void *dst, const std::vector<T> &src) {
    if (!src.empty()) HCK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
    HCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

hho_status copy_in_real(hho_ctx *ctx, void *dst, const std::vector<double> &src) {
    if (ctx->dtype == 0) return copy_in(ctx, dst, src);
    std::vector<float> f(src.begin(), src.end());
    return copy_in(ctx, dst, f);
}

// real-typed upload of float64 host data
hho_status upload_real(hho_ctx *ctx, void **dst, const std::vector<double> &src) {
    if (ctx->dtype == 0) return upload(ctx, (double **)dst, src);
    std::vector<float> f(src.begin(), src.end());
    return upload(ctx, (float **)dst, f);
}

hho_status set_device(hho_ctx *ctx) {
    HCK(hipSetDevice(ctx->device));
    return HHO_OK;
}

// Coefficients of the stage recurrence Y_{i+1} = cU U + cY Y_i + ck dt k_i for the
// explicit tableaux of eq. ERK: row i+1 of A must be lam * (row i of A) on j < i.
//
// The stage buffers hold increments D_i = Y_{i+1} - U; U^{n+1} is formed without an accumulator:
// stage 1 (for s >= 3) stores Q = qa D_0 + qb D_1, and the last stage adds Q + cd D_{s-2} + b_s dt k_s.
struct StageCoef {
    double cU, cY, ck, cb, c;
    double qa, qb, cd;
    int q_write, q_read;
};

bool erk_coefficients(int s, std::vector<StageCoef> &out) {
    double A[4][4] = {{0}}, b[4] = {0}, c[4] = {0};
    if (s == 2) {
        A[1][0] = 0.5;
        b[0] = 0.0; b[1] = 1.0;
        c[1] = 0.5;
    } else if (s == 3) {
        A[1][0] = 0.5;
        A[2][0] = -1.0; A[2][1] = 2.0;
        b[0] = 1.0 / 6.0; b[1] = 2.0 / 3.0; b[2] = 1.0 / 6.0;
        c[1] = 0.5; c[2] = 1.0;
    } else if (s == 4) {
        A[1][0] = 0.5; A[2][1] = 0.5; A[3][2] = 1.0;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0;
        c[1] = 0.5; c[2] = 0.5; c[3] = 1.0;
    } else {
        return false;
    }
    out.assign(s, StageCoef{0, 0, 0, 0, 0, 0, 0, 0, 0, 0});
    for (int i = 0; i < s; ++i) {
        StageCoef &q = out[i];
        q.cb = b[i];
        q.c = c[i];
        if (i == s - 1) continue;
        q.ck = A[i + 1][i];
        if (i == 0) {
            q.cU = 1.0;
            q.cY = 0.0;
            continue;
        }
        int jm = 0;
        for (int j = 0; j < i; ++j)
            if (std::fabs(A[i][j]) > std::fabs(A[i][jm])) jm = j;
        const double lam = A[i][jm] != 0.0 ? A[i + 1][jm] / A[i][jm] : 0.0;
        for (int j = 0; j < i; ++j)
            if (std::fabs(A[i + 1][j] - lam * A[i][j]) > 1e-15) return false;
        q.cU = 1.0 - lam;
        q.cY = lam;
    }
    // increments D_i = Y_{i+1} - U (stage i, 0-based) satisfy D_i = cY_i D_{i-1} + ck_i dt k_i, so
    // dt k_i = (D_i - cY_i D_{i-1}) / ck_i and U^{n+1} = U + sum_m beta_m D_m + b_{s-1} dt k_{s-1}
    double beta[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m + 1 < s; ++m) {
        if (out[m].ck == 0.0) return false;
        beta[m] += out[m].cb / out[m].ck;
        if (m + 2 < s) beta[m] -= out[m + 1].cb * out[m + 1].cY / out[m + 1].ck;
    }
    StageCoef &L = out[s - 1];
    if (s >= 3) {
        // stage 1 folds D_0 and D_1 into Q; for s = 3 D_1 is also the last stage's input
        out[1].q_write = 1;
        out[1].qa = beta[0];
        out[1].qb = beta[1];
        L.q_read = 1;
        L.cd = s == 4 ? beta[2] : 0.0;
    } else {
        L.cd = beta[0];
    }
    if (s > 4) return false;
    return true;
}

unsigned arena_off(const void *arena, const void *p) {
    return p ? (unsigned)((const char *)p - (const char *)arena) : 0u;
}

// byte offsets of the per-stage arrays inside the arena the arguments address (a.arena)
template <typename R>
void set_stage_offsets(hho_ctx *, StageArgs<R> &a) {
    a.o_yin = arena_off(a.arena, a.Yin);
    a.o_yout = arena_off(a.arena, a.Yout);
    a.o_u = arena_off(a.arena, a.U);
    a.o_acc = arena_off(a.arena, a.acc);
    a.o_tin = arena_off(a.arena, a.Tin);
    a.o_tout = arena_off(a.arena, a.Tout);
    a.o_yq = arena_off(a.arena, a.Yq);
}

template <typename R>
StageArgs<R> base_args(hho_ctx *ctx) {
    StageArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.dim = ctx->plan.dim;
    a.link = ctx->link;
    a.c0 = (const R *)ctx->c0;
    a.mat = (const R *)ctx->mat;
    a.tab = (const R *)ctx->tab;
    a.ic_tab = ctx->ic_tab;
    a.has_pooled = ctx->plan.has_pooled ? 1 : 0;
    a.all_pooled = a.has_pooled;
    for (const auto &G : ctx->plan.groups) a.all_pooled &= G.pooled ? 1 : 0;
    a.groups = ctx->launch[ctx->shape].groups;
    a.blk_group = ctx->launch[ctx->shape].blk_group;
    a.n_ic = ctx->plan.n_ic;
    a.S = ctx->plan.S;
    a.cpb = ctx->launch[ctx->shape].cpb;
    a.clock = ctx->clock;
    a.LT = ctx->LT;
    a.emat = ctx->emat;
    a.arena = ctx->arena;
    a.arena_bytes = (unsigned)ctx->arena_bytes;
    a.o_link = arena_off(ctx->arena, ctx->link);
    a.o_c0 = arena_off(ctx->arena, ctx->c0);
    a.o_mat = arena_off(ctx->arena, ctx->mat);
    a.nt_stores = ctx->nt_stores;
    a.dt_scale = ctx->dt_scaled ? ctx->dt_scale : nullptr;
    return a;
}

template <int K, typename R>
hho_status compute_traces(hho_ctx *ctx, hipStream_t st = nullptr) {
    StageArgs<R> a = base_args<R>(ctx);
    a.Yin = (const R *)ctx->U;
    a.Tout = (R *)ctx->T[ctx->tcur];
    set_stage_offsets(ctx, a);
    HCK((launch_traces<K, R>(a, ctx->n_blocks(), st ? st : ctx->stream)));
    ctx->traces_valid = true;
    return HHO_OK;
}

template <int K, typename R>
hho_status energy_now(hho_ctx *ctx, double *out_dev) {
    StageArgs<R> a = base_args<R>(ctx);
    a.e_part = ctx->e_part;
    a.Yin = (const R *)ctx->U;
    set_stage_offsets(ctx, a);
    HCK((launch_energy<K, R>(a, (const R *)ctx->U, ctx->n_blocks(), ctx->stream)));
    HCK(launch_energy_reduce(ctx->e_part, ctx->n_blocks(), ctx->plan.S, out_dev, nullptr, 0, ctx->stream));
    return HHO_OK;
}

// Host-side check of one stage launch's arguments against the buffers they address (run for every
// launch enqueued or captured, before it is): every per-lane array inside the arena, the energy
// partials within the context's allocation, the recording capacities the kernels test against
// within the allocated histories, and the workgroup within the largest block.  A failure is an
// internal error reported as HHO_ERR_DEVICE; nothing is launched.
template <typename R>
hho_status check_stage_args(hho_ctx *ctx, const StageArgs<R> &a, int n_blocks, int ecap) {
    const size_t sbytes = (size_t)ctx->rows * ctx->LT * sizeof(R), tbytes = (size_t)ctx->trows * ctx->LT * sizeof(R);
    std::string bad;
    auto within = [&](const void *p, unsigned off, size_t bytes, const char *what) {
        if (p && (size_t)off + bytes > ctx->arena_bytes) bad = what;
    };
    within(a.Yin, a.o_yin, sbytes, "stage input");
    within(a.Yout, a.o_yout, sbytes, "stage output");
    within(a.U, a.o_u, sbytes, "state");
    within(a.Yq, a.o_yq, sbytes, "partial sum");
    within(a.Tin, a.o_tin, tbytes, "incoming traces");
    within(a.Tout, a.o_tout, tbytes, "outgoing traces");
    if (n_blocks > ctx->max_blocks || (size_t)a.cpb * a.S > (size_t)kBlock) bad = "launch shape";
    if (a.e_part && (a.e_part != ctx->e_part ||
                     (size_t)(std::max(a.e_slots, 1) - 1) * a.e_stride + (size_t)n_blocks * a.S > ctx->e_part_cap))
        bad = "energy partials";
    if ((size_t)std::max(ecap, 0) * a.S > ctx->e_hist_cap) bad = "energy history capacity";
    if (a.rec_first && (size_t)a.rec_steps * a.S * a.nrec * ctx->rec_w > ctx->rec_cap) bad = "receiver capacity";
    if (bad.empty()) return HHO_OK;
    ctx->err = "internal: stage launch argument out of its buffer (" + bad + ")";
    return HHO_ERR_DEVICE;
}

// Enqueue n_steps steps on stream st.  Every launch argument is the same for every step (the
// stage time and step index come from the device clock, advanced by the last stage of each step),
// so the sequence can be captured once into a graph and replayed.
//
// With `store` non-null (the adjoint's forward recompute), step n, stage i additionally writes the
// primal rows of Y_i, k_i and the face values of Y_i to slot n * s + i of `store`
// (AdjWork::slot_elems reals per slot); receivers and energy are not recorded then.
// Step n reads clock slot (parity + n) % 2; the caller names the slot that holds the current clock.
template <int K, typename R>
hho_status enqueue_steps(hho_ctx *ctx, hipStream_t st, int n_steps, R *store = nullptr, int parity = 0) {
    std::vector<StageCoef> co;
    if (!erk_coefficients(ctx->stages, co)) {
        ctx->err = "unsupported ERK stage count";
        return HHO_ERR_ARG;
    }
    const int s = ctx->stages, S = ctx->plan.S;
    StageArgs<R> a = base_args<R>(ctx);
    a.U = (R *)ctx->U;
    a.acc = (R *)ctx->acc;
    a.src_first = ctx->h_src.empty() ? nullptr : ctx->src_first;
    a.src = ctx->src;
    a.nterms = ctx->nterms;
    a.gload = (const R *)ctx->gload;
    for (int m = 0; m < ctx->nterms; ++m) {
        a.omega[m] = ctx->omega[m];
        a.phase[m] = ctx->phase[m];
    }
    a.nrec = ctx->nrec;
    a.rec_w = ctx->rec_w;
    a.rec_steps = ctx->nrec > 0 ? (int)(ctx->rec_cap / ((size_t)S * ctx->nrec * ctx->rec_w)) : 0;
    a.rec_out = ctx->rec_out;
    a.rec = ctx->rec;
    const int ecap = ctx->record_energy ? (int)(ctx->e_hist_cap / S) : 0;
    const int Tc = ctx->tcur, Ta = (Tc + 1) % 3, Tb = (Tc + 2) % 3;
    const int Tbuf[2] = {Ta, Tb};
    // stage increments D_0 .. D_{s-2} in three buffers, kept until the last stage
    void *stg[3] = {ctx->Y[0], ctx->Y[1], ctx->acc};
    for (int n = 0; n < n_steps; ++n) {
        for (int i = 0; i < s; ++i) {
            const StageCoef &q = co[i];
            a.first = i == 0;
            a.last = i == s - 1;
            a.Yin = i == 0 ? (const R *)ctx->U : (const R *)stg[i - 1];
            a.Yout = a.last ? nullptr : (R *)stg[i];
            a.qa = (R)q.qa;
            a.qb = (R)q.qb;
            a.cd = (R)q.cd;
            a.q_write = q.q_write;
            a.q_read = q.q_read;
            a.Yq = (q.q_write || q.q_read) ? (R *)stg[0] : nullptr;  // Q replaces D_0
            a.Tin = (const R *)ctx->T[i == 0 ? Tc : Tbuf[(i - 1) % 2]];
            a.Tout = (R *)ctx->T[a.last ? Tc : Tbuf[i % 2]];
            a.c = q.c;
            a.cU = (R)q.cU;
            a.cY = (R)q.cY;
            a.ck = (R)q.ck;
            a.cb = (R)q.cb;
            // energy partials of step n in slot n % kGraphSteps, summed after every kGraphSteps-th step
            a.e_part = (a.last && ctx->record_energy && !store) ? ctx->e_part : nullptr;
            a.e_slots = kGraphSteps;
            a.e_stride = (long long)ctx->n_blocks() * S;
            a.rec_first = (a.last && ctx->nrec > 0 && !store) ? ctx->rec_first : nullptr;
            a.clock = ctx->clock + ((parity + n) & 1);
            a.clock_next = ctx->clock + ((parity + n + 1) & 1);
            set_stage_offsets(ctx, a);
            if (hho_status cs = check_stage_args(ctx, a, ctx->n_blocks(), ecap)) return cs;
            if (store) {
                const AdjWork &w = ctx->adj;
                R *slot = store + (size_t)(n * s + i) * w.slot_elems;
                a.ystore = slot;
                a.kstore = slot + w.k_off;
                a.fstore = slot + w.f_off;
                HCK((launch_stage_store<K, R>(a, ctx->n_blocks(), st)));
            } else {
                HCK((launch_stage<K, R>(a, ctx->n_blocks(), st)));
            }
        }
        if (ctx->record_energy && !store && ((n + 1) % kGraphSteps == 0 || n == n_steps - 1)) {
            const int count = n - n / kGraphSteps * kGraphSteps + 1;  // steps since the last sum
            HCK(launch_energy_reduce_steps(ctx->e_part, ctx->n_blocks(), S, (long long)ctx->n_blocks() * S,
                                           kGraphSteps, ctx->e_hist, ctx->clock + ((parity + n) & 1), count, ecap,
                                           st));
        }
    }
    return HHO_OK;
}

// Entry points built for polygonal meshes only (point location, loads, the adjoint, the tabulated
// CFL step): ARG on a three-dimensional context.
hho_status two_dim_only(hho_ctx *ctx, const char *what) {
    ctx->err = std::string(what) + ": not available on a three-dimensional context";
    return HHO_ERR_ARG;
}

template <typename Fn>
hho_status dispatch(hho_ctx *ctx, Fn &&fn) {
    const int k = ctx->plan.k;
    if (ctx->dtype == 0) {
        if (k == 1) return fn(std::integral_constant<int, 1>(), (double *)nullptr);
        if (k == 2) return fn(std::integral_constant<int, 2>(), (double *)nullptr);
        return fn(std::integral_constant<int, 3>(), (double *)nullptr);
    }
    if (k == 1) return fn(std::integral_constant<int, 1>(), (float *)nullptr);
    if (k == 2) return fn(std::integral_constant<int, 2>(), (float *)nullptr);
    return fn(std::integral_constant<int, 3>(), (float *)nullptr);
}


template <int K, typename R>
hho_status autotune_shape(hho_ctx *ctx);

// Common start of a stepping call: output capacities, device clock, initial energy, traces.
// With defer, the initial energies are only enqueued (into ctx->h_e0): the caller synchronises
// the context's stream and reads them with read_initial_energy.
// Per-call histories (receiver rows, energies) sized for calls of up to n_steps steps; growing a
// device buffer bumps the context version, so that the graphs are captured again with it.
hho_status reserve_steps(hho_ctx *ctx, int n_steps) {
    const int S = ctx->plan.S;
    hho_status s;
    if (ctx->nrec > 0) {
        const size_t need = (size_t)S * std::max(n_steps, 1) * ctx->nrec * ctx->rec_w;
        if (need > ctx->rec_cap) {
            if ((s = dalloc(ctx, (void **)&ctx->rec_out, need * sizeof(double)))) return s;
            ctx->rec_cap = need;
            ctx->version++;
        }
    }
    if (ctx->record_energy) {
        const size_t need = (size_t)S * std::max(n_steps, 1);
        if (need > ctx->e_hist_cap) {
            if ((s = dalloc(ctx, (void **)&ctx->e_hist, need * sizeof(double)))) return s;
            ctx->e_hist_cap = need;
            ctx->version++;
        }
        if (!ctx->h_e0) HCK(hipHostMalloc((void **)&ctx->h_e0, (size_t)S * sizeof(double), hipHostMallocDefault));
        if (need > ctx->h_ehist_cap) {
            if (ctx->h_ehist) HCK(hipHostFree(ctx->h_ehist));
            ctx->h_ehist = nullptr;
            ctx->h_ehist_cap = 0;
            HCK(hipHostMalloc((void **)&ctx->h_ehist, need * sizeof(double), hipHostMallocDefault));
            ctx->h_ehist_cap = need;
        }
    }
    return HHO_OK;
}

hho_status begin_steps(hho_ctx *ctx, double t0, double dt, int n_steps, std::vector<double> &E0, bool defer = false) {
    const int S = ctx->plan.S;
    hho_status s = reserve_steps(ctx, n_steps);
    if (s != HHO_OK) return s;
    ctx->h_clock.t0 = t0;
    ctx->h_clock.dt = dt;
    ctx->h_clock.step = 0;
    HCK(hipMemcpyAsync(ctx->clock, &ctx->h_clock, sizeof(Clock), hipMemcpyHostToDevice, ctx->stream));
    ctx->last_steps = n_steps;
    E0.assign(S, 0.0);
    if (ctx->record_energy) {
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return energy_now<decltype(kc)::value, R>(ctx, ctx->e_now);
        });
        if (s != HHO_OK) return s;
        HCK(hipMemcpyAsync(ctx->h_e0, ctx->e_now, S * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        if (!defer) {
            HCK(hipStreamSynchronize(ctx->stream));
            std::copy(ctx->h_e0, ctx->h_e0 + S, E0.begin());
        }
    }
    if (!ctx->traces_valid) {
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return compute_traces<decltype(kc)::value, R>(ctx);
        });
        if (s != HHO_OK) return s;
    }
    return HHO_OK;
}

// Initial energies enqueued by begin_steps(defer = true), once the context's stream is synchronised.
void read_initial_energy(const hho_ctx *ctx, std::vector<double> &E0) {
    if (ctx->record_energy) std::copy(ctx->h_e0, ctx->h_e0 + ctx->plan.S, E0.begin());
}

// Enqueue the copy of the recorded energy history (n_steps steps) into ctx->h_ehist on `st`.
hho_status enqueue_history_copy(hho_ctx *ctx, int n_steps, hipStream_t st) {
    if (!ctx->record_energy || n_steps == 0) return HHO_OK;
    HCK(hipMemcpyAsync(ctx->h_ehist, ctx->e_hist, (size_t)n_steps * ctx->plan.S * sizeof(double),
                       hipMemcpyDeviceToHost, st));
    return HHO_OK;
}

// Energy criterion of Algorithm algo_CFL (Sec. 5.1) on the history copied into ctx->h_ehist:
// growth above 5 % over the initial or the previous energy of an undriven run, or a non-finite
// energy.
hho_status check_history(hho_ctx *ctx, int n_steps, const std::vector<double> &E0) {
    if (!ctx->record_energy || n_steps == 0) return HHO_OK;
    const int S = ctx->plan.S;
    const double *E = ctx->h_ehist;
    const bool driven = !ctx->h_src.empty() || ctx->nterms > 0;
    for (int sh = 0; sh < S; ++sh) {
        double prev = E0[sh];
        for (int n = 0; n < n_steps; ++n) {
            const double e = E[(size_t)n * S + sh];
            if (!std::isfinite(e) || (!driven && (e > 1.05 * E0[sh] + 1e-300 || e > 1.05 * prev + 1e-300))) {
                ctx->err = "energy of shot " + std::to_string(sh) +
                           " grew by more than 5 % (or is not finite) at step " + std::to_string(n);
                return HHO_ERR_UNSTABLE;
            }
            prev = e;
        }
    }
    return HHO_OK;
}

// Closing stability check of one context's stepping call (synchronises its stream).
hho_status end_steps(hho_ctx *ctx, int n_steps, const std::vector<double> &E0) {
    if (!ctx->record_energy || n_steps == 0) return HHO_OK;
    hho_status s = enqueue_history_copy(ctx, n_steps, ctx->stream);
    if (s != HHO_OK) return s;
    HCK(hipStreamSynchronize(ctx->stream));
    return check_history(ctx, n_steps, E0);
}

// Capture the step graphs of one context (cached until the configuration changes).  Every graph
// starts on clock slot 0; those of even length also end there, and the one-step graph, whose
// length is odd, is only ever replayed last in a call.
hho_status ensure_graphs(hho_ctx *ctx) {
    if (ctx->gexec[0] && ctx->graph_version == ctx->version) return HHO_OK;
    for (hipGraphExec_t &g : ctx->gexec) {
        if (g) HCK(hipGraphExecDestroy(g));
        g = nullptr;
    }
    for (int i = 0; i < kNumGraphs; ++i) {
        HCK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        hho_status s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return enqueue_steps<decltype(kc)::value, R>(ctx, ctx->cap_stream, kGraphSteps >> i);
        });
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (s != HHO_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        HCK(e);
        const hipError_t ei = hipGraphInstantiate(&ctx->gexec[i], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HCK(ei);
        // make the graph resident now, so that its first replay costs no more than the others
        HCK(hipGraphUpload(ctx->gexec[i], ctx->stream));
    }
    ctx->graph_version = ctx->version;
    return HHO_OK;
}

// Graph replays covering n steps: q full graphs, then one graph per set binary digit of the rest,
// largest first (so that the odd one-step graph comes last).  Calls launch(i) per replay.
template <typename F>
hho_status replay_steps(int n_steps, F &&launch) {
    for (int g = 0; g < n_steps / kGraphSteps; ++g)
        if (hho_status s = launch(0)) return s;
    const int rem = n_steps % kGraphSteps;
    for (int i = 1; i < kNumGraphs; ++i)
        if (rem & (kGraphSteps >> i))
            if (hho_status s = launch(i)) return s;
    return HHO_OK;
}

// One graph advancing every context of a batch by `steps` steps: the contexts' step chains are
// independent branches that fork from and join to one origin stream.
hho_status capture_batch(hho_batch *b, int steps, hipGraphExec_t *out) {
    const int n = (int)b->ctxs.size();
    hipStream_t origin = b->streams[n];
    auto fail = [&](const std::string &m, hho_status st) {
        b->err = m;
        return st;
    };
    if (hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail("batch: hipStreamBeginCapture failed", HHO_ERR_DEVICE);
    hho_status s = HHO_OK;
    if (hipEventRecord(b->events[n], origin) != hipSuccess) s = HHO_ERR_DEVICE;
    for (int i = 0; i < n && s == HHO_OK; ++i) {
        hho_ctx *ctx = b->ctxs[i];
        if (hipStreamWaitEvent(b->streams[i], b->events[n], 0) != hipSuccess) {
            s = HHO_ERR_DEVICE;
            break;
        }
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return enqueue_steps<decltype(kc)::value, R>(ctx, b->streams[i], steps);
        });
        if (s != HHO_OK) {
            b->err = ctx->err;
            break;
        }
        if (hipEventRecord(b->events[i], b->streams[i]) != hipSuccess ||
            hipStreamWaitEvent(origin, b->events[i], 0) != hipSuccess)
            s = HHO_ERR_DEVICE;
    }
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(origin, &graph);
    if (s != HHO_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return s != HHO_OK ? s : fail("batch: hipStreamEndCapture failed", HHO_ERR_DEVICE);
    }
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(std::string("batch: hipGraphInstantiate: ") + hipGetErrorString(ei), HHO_ERR_DEVICE);
    // resident now, so that the first replay costs no more than the others
    if (hipGraphUpload(*out, origin) != hipSuccess) return fail("batch: hipGraphUpload failed", HHO_ERR_DEVICE);
    return HHO_OK;
}

// Autotuner: time the stage kernel in each launch shape (stage-1 form: it reads U and the current
// traces and writes only scratch stage buffers) and keep the fastest.
template <int K, typename R>
hho_status autotune_shape(hho_ctx *ctx) {
    if (!ctx->traces_valid) {
        hho_status s = compute_traces<K, R>(ctx);
        if (s != HHO_OK) return s;
    }
    std::vector<StageCoef> co;
    if (!erk_coefficients(ctx->stages, co)) {
        ctx->err = "unsupported ERK stage count";
        return HHO_ERR_ARG;
    }
    ctx->h_clock = Clock{0.0, 0.0, 0, 0};
    HCK(hipMemcpyAsync(ctx->clock, &ctx->h_clock, sizeof(Clock), hipMemcpyHostToDevice, ctx->stream));
    hipEvent_t e0, e1;
    HCK(hipEventCreate(&e0));
    HCK(hipEventCreate(&e1));
    // Candidates: every launch shape with both store policies.  One pass = the stages before the
    // last of one step (they write only stage buffers and the two trace buffers that are not the
    // current one, so the state and its traces are unchanged).  Candidates take turns over several
    // rounds (so that clock and cache drift hit all of them alike) and each is ranked by the median
    // of its rounds.
    const int keep = ctx->shape, keep_nt = ctx->nt_stores;
    const int n_shape = (int)ctx->launch.size(), n_cand = 2 * n_shape, s = ctx->stages;
    constexpr int kRounds = 5, kPasses = 3;
    std::vector<std::vector<float>> times(n_cand);
    const int Tc = ctx->tcur, Tbuf[2] = {(Tc + 1) % 3, (Tc + 2) % 3};
    void *stg[3] = {ctx->Y[0], ctx->Y[1], ctx->acc};
    auto pass = [&](StageArgs<R> &a) -> bool {
        for (int i = 0; i < std::max(s - 1, 1); ++i) {
            const StageCoef &q = co[i];
            a.first = i == 0;
            a.last = 0;
            a.Yin = i == 0 ? (const R *)ctx->U : (const R *)stg[i - 1];
            a.Yout = (R *)stg[i];
            a.qa = (R)q.qa;
            a.qb = (R)q.qb;
            a.cd = (R)q.cd;
            a.q_write = q.q_write;
            a.q_read = 0;
            a.Yq = q.q_write ? (R *)stg[0] : nullptr;
            a.Tin = (const R *)ctx->T[i == 0 ? Tc : Tbuf[(i - 1) % 2]];
            a.Tout = (R *)ctx->T[Tbuf[i % 2]];
            a.c = q.c;
            a.cU = (R)q.cU;
            a.cY = (R)q.cY;
            a.ck = (R)q.ck;
            a.cb = (R)q.cb;
            set_stage_offsets(ctx, a);
            if (launch_stage<K, R>(a, ctx->n_blocks(), ctx->stream) != hipSuccess) return false;
        }
        return true;
    };
    hho_status st = HHO_OK;
    for (int round = 0; round < kRounds && st == HHO_OK; ++round) {
        for (int c = 0; c < n_cand && st == HHO_OK; ++c) {
            ctx->nt_stores = c / n_shape;
            ctx->shape = c % n_shape;
            StageArgs<R> a = base_args<R>(ctx);
            a.U = (R *)ctx->U;
            a.acc = (R *)ctx->acc;
            float ms = 0.f;
            if (!pass(a) || hipEventRecord(e0, ctx->stream) != hipSuccess) st = HHO_ERR_DEVICE;
            for (int p = 0; p < kPasses && st == HHO_OK; ++p)
                if (!pass(a)) st = HHO_ERR_DEVICE;
            if (st == HHO_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                                 hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = HHO_ERR_DEVICE;
            times[c].push_back(ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int best = keep, best_nt = keep_nt;
    if (st == HHO_OK) {
        float best_ms = 1e30f;
        for (int c = 0; c < n_cand; ++c) {
            std::vector<float> &t = times[c];
            std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
            if (t[t.size() / 2] < best_ms) {
                best_ms = t[t.size() / 2];
                best = c % n_shape;
                best_nt = c / n_shape;
            }
        }
    }
    ctx->shape = best;
    ctx->nt_stores = best_nt;
    if (best != keep || best_nt != keep_nt) ctx->version++;
    if (st != HHO_OK) ctx->err = "autotune: kernel launch or timing failed";
    return st;
}

hho_status rebuild_sources(hho_ctx *ctx) {
    std::vector<SrcDev> v = ctx->h_src;
    std::stable_sort(v.begin(), v.end(), [](const SrcDev &x, const SrcDev &y) { return x.ic < y.ic; });
    std::vector<int32_t> first(ctx->plan.n_ic, -1);
    for (size_t e = 0; e < v.size(); ++e) {
        v[e].next = (e + 1 < v.size() && v[e + 1].ic == v[e].ic) ? (int)e + 1 : -1;
        if (e == 0 || v[e - 1].ic != v[e].ic) first[v[e].ic] = (int)e;
    }
    if (!ctx->src_first) {
        hho_status s = dalloc(ctx, (void **)&ctx->src_first, first.size() * sizeof(int32_t));
        if (s != HHO_OK) return s;
    }
    if (v.size() > ctx->src_cap) {
        hho_status s = dalloc(ctx, (void **)&ctx->src, v.size() * sizeof(SrcDev));
        if (s != HHO_OK) return s;
        ctx->src_cap = v.size();
    }
    HCK(hipMemcpyAsync(ctx->src_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       ctx->stream));
    if (!v.empty())
        HCK(hipMemcpyAsync(ctx->src, v.data(), v.size() * sizeof(SrcDev), hipMemcpyHostToDevice, ctx->stream));
    HCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}


// Geometric corners of a cell: the vertices where its boundary turns.  A hanging node lies on a
// straight edge and is not a corner, so a square with hanging nodes counts 4 and a triangle with
// one counts 3.
int geometric_corners(const Plan &P, int c) {
    const int b = P.cell_ptr[c], n = P.cell_ptr[c + 1] - b;
    int corners = 0;
    for (int i = 0; i < n; ++i) {
        const int v0 = P.cell_vtx[b + (i + n - 1) % n], v1 = P.cell_vtx[b + i], v2 = P.cell_vtx[b + (i + 1) % n];
        const double ax = P.xy[2 * v1] - P.xy[2 * v0], ay = P.xy[2 * v1 + 1] - P.xy[2 * v0 + 1];
        const double bx = P.xy[2 * v2] - P.xy[2 * v1], by = P.xy[2 * v2 + 1] - P.xy[2 * v1 + 1];
        const double cross = ax * by - ay * bx;
        if (std::fabs(cross) > 1e-9 * std::sqrt((ax * ax + ay * ay) * (bx * bx + by * by))) ++corners;
    }
    return corners;
}

// CFL-limited time step (eq. CFL, Sec. 5.1): min over cells of CFL*(s, k, shape) h_T / c_T, with
// c_T the largest wave speed of the cell (c, or c_P in the solid), the shape from the cell's
// geometric corners (3: triangle, 4: quadrilateral, 5 or more: polygon, hexagon column) and h_T
// the side of the generating square (sqrt of the area; sqrt of twice the area for triangles).
// CFL* is the paper's Table tab::ratio_geo value, lowered to 0.9 times this discretisation's own
// stability limit where that is smaller, so that factor 1 is stable on every shape.  Those limits
// were measured with hho_cfl_search (Algorithm algo_CFL from a random state, which excites every
// mode, T_f = 1, delta = 1 %) on the two-material CFL geometry at h = 1/16 (squares, the squares
// cut along a diagonal, and hexagons), with the weights eta^f = 0.8, eta^s = 1.5 and both readings
// of the solid stabilisation speed; with other weights the limit moves (hho_cfl_search measures it).
double cfl_time_step(const Plan &P, int stages) {
    static const double paper[3][3][3] = {
        // s = 2: triangle, square, hexagon for k = 1, 2, 3
        {{0.191, 0.106, 0.072}, {0.205, 0.099, 0.063}, {0.264, 0.136, 0.082}},
        // s = 3
        {{0.238, 0.133, 0.090}, {0.253, 0.123, 0.079}, {0.329, 0.170, 0.102}},
        // s = 4
        {{0.265, 0.147, 0.100}, {0.282, 0.138, 0.087}, {0.363, 0.188, 0.115}},
    };
    // measured limits [stab_speed][s - 2][shape][k - 1]
    static const double measured[2][3][3][3] = {
        {{{0.0979, 0.0540, 0.0360}, {0.1680, 0.0871, 0.0585}, {0.0946, 0.0509, 0.0331}},
         {{0.1232, 0.0678, 0.0454}, {0.2099, 0.1087, 0.0733}, {0.1188, 0.0636, 0.0415}},
         {{0.1358, 0.0751, 0.0504}, {0.2329, 0.1210, 0.0817}, {0.1317, 0.0705, 0.0460}}},
        {{{0.1732, 0.0979, 0.0628}, {0.2857, 0.1459, 0.0909}, {0.1723, 0.0946, 0.0618}},
         {{0.2165, 0.1226, 0.0792}, {0.3553, 0.1823, 0.1140}, {0.2148, 0.1188, 0.0776}},
         {{0.2410, 0.1352, 0.0880}, {0.3959, 0.2023, 0.1265}, {0.2386, 0.1311, 0.0854}}},
    };
    double dt = 1e300;
    for (int c = 0; c < P.n_cells; ++c) {
        const int corners = geometric_corners(P, c);
        const int shape = corners <= 3 ? 0 : (corners == 4 ? 1 : 2);
        const double h = std::sqrt(P.area[c] * (shape == 0 ? 2.0 : 1.0));
        const double cfl = std::min(paper[stages - 2][shape][P.k - 1],
                                    0.9 * measured[P.stab_speed ? 1 : 0][stages - 2][shape][P.k - 1]);
        // c (fluid: kappa / rho = c^2) or c_P (solid: (lambda + 2 mu) / rho)
        const int ic = P.ic_of_cell[c];
        const double speed = std::sqrt(P.mat[(size_t)kStiff * P.n_ic + ic] * P.mat[(size_t)kInvRho * P.n_ic + ic]);
        dt = std::min(dt, cfl * h / speed);
    }
    return dt;
}

// ----------------------------------------------------------------------------- discrete adjoint

// Allocate (or grow) the adjoint workspace for segments of `every` steps and n_seg checkpoints.
hho_status ensure_adjoint(hho_ctx *ctx, int every, int n_seg) {
    AdjWork &w = ctx->adj;
    const Plan &P = ctx->plan;
    const size_t LT = (size_t)ctx->LT, rs = ctx->rsize;
    const size_t sbytes = (size_t)ctx->rows * LT * rs;
    hho_status s;
    if (!w.arena) {
        const size_t tbytes = (size_t)ctx->trows * LT * rs;
        const size_t lbytes = (size_t)P.max_nf * P.n_ic * 4;
        const size_t cbytes = (size_t)P.max_nf * P.n_ic * rs;
        const size_t mbytes = (size_t)kNumMat * P.n_ic * rs;
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t total = 4 * al(sbytes) + 2 * al(tbytes) + al(lbytes) + al(cbytes) + al(mbytes);
        if ((s = dalloc(ctx, &w.arena, total))) return s;
        w.arena_bytes = total;
        char *p = (char *)w.arena;
        auto take = [&](size_t b) {
            void *q = p;
            p += al(b);
            return q;
        };
        w.lam = take(sbytes);
        w.Z[0] = take(sbytes);
        w.Z[1] = take(sbytes);
        w.acc = take(sbytes);
        w.T[0] = take(tbytes);
        w.T[1] = take(tbytes);
        w.link = (int32_t *)take(lbytes);
        w.c0 = take(cbytes);
        w.mat = take(mbytes);
        HCK(hipMemcpyAsync(w.link, ctx->link, lbytes, hipMemcpyDeviceToDevice, ctx->stream));
        HCK(hipMemcpyAsync(w.c0, ctx->c0, cbytes, hipMemcpyDeviceToDevice, ctx->stream));
        HCK(hipMemcpyAsync(w.mat, ctx->mat, mbytes, hipMemcpyDeviceToDevice, ctx->stream));
        const size_t N = P.N;
        w.k_off = 2 * N * LT;
        w.f_off = 7 * N * LT;
        w.slot_elems = (7 * N + ctx->trows) * LT;
        std::vector<int32_t> ic(P.ic_of_cell.begin(), P.ic_of_cell.end());
        if ((s = dalloc(ctx, (void **)&w.gacc, 3 * LT * sizeof(double))) || (s = upload(ctx, &w.gm, P.gm)) ||
            (s = dalloc(ctx, (void **)&w.grad, 3 * (size_t)std::max(1, P.n_cells) * sizeof(double))) ||
            (s = upload(ctx, &w.ic_of_cell, ic)))
            return s;
    }
    if (!w.aux) {
        HCK(hipStreamCreateWithFlags(&w.aux, hipStreamNonBlocking));
        HCK(hipEventCreateWithFlags(&w.ev_start, hipEventDisableTiming));
        for (int b = 0; b < 2; ++b) {
            HCK(hipEventCreateWithFlags(&w.ev_rec[b], hipEventDisableTiming));
            HCK(hipEventCreateWithFlags(&w.ev_adj[b], hipEventDisableTiming));
        }
        if ((s = dalloc(ctx, (void **)&w.aclock, sizeof(Clock)))) return s;
    }
    const size_t slots = (size_t)every * ctx->stages;
    if (slots > w.store_slots) {
        for (int b = 0; b < 2; ++b) {
            dfree(ctx, w.store[b]);
            w.store[b] = nullptr;
        }
        w.store_slots = 0;
        for (int b = 0; b < 2; ++b)
            if ((s = dalloc(ctx, &w.store[b], slots * w.slot_elems * rs))) return s;
        w.store_slots = slots;
    }
    if ((size_t)n_seg + 1 > w.ckpt_states) {
        dfree(ctx, w.ckpt);
        w.ckpt = nullptr;
        w.ckpt_states = 0;
        if ((s = dalloc(ctx, &w.ckpt, ((size_t)n_seg + 1) * sbytes))) return s;
        w.ckpt_states = (size_t)n_seg + 1;
    }
    return HHO_OK;
}

// Reverse sweep (see adjoint.hip): terminal misfit derivative, then for every checkpoint segment
// from the last, the forward recompute with stores and the adjoint stages of its steps in reverse.
template <int K, typename R>
hho_status adjoint_sweep(hho_ctx *ctx, const std::vector<StageCoef> &co, int every, int n_seg, int n_steps,
                         double t0, double dt, std::vector<Clock> &clocks) {
    AdjWork &w = ctx->adj;
    const int s = ctx->stages;
    const size_t sbytes = (size_t)ctx->rows * ctx->LT * ctx->rsize;
    StageArgs<R> a = base_args<R>(ctx);
    a.arena = w.arena;
    a.arena_bytes = (unsigned)w.arena_bytes;
    a.link = w.link;
    a.c0 = (const R *)w.c0;
    a.mat = (const R *)w.mat;
    a.o_link = arena_off(w.arena, w.link);
    a.o_c0 = arena_off(w.arena, w.c0);
    a.o_mat = arena_off(w.arena, w.mat);
    a.U = (R *)w.lam;
    a.acc = (R *)w.acc;
    a.gacc = w.gacc;
    a.gm = w.gm;
    a.rec_first = ctx->nrec > 0 ? ctx->rec_first : nullptr;
    a.rec = ctx->rec;
    a.nrec = ctx->nrec;
    a.dobs = w.dobs;
    a.nobs = n_steps;
    a.zs_b = (R)(dt * co[s - 1].cb);
    // lambda^N = dJ/dU^N, z for the last stage of the last step
    a.yfwd = (const R *)ctx->U;
    a.Yout = (R *)w.Z[0];
    a.Tout = (R *)w.T[0];
    a.inject = n_steps;
    // the adjoint kernels read dt, and the offset of the injected step, from a clock of their own
    w.h_aclock = Clock{t0, dt, 0, 0};
    HCK(hipMemcpyAsync(w.aclock, &w.h_aclock, sizeof(Clock), hipMemcpyHostToDevice, ctx->stream));
    a.clock = w.aclock;
    set_stage_offsets(ctx, a);
    HCK((launch_adjoint_start<K, R>(a, ctx->n_blocks(), ctx->stream)));
    // The adjoint stages of one segment, from the last step back (stage inputs alternate between
    // Z[0] and Z[1]; s * len stages per segment is even, so every segment starts on Z[0]).  The step
    // whose misfit enters lambda is the segment's first step plus the relative index in a.inject.
    auto adjoint_stages = [&](const R *store, int len, hipStream_t st) -> hho_status {
        int cur = 0;
        for (int n = len - 1; n >= 0; --n) {
            for (int i = s - 1; i >= 0; --i) {
                const R *slot = store + (size_t)(n * s + i) * w.slot_elems;
                a.yfwd = slot;
                a.kfwd = slot + w.k_off;
                a.ffwd = slot + w.f_off;
                a.Yin = (const R *)w.Z[cur];
                a.Yout = (R *)w.Z[1 - cur];
                a.Tin = (const R *)w.T[cur];
                a.Tout = (R *)w.T[1 - cur];
                a.first = i == s - 1;
                a.last = i == 0;
                a.mu_b = i > 0 ? (R)(dt * co[i - 1].cb) : R(0);
                a.mu_a = i > 0 ? (R)(dt * co[i - 1].ck) : R(0);
                a.inject = i == 0 ? n + 1 : 0;
                set_stage_offsets(ctx, a);
                HCK((launch_adjoint_stage<K, R>(a, ctx->n_blocks(), st)));
                cur ^= 1;
            }
        }
        return HHO_OK;
    };
    // Graphs of a full segment (every steps) for both store buffers, captured once per key.
    const void *key[4] = {w.store[0], w.store[1], w.dobs, w.arena};
    bool fresh = w.rec_graph[0] && w.g_every == every && w.g_steps == n_steps && w.g_dt == dt &&
                 w.g_version == ctx->version;
    for (int q = 0; q < 4 && fresh; ++q) fresh = key[q] == w.g_key[q];
    if (!fresh) {
        for (int b = 0; b < 2; ++b) {
            if (w.rec_graph[b]) HCK(hipGraphExecDestroy(w.rec_graph[b]));
            if (w.adj_graph[b]) HCK(hipGraphExecDestroy(w.adj_graph[b]));
            w.rec_graph[b] = w.adj_graph[b] = nullptr;
        }
        auto capture = [&](hipGraphExec_t *out, auto &&body) -> hho_status {
            HCK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            hho_status st = body();
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
            if (st != HHO_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            HCK(e);
            const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HCK(ei);
            HCK(hipGraphUpload(*out, ctx->stream));
            return HHO_OK;
        };
        for (int b = 0; b < 2; ++b) {
            hho_status st = capture(&w.rec_graph[b], [&]() {
                return enqueue_steps<K, R>(ctx, ctx->cap_stream, every, (R *)w.store[b]);
            });
            if (st == HHO_OK)
                st = capture(&w.adj_graph[b], [&]() { return adjoint_stages((const R *)w.store[b], every, ctx->cap_stream); });
            if (st != HHO_OK) return st;
        }
        w.g_every = every;
        w.g_steps = n_steps;
        w.g_dt = dt;
        w.g_version = ctx->version;
        for (int q = 0; q < 4; ++q) w.g_key[q] = key[q];
    }
    // Segments from the last: the forward recompute of segment g - 1 (stream aux: the forward
    // state, traces and clock of the context, store buffer (g - 1) % 2) runs while the adjoint
    // stages of segment g (the caller's stream: the adjoint arena, store buffer g % 2) run.
    // Events order the recompute of a segment before its adjoint stages, and the adjoint stages
    // that read a store buffer before the recompute that overwrites it.
    HCK(hipEventRecord(w.ev_start, ctx->stream));  // the start kernel has read U^N
    HCK(hipStreamWaitEvent(w.aux, w.ev_start, 0));
    bool adj_pending[2] = {false, false};
    auto recompute = [&](int g) -> hho_status {
        const int b = g % 2, n0 = g * every, len = std::min(every, n_steps - n0);
        if (adj_pending[b]) HCK(hipStreamWaitEvent(w.aux, w.ev_adj[b], 0));
        HCK(hipMemcpyAsync(ctx->U, (char *)w.ckpt + (size_t)g * sbytes, sbytes, hipMemcpyDeviceToDevice, w.aux));
        hho_status st = compute_traces<K, R>(ctx, w.aux);
        if (st != HHO_OK) return st;
        clocks[g] = Clock{t0, dt, n0, 0};
        HCK(hipMemcpyAsync(ctx->clock, &clocks[g], sizeof(Clock), hipMemcpyHostToDevice, w.aux));
        if (len == every) HCK(hipGraphLaunch(w.rec_graph[b], w.aux));
        else if ((st = enqueue_steps<K, R>(ctx, w.aux, len, (R *)w.store[b]))) return st;
        HCK(hipEventRecord(w.ev_rec[b], w.aux));
        return HHO_OK;
    };
    hho_status st = recompute(n_seg - 1);
    if (st != HHO_OK) return st;
    std::vector<int> offset(n_seg);
    for (int g = n_seg - 1; g >= 0; --g) {
        const int b = g % 2, n0 = g * every, len = std::min(every, n_steps - n0);
        HCK(hipStreamWaitEvent(ctx->stream, w.ev_rec[b], 0));
        if (g > 0 && (st = recompute(g - 1)) != HHO_OK) return st;
        // the adjoint clock's step: the offset of the segment's injected steps (n0 + n = n + 1 + offset)
        offset[g] = n0 - 1;
        HCK(hipMemcpyAsync(&w.aclock->step, &offset[g], sizeof(int), hipMemcpyHostToDevice, ctx->stream));
        if (len == every) HCK(hipGraphLaunch(w.adj_graph[b], ctx->stream));
        else if ((st = adjoint_stages((const R *)w.store[b], len, ctx->stream))) return st;
        HCK(hipEventRecord(w.ev_adj[b], ctx->stream));
        adj_pending[b] = true;
    }
    // the host-side values the copies above read stay alive until the stream has consumed them
    HCK(hipStreamSynchronize(ctx->stream));
    HCK(hipStreamSynchronize(w.aux));
    return HHO_OK;
}

// Steps of hho_erk_step without the closing stability check, all from captured graphs.
// E0 receives the initial energies when recorded.
hho_status run_steps(hho_ctx *ctx, double t0, double dt, int n_steps, std::vector<double> &E0) {
    hho_status s;
    if ((s = begin_steps(ctx, t0, dt, n_steps, E0))) return s;
    if (n_steps == 0) return HHO_OK;
    if ((s = ensure_graphs(ctx))) return s;
    return replay_steps(n_steps, [&](int i) -> hho_status {
        HCK(hipGraphLaunch(ctx->gexec[i], ctx->stream));
        return HHO_OK;
    });
}

}  // namespace

namespace hho {

int ctx_device(const hho_ctx *ctx) { return ctx->device; }

void ctx_set_error(hho_ctx *ctx, const std::string &msg) { ctx->err = msg; }

hho_status energy_into(hho_ctx *ctx, double *part, size_t cap, double *out) {
    const size_t need = (size_t)ctx->n_blocks() * (size_t)ctx->plan.S;
    if (need > cap) {
        ctx->err = "energy: " + std::to_string(need) + " partial sums (blocks x shots) exceed the scratch capacity of " +
                   std::to_string(cap);
        return HHO_ERR_ARG;
    }
    return dispatch(ctx, [&](auto kc, auto *r) -> hho_status {
        using R = std::remove_pointer_t<decltype(r)>;
        StageArgs<R> a = base_args<R>(ctx);
        a.e_part = part;
        a.Yin = (const R *)ctx->U;
        set_stage_offsets(ctx, a);
        HCK((launch_energy<decltype(kc)::value, R>(a, (const R *)ctx->U, ctx->n_blocks(), ctx->stream)));
        HCK(launch_energy_reduce(part, ctx->n_blocks(), ctx->plan.S, out, nullptr, 0, ctx->stream));
        return HHO_OK;
    });
}

}  // namespace hho

// Runs one C ABI call; a C++ exception (a failed host allocation, above all) becomes a status
// code and a message instead of crossing the ABI.
template <typename F>
hho_status guarded(std::string *err, F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        if (err) *err = "host memory allocation failed";
        return HHO_ERR_OOM;
    } catch (const std::exception &e) {
        if (err) *err = std::string("internal error: ") + e.what();
        return HHO_ERR_DEVICE;
    } catch (...) {
        if (err) *err = "internal error";
        return HHO_ERR_DEVICE;
    }
}

namespace {

// Device side of hho_setup / hho_setup3d once the context's plan is built: buffers, uploads,
// launch shapes, capture stream.  On failure the context is destroyed and the message kept as
// the setup error.
hho_status setup_device(hho_ctx *ctx, const hho_params *prm, hho_ctx **out) {
    auto fail = [&](hho_status s) {
        g_setup_error = ctx->err;
        hho_destroy(ctx);
        return s;
    };
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return fail(s);
    Plan &P = ctx->plan;
    ctx->rec_w = P.dim == 3 ? 3 : 2;
    ctx->LT = (long long)P.n_ic * P.S;
    ctx->rows = P.rows_s * P.N;
    ctx->trows = trace_rows(P);
    const size_t sbytes = (size_t)ctx->rows * ctx->LT * ctx->rsize;
    const size_t tbytes = (size_t)ctx->trows * ctx->LT * ctx->rsize;
    const size_t lbytes = (size_t)P.max_nf * P.n_ic * 4;
    const size_t cbytes = (size_t)P.max_nf * P.n_ic * ctx->rsize;
    const size_t mbytes = (size_t)kNumMat * P.n_ic * ctx->rsize;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t total = 4 * al(sbytes) + 3 * al(tbytes) + al(lbytes) + al(cbytes) + al(mbytes);
    // the kernels address the arena through one buffer resource with 32-bit byte offsets
    if (total >= (1ull << 32)) {
        ctx->err = "cells x shots too large for one context (arena of " + std::to_string(total) +
                   " bytes exceeds 4 GiB)";
        return fail(HHO_ERR_ARG);
    }
    if ((s = dalloc(ctx, &ctx->arena, total))) return fail(s);
    ctx->arena_bytes = total;
    {
        char *p = (char *)ctx->arena;
        auto take = [&](size_t b) {
            void *q = p;
            p += al(b);
            return q;
        };
        ctx->U = take(sbytes);
        ctx->Y[0] = take(sbytes);
        ctx->Y[1] = take(sbytes);
        ctx->acc = take(sbytes);
        for (int i = 0; i < 3; ++i) ctx->T[i] = take(tbytes);
        ctx->link = (int32_t *)take(lbytes);
        ctx->c0 = take(cbytes);
        ctx->mat = take(mbytes);
    }
    std::vector<int64_t> map(P.n_ext);
    for (int c = 0; c < P.n_cells; ++c) {
        const int nr = (P.medium[c] == kFluid ? P.rows_f : P.rows_s) * P.N;
        for (int r = 0; r < nr; ++r)
            map[P.ext_off[c] + r] = (int64_t)r * ctx->LT + (int64_t)P.ic_of_cell[c] * P.S;
    }
    if ((s = copy_in(ctx, ctx->link, P.link)) || (s = copy_in_real(ctx, ctx->c0, P.c0)) ||
        (s = copy_in_real(ctx, ctx->mat, P.mat)) || (s = upload_real(ctx, &ctx->tab, P.tables)) ||
        (s = upload(ctx, &ctx->emat, P.emat)) || (s = upload(ctx, &ctx->map, map)) ||
        (s = upload(ctx, &ctx->ic_tab, P.ic_tab)) ||
        (s = dalloc(ctx, (void **)&ctx->staging, std::max<size_t>(1, P.n_ext) * 4 * sizeof(double))) ||
        (s = dalloc(ctx, (void **)&ctx->e_now, (size_t)P.S * sizeof(double))) ||
        (s = dalloc(ctx, (void **)&ctx->clock, 2 * sizeof(Clock))))
        return fail(s);
    for (const Plan::Launch &L : P.launches) {
        std::vector<GroupDev> gd;
        for (size_t g = 0; g < P.groups.size(); ++g) {
            const Group &G = P.groups[g];
            gd.push_back({G.medium, G.nF, G.tab_off, G.ic_begin, G.ncells, L.blk_begin[g], G.pooled ? 1 : 0});
        }
        hho_ctx::LaunchDev d;
        d.n_blocks = (int)L.blk_group.size();
        d.cpb = L.cpb;
        d.lanes = L.lanes;
        if ((s = upload(ctx, &d.groups, gd)) || (s = upload(ctx, &d.blk_group, L.blk_group))) return fail(s);
        ctx->launch.push_back(d);
        ctx->max_blocks = std::max(ctx->max_blocks, d.n_blocks);
    }
    ctx->e_part_cap = (size_t)kGraphSteps * ctx->max_blocks * P.S;
    if ((s = dalloc(ctx, (void **)&ctx->e_part, ctx->e_part_cap * sizeof(double)))) return fail(s);
    ctx->cfl_dt = P.dim == 2 ? cfl_time_step(P, prm->rk_stages) : 0.0;
    {
        hipError_t e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ctx->err = std::string("hipStreamCreate: ") + hipGetErrorString(e);
            return fail(HHO_ERR_DEVICE);
        }
    }
    {
        const std::string m = noalloc_init(ctx->device);
        if (!m.empty()) {
            ctx->err = m;
            return fail(HHO_ERR_DEVICE);
        }
    }
    *out = ctx;
    return HHO_OK;
}

// Checks of the parameters shared by both dimensions; creates the context (plan not built).
hho_status new_context(const hho_params *prm, hho_ctx **ctx_out) {
    if (prm->dtype != 0 && prm->dtype != 1) {
        g_setup_error = "dtype must be 0 (float64) or 1 (float32)";
        return HHO_ERR_ARG;
    }
    std::vector<StageCoef> co;
    if (!erk_coefficients(prm->rk_stages, co)) {
        g_setup_error = "rk_stages must be 2, 3 or 4";
        return HHO_ERR_ARG;
    }
    hho_ctx *ctx = new hho_ctx();
    ctx->dtype = prm->dtype;
    ctx->stages = prm->rk_stages;
    ctx->record_energy = prm->record_energy ? 1 : 0;
    ctx->device = prm->device;
    ctx->stream = (hipStream_t)prm->stream;
    ctx->rsize = prm->dtype == 0 ? 8 : 4;
    *ctx_out = ctx;
    return HHO_OK;
}

}  // namespace

extern "C" {

const char *hho_last_error(const hho_ctx *ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

hho_status hho_setup(const hho_mesh *mesh, const hho_params *prm, hho_ctx **out) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        g_setup_error.clear();
        if (!out) return HHO_ERR_ARG;
        *out = nullptr;
        if (!mesh || !prm) {
            g_setup_error = "null mesh or params";
            return HHO_ERR_ARG;
        }
        hho_ctx *ctx = nullptr;
        if (hho_status s = new_context(prm, &ctx)) return s;
        int code = 0;
        std::string msg = build_plan(mesh->n_vertices, mesh->xy, mesh->n_cells, mesh->cell_ptr, mesh->cell_vtx,
                                     mesh->medium, mesh->rho, mesh->a, mesh->b, prm->k, prm->eta_f, prm->eta_s,
                                     prm->stab_speed, prm->n_shots, ctx->plan, &code);
        if (code != 0) {
            g_setup_error = msg;
            delete ctx;
            return (hho_status)code;
        }
        return setup_device(ctx, prm, out);
    });
}

hho_status hho_setup3d(const hho_mesh3d *mesh, const hho_params *prm, hho_ctx **out) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        g_setup_error.clear();
        if (!out) return HHO_ERR_ARG;
        *out = nullptr;
        if (!mesh || !prm) {
            g_setup_error = "null mesh or params";
            return HHO_ERR_ARG;
        }
        hho_ctx *ctx = nullptr;
        if (hho_status s = new_context(prm, &ctx)) return s;
        int code = 0;
        std::string msg = build_plan3d(mesh->n_vertices, mesh->xyz, mesh->n_cells, mesh->cell_ptr, mesh->cell_vtx,
                                       mesh->medium, mesh->rho, mesh->a, mesh->b, prm->k, prm->eta_f, prm->eta_s,
                                       prm->stab_speed, prm->n_shots, ctx->plan, &code);
        if (code != 0) {
            g_setup_error = msg;
            delete ctx;
            return (hho_status)code;
        }
        return setup_device(ctx, prm, out);
    });
}

void hho_destroy(hho_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (hipGraphExec_t g : ctx->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->h_e0) (void)hipHostFree(ctx->h_e0);
    if (ctx->h_ehist) (void)hipHostFree(ctx->h_ehist);
    AdjWork &w = ctx->adj;
    for (int b = 0; b < 2; ++b) {
        if (w.rec_graph[b]) (void)hipGraphExecDestroy(w.rec_graph[b]);
        if (w.adj_graph[b]) (void)hipGraphExecDestroy(w.adj_graph[b]);
    }
    if (w.aux) {
        (void)hipStreamSynchronize(w.aux);
        (void)hipStreamDestroy(w.aux);
    }
    for (hipEvent_t e : {w.ev_start, w.ev_rec[0], w.ev_rec[1], w.ev_adj[0], w.ev_adj[1]})
        if (e) (void)hipEventDestroy(e);
    for (void *p : ctx->allocs) (void)hipFree(p);
    delete ctx;
}

hho_status hho_sizes(const hho_ctx *ctx, int64_t *n_dof, int32_t *n_cells, int32_t *n_faces) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n_dof) *n_dof = ctx->plan.n_ext;
        if (n_cells) *n_cells = ctx->plan.n_cells;
        if (n_faces) *n_faces = ctx->plan.n_faces;
        return HHO_OK;
    });
}

hho_status hho_set_state(hho_ctx *ctx, int32_t shot, const double *U, int32_t on_device) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!U || shot < 0 || shot >= ctx->plan.S) {
            ctx->err = "set_state: null pointer or shot out of range";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const long long n = ctx->plan.n_ext;
        const double *src = U;
        if (!on_device) {
            HCK(hipMemcpyAsync(ctx->staging, U, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
            src = ctx->staging;
        }
        if (ctx->dtype == 0) HCK(launch_scatter<double>(src, ctx->map, n, shot, (double *)ctx->U, ctx->stream));
        else HCK(launch_scatter<float>(src, ctx->map, n, shot, (float *)ctx->U, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        ctx->traces_valid = false;
        return HHO_OK;
    });
}

hho_status hho_set_ricker_ic(hho_ctx *ctx, int32_t shot, double xc, double yc, double theta, double lambda,
                             int32_t field) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (ctx->plan.dim != 2) return two_dim_only(ctx, "set_ricker_ic");
        if (shot < 0 || shot >= ctx->plan.S || !(lambda > 0.0) || !std::isfinite(lambda) || !std::isfinite(xc) ||
            !std::isfinite(yc) || !std::isfinite(theta) || (field != 0 && field != 1)) {
            ctx->err = "set_ricker_ic: shot out of range, lambda <= 0, a non-finite value or field not 0 / 1";
            return HHO_ERR_ARG;
        }
        const Plan &P = ctx->plan;
        const RickerIC ic{xc, yc, theta, lambda, field};
        // graded exponents of the scaled monomials (degree-major, decreasing power of x)
        int px[kMaxN], py[kMaxN];
        for (int d = 0, m = 0; d <= P.k; ++d)
            for (int a = d; a >= 0; --a, ++m) {
                px[m] = a;
                py[m] = d - a;
            }
        std::vector<double> U((size_t)P.n_ext, 0.0);
        for (int c = 0; c < P.n_cells; ++c) {
            const double h = P.hT[c], cx = P.centroid[2 * c], cy = P.centroid[2 * c + 1];
            const double *C = P.basisC.data() + (size_t)P.cell_class[c] * P.N * P.N;
            auto eval = [&](double x, double y, double *phi) {
                const double X = (x - cx) / h, Y = (y - cy) / h;
                double mu[kMaxN];
                for (int m = 0; m < P.N; ++m) mu[m] = std::pow(X, px[m]) * std::pow(Y, py[m]);
                for (int a = 0; a < P.N; ++a) {
                    double v = 0.0;
                    for (int m = 0; m <= a; ++m) v += C[a * P.N + m] * mu[m];
                    phi[a] = v;
                }
            };
            const int b = P.cell_ptr[c];
            project_ricker_cell(ic, P.xy.data(), P.cell_vtx.data() + b, P.cell_ptr[c + 1] - b, cx, cy,
                                P.medium[c] == kFluid, P.N, P.N, P.N, eval, U.data() + P.ext_off[c]);
        }
        const hho_status s = hho_set_state(ctx, shot, U.data(), 0);
        return s;
    });
}

hho_status hho_get_state(hho_ctx *ctx, int32_t shot, double *U, int32_t on_device) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!U || shot < 0 || shot >= ctx->plan.S) {
            ctx->err = "get_state: null pointer or shot out of range";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const long long n = ctx->plan.n_ext;
        double *dst = on_device ? U : ctx->staging;
        if (ctx->dtype == 0) HCK(launch_gather<double>((const double *)ctx->U, ctx->map, n, shot, dst, ctx->stream));
        else HCK(launch_gather<float>((const float *)ctx->U, ctx->map, n, shot, dst, ctx->stream));
        if (!on_device) HCK(hipMemcpyAsync(U, ctx->staging, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_set_sources(hho_ctx *ctx, int32_t shot, int32_t n, const double *xy, const double *dir,
                           const double *f0, const double *t0, const double *amp) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (shot < 0 || shot >= ctx->plan.S || n < 0 || (n > 0 && (!xy || !dir || !f0 || !t0 || !amp))) {
            ctx->err = "set_sources: bad arguments";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        std::vector<SrcDev> keep;
        for (const SrcDev &e : ctx->h_src)
            if (e.shot != shot) keep.push_back(e);
        const int d = ctx->plan.dim;
        for (int i = 0; i < n; ++i) {
            const double *x = xy + (size_t)d * i;
            const int c = d == 2 ? locate_cell(ctx->plan, x[0], x[1]) : locate_cell3(ctx->plan, x[0], x[1], x[2]);
            if (c < 0) {
                ctx->err = "set_sources: source " + std::to_string(i) + " lies outside the mesh";
                return HHO_ERR_ARG;
            }
            SrcDev e;
            std::memset(&e, 0, sizeof(e));
            e.ic = ctx->plan.ic_of_cell[c];
            e.shot = shot;
            e.dirx = dir[(size_t)d * i];
            e.diry = dir[(size_t)d * i + 1];
            e.dirz = d == 3 ? dir[(size_t)d * i + 2] : 0.0;
            e.f0 = f0[i];
            e.t0 = t0[i];
            e.amp = amp[i];
            if (d == 2) eval_basis(ctx->plan, c, x[0], x[1], e.phi);
            else eval_basis3(ctx->plan, c, x[0], x[1], x[2], e.phi);
            keep.push_back(e);
        }
        ctx->h_src = keep;
        ctx->version++;
        return rebuild_sources(ctx);
    });
}

hho_status hho_set_loads(hho_ctx *ctx, int32_t n_terms, const double *g, const double *omega,
                         const double *phase) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (ctx->plan.dim != 2) return two_dim_only(ctx, "set_loads");
        if (n_terms < 0 || n_terms > 4 || (n_terms > 0 && (!g || !omega || !phase))) {
            ctx->err = "set_loads: 0..4 terms with non-null arrays";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const Plan &P = ctx->plan;
        ctx->nterms = 0;
        ctx->version++;
        if (n_terms == 0) return HHO_OK;
        const int rows = 5 * P.N;
        std::vector<double> h((size_t)n_terms * rows * P.n_ic, 0.0);
        for (int m = 0; m < n_terms; ++m)
            for (int c = 0; c < P.n_cells; ++c) {
                const int nr = (P.medium[c] == kFluid ? 3 : 5) * P.N, ic = P.ic_of_cell[c];
                for (int r = 0; r < nr; ++r)
                    h[((size_t)m * rows + r) * P.n_ic + ic] = g[(size_t)m * P.n_ext + P.ext_off[c] + r];
            }
        if (ctx->gload) {
            (void)hipFree(ctx->gload);
            ctx->allocs.erase(std::find(ctx->allocs.begin(), ctx->allocs.end(), ctx->gload));
            ctx->gload = nullptr;
        }
        if ((s = upload_real(ctx, &ctx->gload, h))) return s;
        for (int m = 0; m < n_terms; ++m) {
            ctx->omega[m] = omega[m];
            ctx->phase[m] = phase[m];
        }
        ctx->nterms = n_terms;
        return HHO_OK;
    });
}

hho_status hho_receivers(hho_ctx *ctx, int32_t n, const double *xy, const int32_t *field) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n < 0 || (n > 0 && (!xy || !field))) {
            ctx->err = "receivers: bad arguments";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const Plan &P = ctx->plan;
        std::vector<RecDev> v;
        const int d = P.dim;
        for (int i = 0; i < n; ++i) {
            const double *x = xy + (size_t)d * i;
            const int c = d == 2 ? locate_cell(P, x[0], x[1]) : locate_cell3(P, x[0], x[1], x[2]);
            if (c < 0) {
                ctx->err = "receivers: receiver " + std::to_string(i) + " lies outside the mesh";
                return HHO_ERR_ARG;
            }
            if (field[i] != (int)P.medium[c]) {
                ctx->err = "receivers: receiver " + std::to_string(i) + " records " +
                           (field[i] == 0 ? "p but lies in the solid" : "v but lies in the fluid");
                return HHO_ERR_ARG;
            }
            RecDev r;
            std::memset(&r, 0, sizeof(r));
            r.ic = P.ic_of_cell[c];
            r.field = field[i];
            r.r = i;
            if (d == 2) eval_basis(P, c, x[0], x[1], r.phi);
            else eval_basis3(P, c, x[0], x[1], x[2], r.phi);
            v.push_back(r);
        }
        std::stable_sort(v.begin(), v.end(), [](const RecDev &x, const RecDev &y) { return x.ic < y.ic; });
        std::vector<int32_t> first(P.n_ic, -1);
        for (size_t e = 0; e < v.size(); ++e) {
            v[e].next = (e + 1 < v.size() && v[e + 1].ic == v[e].ic) ? (int)e + 1 : -1;
            if (e == 0 || v[e - 1].ic != v[e].ic) first[v[e].ic] = (int)e;
        }
        if (!ctx->rec_first && (s = dalloc(ctx, (void **)&ctx->rec_first, first.size() * sizeof(int32_t)))) return s;
        if ((size_t)n > 0) {
            RecDev *d = nullptr;
            if ((s = dalloc(ctx, (void **)&d, v.size() * sizeof(RecDev)))) return s;
            HCK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(RecDev), hipMemcpyHostToDevice, ctx->stream));
            ctx->rec = d;
        }
        HCK(hipMemcpyAsync(ctx->rec_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        ctx->nrec = n;
        ctx->version++;
        return HHO_OK;
    });
}

hho_status hho_reserve_steps(hho_ctx *ctx, int32_t n_steps) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n_steps < 0) {
            ctx->err = "reserve_steps: n_steps >= 0 required";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        return reserve_steps(ctx, n_steps);
    });
}

hho_status hho_erk_step(hho_ctx *ctx, double t0, double dt, int32_t n_steps) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(t0)) {
            ctx->err = "erk_step: n_steps >= 0 and dt > 0 required";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        std::vector<double> E0;
        if ((s = run_steps(ctx, t0, dt, n_steps, E0))) return s;
        return end_steps(ctx, n_steps, E0);
    });
}

hho_status hho_set_dt_scale(hho_ctx *ctx, const double *scale) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        const int S = ctx->plan.S;
        if (!scale) {
            if (ctx->dt_scaled) ctx->version++;
            ctx->dt_scaled = false;
            return HHO_OK;
        }
        for (int i = 0; i < S; ++i)
            if (!(scale[i] > 0.0) || !std::isfinite(scale[i])) {
                ctx->err = "set_dt_scale: multipliers must be finite and > 0";
                return HHO_ERR_ARG;
            }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        if (!ctx->dt_scale && (s = dalloc(ctx, (void **)&ctx->dt_scale, (size_t)S * sizeof(double)))) return s;
        HCK(hipMemcpyAsync(ctx->dt_scale, scale, (size_t)S * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        if (!ctx->dt_scaled) ctx->version++;
        ctx->dt_scaled = true;
        return HHO_OK;
    });
}

hho_status hho_cfl_search(hho_ctx *ctx, double t_final, int32_t n_start, double delta, double eps,
                          int32_t max_rounds, int32_t *n_stable, int32_t *n_unstable, int32_t *tried,
                          double *growth, int32_t cap, int32_t *n_tried) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!(t_final > 0.0) || !std::isfinite(t_final) || n_start < 1 || !(delta > 0.0) || !(delta < 1.0) ||
            !(eps > 0.0) || max_rounds < 1 || !n_stable || !n_unstable || cap < 0 || (cap > 0 && (!tried || !growth))) {
            ctx->err = "cfl_search: t_final > 0, n_start >= 1, 0 < delta < 1, eps > 0, max_rounds >= 1 required";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const int S = ctx->plan.S;
        const size_t sbytes = (size_t)ctx->rows * ctx->LT * ctx->rsize;
        if (!ctx->cfl_save && (s = dalloc(ctx, &ctx->cfl_save, sbytes))) return s;
        HCK(hipMemcpyAsync(ctx->cfl_save, ctx->U, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
        const int keep_energy = ctx->record_energy;
        if (!keep_energy) {
            ctx->record_energy = 1;
            ctx->version++;
        }
        *n_stable = 0;
        *n_unstable = 0;
        int count = 0;
        // the rounds (a device failure returns from here; the restore below runs in every case)
        auto rounds = [&]() -> hho_status {
            long long next = n_start;
            std::vector<double> scale(S), E;
            hho_status st = HHO_OK;
            for (int round = 0; round < max_rounds && *n_unstable == 0 && next >= 1; ++round) {
                // this round's candidates: N_j, N_{j+1} = N_j - max(1, floor(delta N_j)), ...
                std::vector<int> N;
                for (int i = 0; i < S && next >= 1; ++i) {
                    N.push_back((int)next);
                    next -= std::max<long long>(1, (long long)std::floor(delta * (double)next));
                }
                const int nmax = N[0];
                for (int i = 0; i < S; ++i) scale[i] = i < (int)N.size() ? (double)nmax / N[i] : 1.0;
                if ((st = hho_set_dt_scale(ctx, scale.data()))) return st;
                HCK(hipMemcpyAsync(ctx->U, ctx->cfl_save, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
                ctx->traces_valid = false;
                std::vector<double> E0;
                if ((st = run_steps(ctx, 0.0, t_final / nmax, nmax, E0))) return st;
                E.resize((size_t)nmax * S);
                HCK(hipMemcpyAsync(E.data(), ctx->e_hist, E.size() * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream));
                HCK(hipStreamSynchronize(ctx->stream));
                // Algorithm algo_CFL: relative energy increase over the initial and the previous energy
                for (size_t i = 0; i < N.size(); ++i) {
                    double g = 0.0, prev = E0[i];
                    bool bad = !(E0[i] > 0.0) || !std::isfinite(E0[i]);
                    for (int n = 0; n < N[i] && !bad; ++n) {
                        const double e = E[(size_t)n * S + i];
                        if (!std::isfinite(e)) {
                            bad = true;
                            break;
                        }
                        g = std::max(g, std::max((e - E0[i]) / E0[i], (e - prev) / prev));
                        prev = e;
                    }
                    if (bad) g = std::numeric_limits<double>::infinity();
                    if (count < cap) {
                        tried[count] = N[i];
                        growth[count] = g;
                    }
                    ++count;
                    if (g > eps) {
                        *n_unstable = N[i];
                        break;
                    }
                    *n_stable = N[i];
                }
            }
            return st;
        };
        s = rounds();
        if (n_tried) *n_tried = count;
        const hho_status s2 = hho_set_dt_scale(ctx, nullptr);
        if (!keep_energy) {
            ctx->record_energy = 0;
            ctx->version++;
        }
        HCK(hipMemcpyAsync(ctx->U, ctx->cfl_save, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        ctx->traces_valid = false;
        return s != HHO_OK ? s : s2;
    });
}


hho_status hho_adjoint_step(hho_ctx *ctx, double t0, double dt, int32_t n_steps, int32_t ckpt_every,
                            const double *d_obs, double *J, double *grad) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (ctx->plan.dim != 2) return two_dim_only(ctx, "adjoint_step");
        if (n_steps < 1 || !(dt > 0.0) || !std::isfinite(t0) || ckpt_every < 0 || !J || !grad ||
            (ctx->nrec > 0 && !d_obs)) {
            ctx->err = "adjoint_step: n_steps >= 1, dt > 0, ckpt_every >= 0, J, grad (and d_obs with receivers) required";
            return HHO_ERR_ARG;
        }
        if (ctx->dt_scaled) {
            ctx->err = "adjoint_step: per-shot time-step multipliers are set (hho_set_dt_scale); reset them first";
            return HHO_ERR_ARG;
        }
        std::vector<StageCoef> co;
        if (!erk_coefficients(ctx->stages, co)) return HHO_ERR_ARG;
        for (const StageCoef &q : co)
            if (q.cY != 0.0) {
                ctx->err = "adjoint_step: the reverse sweep needs a subdiagonal Runge-Kutta matrix (rk_stages 2 or 4)";
                return HHO_ERR_ARG;
            }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const int every = ckpt_every > 0 ? std::min<int>(ckpt_every, n_steps)
                                         : std::max(1, (int)std::ceil(std::sqrt((double)n_steps)));
        const int n_seg = (n_steps + every - 1) / every;
        if ((s = ensure_adjoint(ctx, every, n_seg))) return s;
        AdjWork &w = ctx->adj;
        const Plan &P = ctx->plan;
        const int S = P.S;
        const size_t sbytes = (size_t)ctx->rows * ctx->LT * ctx->rsize;
        // forward pass with checkpoints U^{g * every}, then U^N
        std::vector<double> E0;
        if ((s = begin_steps(ctx, t0, dt, n_steps, E0))) return s;
        if ((s = ensure_graphs(ctx))) return s;
        // segments replayed from the step graphs, which start on clock slot 0: after a segment of odd
        // length the current clock sits in slot 1 and is copied back to slot 0
        int slot = 0;
        for (int g = 0; g < n_seg; ++g) {
            HCK(hipMemcpyAsync((char *)w.ckpt + (size_t)g * sbytes, ctx->U, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
            const int len = std::min(every, n_steps - g * every);
            if (slot == 1) HCK(hipMemcpyAsync(ctx->clock, ctx->clock + 1, sizeof(Clock), hipMemcpyDeviceToDevice, ctx->stream));
            s = replay_steps(len, [&](int i) -> hho_status {
                HCK(hipGraphLaunch(ctx->gexec[i], ctx->stream));
                return HHO_OK;
            });
            if (s != HHO_OK) return s;
            slot = len & 1;
        }
        if ((s = end_steps(ctx, n_steps, E0))) return s;
        void *uN = (char *)w.ckpt + (size_t)n_seg * sbytes;
        HCK(hipMemcpyAsync(uN, ctx->U, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
        // misfit J = 1/2 dt sum_shots sum_n sum_r |R_r U^n - d_r^n|^2 from the recorded traces
        double Jv = 0.0;
        const size_t per_shot = (size_t)n_steps * ctx->nrec * 2;
        if (ctx->nrec > 0) {
            const size_t stride = ctx->rec_cap / (size_t)S;
            std::vector<double> tr(stride * S);
            HCK(hipMemcpyAsync(tr.data(), ctx->rec_out, tr.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            HCK(hipStreamSynchronize(ctx->stream));
            for (int sh = 0; sh < S; ++sh)
                for (size_t e = 0; e < per_shot; ++e) {
                    const double d = tr[sh * stride + e] - d_obs[sh * per_shot + e];
                    Jv += d * d;
                }
            Jv *= 0.5 * dt;
            const size_t need = per_shot * S;
            if (need > w.dobs_cap) {
                dfree(ctx, w.dobs);
                w.dobs = nullptr;
                w.dobs_cap = 0;
                if ((s = dalloc(ctx, (void **)&w.dobs, need * sizeof(double)))) return s;
                w.dobs_cap = need;
            }
            HCK(hipMemcpyAsync(w.dobs, d_obs, need * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        }
        // reverse sweep
        HCK(hipMemsetAsync(w.lam, 0, sbytes, ctx->stream));
        HCK(hipMemsetAsync(w.gacc, 0, 3 * (size_t)ctx->LT * sizeof(double), ctx->stream));
        std::vector<Clock> clocks(n_seg);
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return adjoint_sweep<decltype(kc)::value, R>(ctx, co, every, n_seg, n_steps, t0, dt, clocks);
        });
        if (s != HHO_OK) return s;
        HCK(launch_grad_reduce(w.gacc, ctx->LT, S, w.ic_of_cell, P.n_cells, w.grad, ctx->stream));
        HCK(hipMemcpyAsync(grad, w.grad, 3 * (size_t)P.n_cells * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        // leave the context at U^N, as after hho_erk_step
        HCK(hipMemcpyAsync(ctx->U, uN, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
        ctx->h_clock = Clock{t0, dt, n_steps, 0};
        HCK(hipMemcpyAsync(ctx->clock, &ctx->h_clock, sizeof(Clock), hipMemcpyHostToDevice, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        ctx->traces_valid = false;
        *J = Jv;
        return HHO_OK;
    });
}

hho_status hho_autotune(hho_ctx *ctx, int32_t *lanes) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return autotune_shape<decltype(kc)::value, R>(ctx);
        });
        if (s != HHO_OK) return s;
        if (lanes) *lanes = ctx->launch[ctx->shape].lanes;
        return HHO_OK;
    });
}

hho_status hho_set_launch(hho_ctx *ctx, int32_t lanes) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        for (size_t i = 0; i < ctx->launch.size(); ++i)
            if (ctx->launch[i].lanes == lanes || ctx->launch[i].lanes == lanes / ctx->plan.S * ctx->plan.S) {
                if ((int)i != ctx->shape) {
                    ctx->shape = (int)i;
                    ctx->version++;
                }
                return HHO_OK;
            }
        ctx->err = "set_launch: no launch shape with " + std::to_string(lanes) + " lanes";
        return HHO_ERR_ARG;
    });
}

hho_status hho_set_tuning(hho_ctx *ctx, int32_t lanes, int32_t flags) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (flags & ~HHO_TUNE_NT_STORES) {
            ctx->err = "set_tuning: unknown flag bits " + std::to_string(flags);
            return HHO_ERR_ARG;
        }
        const hho_status s = hho_set_launch(ctx, lanes);
        if (s != HHO_OK) return s;
        const int nt = (flags & HHO_TUNE_NT_STORES) ? 1 : 0;
        if (nt != ctx->nt_stores) {
            ctx->nt_stores = nt;
            ctx->version++;
        }
        return HHO_OK;
    });
}

hho_status hho_get_tuning(const hho_ctx *ctx, int32_t *lanes, int32_t *flags) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (lanes) *lanes = ctx->launch[ctx->shape].lanes;
        if (flags) *flags = ctx->nt_stores ? HHO_TUNE_NT_STORES : 0;
        return HHO_OK;
    });
}

hho_status hho_dt_cfl(const hho_ctx *ctx, double factor, double *dt) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx || !dt || !(factor > 0.0)) return HHO_ERR_ARG;
        if (ctx->plan.dim != 2) return two_dim_only(const_cast<hho_ctx *>(ctx), "dt_cfl");
        *dt = factor * ctx->cfl_dt;
        return HHO_OK;
    });
}

hho_status hho_batch_create(hho_ctx *const *ctxs, int32_t n, hho_batch **out) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        if (!ctxs || n <= 0 || !out) return HHO_ERR_ARG;
        *out = nullptr;
        for (int i = 0; i < n; ++i)
            if (!ctxs[i] || ctxs[i]->device != ctxs[0]->device) {
                g_setup_error = "batch: contexts must be non-null and on one device";
                return HHO_ERR_ARG;
            }
        hho_batch *b = new hho_batch();
        b->ctxs.assign(ctxs, ctxs + n);
        (void)hipSetDevice(ctxs[0]->device);
        for (int i = 0; i <= n; ++i) {
            hipStream_t st;
            hipEvent_t ev;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                g_setup_error = "batch: stream or event creation failed";
                hho_batch_destroy(b);
                return HHO_ERR_DEVICE;
            }
            b->streams.push_back(st);
            b->events.push_back(ev);
        }
        *out = b;
        return HHO_OK;
    });
}

void hho_batch_destroy(hho_batch *b) {
    if (!b) return;
    if (!b->ctxs.empty()) (void)hipSetDevice(b->ctxs[0]->device);
    for (hipStream_t st : b->streams) (void)hipStreamSynchronize(st);
    for (hipGraphExec_t g : b->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (b->t_begin) (void)hipEventDestroy(b->t_begin);
    if (b->t_end) (void)hipEventDestroy(b->t_end);
    for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : b->events) (void)hipEventDestroy(ev);
    delete b;
}

const char *hho_batch_last_error(const hho_batch *b) { return b ? b->err.c_str() : g_setup_error.c_str(); }

hho_status hho_batch_last_time(const hho_batch *b, double *ms) {
    if (!b || !ms) return HHO_ERR_ARG;
    *ms = (double)b->last_ms;
    return HHO_OK;
}

hho_status hho_batch_erk_step(hho_batch *b, const double *t0, const double *dt, int32_t n_steps) {
    return guarded(b ? &const_cast<hho_batch *>(b)->err : &g_setup_error, [&]() -> hho_status {
        if (!b || !t0 || !dt || n_steps < 0) return HHO_ERR_ARG;
        const int n = (int)b->ctxs.size();
        hho_ctx *c0 = b->ctxs[0];
        hipStream_t launch_st = c0->stream;
        if (hipSetDevice(c0->device) != hipSuccess) return HHO_ERR_DEVICE;
        std::vector<std::vector<double>> E0(n);
        for (int i = 0; i < n; ++i) {
            hho_ctx *ctx = b->ctxs[i];
            if (!(dt[i] > 0.0)) {
                b->err = "batch_erk_step: dt must be positive";
                return HHO_ERR_ARG;
            }
            hho_status s = begin_steps(ctx, t0[i], dt[i], n_steps, E0[i], true);
            if (s != HHO_OK) {
                b->err = ctx->err;
                return s;
            }
        }
        // the batch launches on the first context's stream: every context's set-up work is done
        for (int i = 0; i < n; ++i)
            if (b->ctxs[i]->stream != launch_st && hipStreamSynchronize(b->ctxs[i]->stream) != hipSuccess)
                return HHO_ERR_DEVICE;
        if (hipStreamSynchronize(launch_st) != hipSuccess) return HHO_ERR_DEVICE;
        for (int i = 0; i < n; ++i) read_initial_energy(b->ctxs[i], E0[i]);
        bool fresh = b->gexec[0] && (int)b->versions.size() == n;
        for (int i = 0; fresh && i < n; ++i) fresh = b->versions[i] == b->ctxs[i]->version;
        if (n_steps > 0 && !fresh) {
            for (hipGraphExec_t &g : b->gexec) {
                if (g) (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
            for (int i = 0; i < kNumGraphs; ++i) {
                hho_status s = capture_batch(b, kGraphSteps >> i, &b->gexec[i]);
                if (s != HHO_OK) return s;
            }
            b->versions.clear();
            for (hho_ctx *ctx : b->ctxs) b->versions.push_back(ctx->version);
        }
        if (!b->t_begin && (hipEventCreate(&b->t_begin) != hipSuccess || hipEventCreate(&b->t_end) != hipSuccess)) {
            b->err = "batch: event creation failed";
            return HHO_ERR_DEVICE;
        }
        if (hipEventRecord(b->t_begin, launch_st) != hipSuccess) return HHO_ERR_DEVICE;
        hho_status rs = replay_steps(n_steps, [&](int i) -> hho_status {
            if (hipGraphLaunch(b->gexec[i], launch_st) != hipSuccess) {
                b->err = "batch: hipGraphLaunch failed";
                return HHO_ERR_DEVICE;
            }
            return HHO_OK;
        });
        if (rs != HHO_OK) return rs;
        if (hipEventRecord(b->t_end, launch_st) != hipSuccess) return HHO_ERR_DEVICE;
        for (int i = 0; i < n; ++i) {
            hho_status s = enqueue_history_copy(b->ctxs[i], n_steps, launch_st);
            if (s != HHO_OK) {
                b->err = b->ctxs[i]->err;
                return s;
            }
        }
        if (hipStreamSynchronize(launch_st) != hipSuccess) return HHO_ERR_DEVICE;
        if (hipEventElapsedTime(&b->last_ms, b->t_begin, b->t_end) != hipSuccess) return HHO_ERR_DEVICE;
        hho_status worst = HHO_OK;
        for (int i = 0; i < n; ++i) {
            hho_status s = check_history(b->ctxs[i], n_steps, E0[i]);
            if (s != HHO_OK && worst == HHO_OK) {
                worst = s;
                b->err = "context " + std::to_string(i) + ": " + b->ctxs[i]->err;
            }
        }
        return worst;
    });
}

hho_status hho_synchronize(hho_ctx *ctx) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        HCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_get_traces(hho_ctx *ctx, int32_t shot, double *out) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!out || shot < 0 || shot >= ctx->plan.S) {
            ctx->err = "get_traces: bad arguments";
            return HHO_ERR_ARG;
        }
        if (ctx->nrec == 0 || ctx->last_steps == 0) return HHO_OK;
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        // shots are strided by the recording capacity, which may exceed the last call's steps
        const size_t n = (size_t)ctx->last_steps * ctx->nrec * ctx->rec_w;
        const size_t stride = ctx->rec_cap / (size_t)ctx->plan.S;
        HCK(hipMemcpyAsync(out, ctx->rec_out + (size_t)shot * stride, n * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_energy(hho_ctx *ctx, double *E) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!E) {
            ctx->err = "energy: null output";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return energy_now<decltype(kc)::value, R>(ctx, ctx->e_now);
        });
        if (s != HHO_OK) return s;
        HCK(hipMemcpyAsync(E, ctx->e_now, ctx->plan.S * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        return HHO_OK;
    });
}

hho_status hho_energy_history(hho_ctx *ctx, int32_t shot, double *out) {
    return guarded(ctx ? &const_cast<hho_ctx *>(ctx)->err : &g_setup_error, [&]() -> hho_status {
        if (!ctx) return HHO_ERR_ARG;
        if (!out || shot < 0 || shot >= ctx->plan.S || !ctx->record_energy) {
            ctx->err = "energy_history: bad arguments or record_energy = 0";
            return HHO_ERR_ARG;
        }
        hho_status s = set_device(ctx);
        if (s != HHO_OK) return s;
        const int S = ctx->plan.S;
        std::vector<double> E((size_t)ctx->last_steps * S);
        if (!E.empty())
            HCK(hipMemcpyAsync(E.data(), ctx->e_hist, E.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        for (int n = 0; n < ctx->last_steps; ++n) out[n] = E[(size_t)n * S + shot];
        return HHO_OK;
    });
}

}  // extern "C"

// ----------------------------------------------------------------------------- host-only inspection
#include "../../include/hho_inspect.h"

struct hho_inspect {
    Plan plan;
};

extern "C" {

hho_status hho_inspect_create(const hho_mesh *mesh, const hho_params *prm, hho_inspect **out) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        g_setup_error.clear();
        if (!out || !mesh || !prm) return HHO_ERR_ARG;
        *out = nullptr;
        hho_inspect *p = new hho_inspect();
        int code = 0;
        std::string msg = build_plan(mesh->n_vertices, mesh->xy, mesh->n_cells, mesh->cell_ptr, mesh->cell_vtx,
                                     mesh->medium, mesh->rho, mesh->a, mesh->b, prm->k, prm->eta_f, prm->eta_s,
                                     prm->stab_speed, prm->n_shots, p->plan, &code);
        if (code != 0) {
            g_setup_error = msg;
            delete p;
            return (hho_status)code;
        }
        *out = p;
        return HHO_OK;
    });
}

hho_status hho_inspect3d_create(const hho_mesh3d *mesh, const hho_params *prm, hho_inspect **out) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        g_setup_error.clear();
        if (!out || !mesh || !prm) return HHO_ERR_ARG;
        *out = nullptr;
        hho_inspect *p = new hho_inspect();
        int code = 0;
        std::string msg = build_plan3d(mesh->n_vertices, mesh->xyz, mesh->n_cells, mesh->cell_ptr, mesh->cell_vtx,
                                       mesh->medium, mesh->rho, mesh->a, mesh->b, prm->k, prm->eta_f, prm->eta_s,
                                       prm->stab_speed, prm->n_shots, p->plan, &code);
        if (code != 0) {
            g_setup_error = msg;
            delete p;
            return (hho_status)code;
        }
        *out = p;
        return HHO_OK;
    });
}

void hho_inspect_destroy(hho_inspect *p) { delete p; }

hho_status hho_inspect_sizes(const hho_inspect *p, int64_t *sz) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        if (!p || !sz) return HHO_ERR_ARG;
        const Plan &P = p->plan;
        const int64_t v[10] = {P.N, P.F, P.n_ic, P.max_nf, (int64_t)P.groups.size(), (int64_t)P.tables.size(),
                               P.n_cells, P.n_faces, P.cpb, (int64_t)P.blk_group.size()};
        std::memcpy(sz, v, sizeof(v));
        return HHO_OK;
    });
}

hho_status hho_inspect_cell_tables(const hho_inspect *p, int32_t *ic_tab, int32_t *pooled) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        if (!p) return HHO_ERR_ARG;
        const Plan &P = p->plan;
        if (ic_tab) std::copy(P.ic_tab.begin(), P.ic_tab.end(), ic_tab);
        if (pooled)
            for (size_t g = 0; g < P.groups.size(); ++g) pooled[g] = P.groups[g].pooled ? 1 : 0;
        return HHO_OK;
    });
}

hho_status hho_inspect_arrays(const hho_inspect *p, double *tables, int32_t *groups, int32_t *link, double *c0,
                              double *mat, int32_t *ic_of_cell) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        if (!p) return HHO_ERR_ARG;
        const Plan &P = p->plan;
        if (tables) std::copy(P.tables.begin(), P.tables.end(), tables);
        if (groups)
            for (size_t g = 0; g < P.groups.size(); ++g) {
                const Group &G = P.groups[g];
                const int32_t v[6] = {G.medium, G.nF, G.tab_off, G.ic_begin, G.ncells, G.blk_begin};
                std::memcpy(groups + 6 * g, v, sizeof(v));
            }
        if (link) std::copy(P.link.begin(), P.link.end(), link);
        if (c0) std::copy(P.c0.begin(), P.c0.end(), c0);
        if (mat) std::copy(P.mat.begin(), P.mat.end(), mat);
        if (ic_of_cell) std::copy(P.ic_of_cell.begin(), P.ic_of_cell.end(), ic_of_cell);
        return HHO_OK;
    });
}

hho_status hho_inspect_dt_cfl(const hho_inspect *p, int32_t stages, double factor, double *dt) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        std::vector<StageCoef> co;
        if (!p || !dt || !(factor > 0.0) || !erk_coefficients(stages, co)) return HHO_ERR_ARG;
        if (p->plan.dim != 2) return HHO_ERR_ARG;
        *dt = factor * cfl_time_step(p->plan, stages);
        return HHO_OK;
    });
}

hho_status hho_inspect_erk(int32_t stages, double *coefs) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        std::vector<StageCoef> co;
        if (!coefs || !erk_coefficients(stages, co)) return HHO_ERR_ARG;
        for (int i = 0; i < stages; ++i) {
            const StageCoef &q = co[i];
            const double v[9] = {q.c, q.cY, q.ck, q.cb, q.qa, q.qb, q.cd, (double)q.q_write, (double)q.q_read};
            std::memcpy(coefs + 9 * i, v, sizeof(v));
        }
        return HHO_OK;
    });
}

hho_status hho_inspect_grad_coefs(const hho_inspect *p, double *gm) {
    return guarded(&g_setup_error, [&]() -> hho_status {
        if (!p || !gm) return HHO_ERR_ARG;
        std::copy(p->plan.gm.begin(), p->plan.gm.end(), gm);
        return HHO_OK;
    });
}

}  // extern "C"
