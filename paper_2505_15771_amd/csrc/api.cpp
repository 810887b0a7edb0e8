// C ABI of the HHO elasto-acoustic ERK engine (declared in include/hho.h): context
// lifetime, device buffers, state transfer, sources, loads, receivers and the
// explicit Runge-Kutta driver (Sec. 4.2, eq. ERK_compact / ex_solve, tableaux eq. ERK).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hho.h"
#include "device.h"
#include "plan.h"

using namespace hho;

struct hho_ctx {
    Plan plan;
    int dtype = 0, stages = 4, record_energy = 0, device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<void *> allocs;
    size_t rsize = 8;          // bytes per real
    long long LT = 0;          // lanes
    int rows = 0, trows = 0;   // state rows (5N), trace rows
    int n_blocks = 0;
    void *U = nullptr, *Y[2] = {nullptr, nullptr}, *acc = nullptr, *T[3] = {nullptr, nullptr, nullptr};
    int tcur = 0;
    bool traces_valid = false;
    void *arena = nullptr;  // state, stage, trace, link, c0 and mat arrays (one buffer resource)
    size_t arena_bytes = 0;
    int32_t *link = nullptr;
    void *c0 = nullptr, *mat = nullptr, *tab = nullptr;
    double *emat = nullptr;
    GroupDev *groups = nullptr;
    int32_t *blk_group = nullptr;
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
    int32_t *rec_first = nullptr;
    RecDev *rec = nullptr;
    double *rec_out = nullptr;
    size_t rec_cap = 0;
    int last_steps = 0;
    // energy
    double *e_part = nullptr, *e_hist = nullptr, *e_now = nullptr;
    size_t e_hist_cap = 0;
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
struct StageCoef {
    double cU, cY, ck, cb, c;
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
    out.assign(s, StageCoef{0, 0, 0, 0, 0});
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
    return true;
}

unsigned arena_off(const hho_ctx *ctx, const void *p) {
    return p ? (unsigned)((const char *)p - (const char *)ctx->arena) : 0u;
}

template <typename R>
void set_stage_offsets(hho_ctx *ctx, StageArgs<R> &a) {
    a.o_yin = arena_off(ctx, a.Yin);
    a.o_yout = arena_off(ctx, a.Yout);
    a.o_u = arena_off(ctx, a.U);
    a.o_acc = arena_off(ctx, a.acc);
    a.o_tin = arena_off(ctx, a.Tin);
    a.o_tout = arena_off(ctx, a.Tout);
}

template <typename R>
StageArgs<R> base_args(hho_ctx *ctx) {
    StageArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.link = ctx->link;
    a.c0 = (const R *)ctx->c0;
    a.mat = (const R *)ctx->mat;
    a.tab = (const R *)ctx->tab;
    a.groups = ctx->groups;
    a.blk_group = ctx->blk_group;
    a.n_ic = ctx->plan.n_ic;
    a.S = ctx->plan.S;
    a.cpb = ctx->plan.cpb;
    a.LT = ctx->LT;
    a.emat = ctx->emat;
    a.arena = ctx->arena;
    a.arena_bytes = (unsigned)ctx->arena_bytes;
    a.o_link = arena_off(ctx, ctx->link);
    a.o_c0 = arena_off(ctx, ctx->c0);
    a.o_mat = arena_off(ctx, ctx->mat);
    return a;
}

template <int K, typename R>
hho_status compute_traces(hho_ctx *ctx) {
    StageArgs<R> a = base_args<R>(ctx);
    a.Yin = (const R *)ctx->U;
    a.Tout = (R *)ctx->T[ctx->tcur];
    set_stage_offsets(ctx, a);
    HCK((launch_traces<K, R>(a, ctx->n_blocks, ctx->stream)));
    ctx->traces_valid = true;
    return HHO_OK;
}

template <int K, typename R>
hho_status energy_now(hho_ctx *ctx, double *out_dev) {
    StageArgs<R> a = base_args<R>(ctx);
    a.e_part = ctx->e_part;
    a.Yin = (const R *)ctx->U;
    set_stage_offsets(ctx, a);
    HCK((launch_energy<K, R>(a, (const R *)ctx->U, ctx->n_blocks, ctx->stream)));
    HCK(launch_energy_reduce(ctx->e_part, ctx->n_blocks, ctx->plan.S, out_dev, ctx->stream));
    return HHO_OK;
}

template <int K, typename R>
hho_status run_steps(hho_ctx *ctx, double t0, double dt, int n_steps) {
    std::vector<StageCoef> co;
    if (!erk_coefficients(ctx->stages, co)) {
        ctx->err = "unsupported ERK stage count";
        return HHO_ERR_ARG;
    }
    if (!ctx->traces_valid) {
        hho_status s = compute_traces<K, R>(ctx);
        if (s != HHO_OK) return s;
    }
    const int s = ctx->stages, S = ctx->plan.S;
    StageArgs<R> a = base_args<R>(ctx);
    a.U = (R *)ctx->U;
    a.acc = (R *)ctx->acc;
    a.dt = (R)dt;
    a.src_first = ctx->h_src.empty() ? nullptr : ctx->src_first;
    a.src = ctx->src;
    a.nterms = ctx->nterms;
    a.gload = (const R *)ctx->gload;
    a.nrec = ctx->nrec;
    a.rec_steps = n_steps;
    a.rec_out = ctx->rec_out;
    const int Tc = ctx->tcur, Ta = (Tc + 1) % 3, Tb = (Tc + 2) % 3;
    const int Tbuf[2] = {Ta, Tb};
    for (int n = 0; n < n_steps; ++n) {
        const double tn = t0 + n * dt;
        for (int i = 0; i < s; ++i) {
            const StageCoef &q = co[i];
            a.first = i == 0;
            a.last = i == s - 1;
            a.Yin = i == 0 ? (const R *)ctx->U : (const R *)ctx->Y[(i - 1) % 2];
            a.Yout = a.last ? nullptr : (R *)ctx->Y[i % 2];
            a.Tin = (const R *)ctx->T[i == 0 ? Tc : Tbuf[(i - 1) % 2]];
            a.Tout = (R *)ctx->T[a.last ? Tc : Tbuf[i % 2]];
            a.t = tn + q.c * dt;
            a.cU = (R)q.cU;
            a.cY = (R)q.cY;
            a.ck = (R)q.ck;
            a.cb = (R)q.cb;
            for (int m = 0; m < ctx->nterms; ++m) a.wterm[m] = (R)std::sin(ctx->omega[m] * a.t + ctx->phase[m]);
            a.e_part = (a.last && ctx->record_energy) ? ctx->e_part : nullptr;
            a.rec_first = (a.last && ctx->nrec > 0) ? ctx->rec_first : nullptr;
            a.rec = ctx->rec;
            a.step = n;
            set_stage_offsets(ctx, a);
            HCK((launch_stage<K, R>(a, ctx->n_blocks, ctx->stream)));
        }
        if (ctx->record_energy)
            HCK(launch_energy_reduce(ctx->e_part, ctx->n_blocks, S, ctx->e_hist + (size_t)n * S, ctx->stream));
    }
    return HHO_OK;
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

}  // namespace

extern "C" {

const char *hho_last_error(const hho_ctx *ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

hho_status hho_setup(const hho_mesh *mesh, const hho_params *prm, hho_ctx **out) {
    g_setup_error.clear();
    if (!out) return HHO_ERR_ARG;
    *out = nullptr;
    if (!mesh || !prm) {
        g_setup_error = "null mesh or params";
        return HHO_ERR_ARG;
    }
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
    int code = 0;
    std::string msg = build_plan(mesh->n_vertices, mesh->xy, mesh->n_cells, mesh->cell_ptr, mesh->cell_vtx,
                                 mesh->medium, mesh->rho, mesh->a, mesh->b, prm->k, prm->eta_f, prm->eta_s,
                                 prm->stab_speed, prm->n_shots, ctx->plan, &code);
    if (code != 0) {
        g_setup_error = msg;
        delete ctx;
        return (hho_status)code;
    }
    auto fail = [&](hho_status s) {
        g_setup_error = ctx->err;
        hho_destroy(ctx);
        return s;
    };
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return fail(s);
    Plan &P = ctx->plan;
    ctx->LT = (long long)P.n_ic * P.S;
    ctx->rows = 5 * P.N;
    ctx->trows = trace_rows(P);
    ctx->n_blocks = (int)P.blk_group.size();
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
    std::vector<GroupDev> gd;
    for (const Group &g : P.groups) gd.push_back({g.medium, g.nF, g.tab_off, g.ic_begin, g.ncells, g.blk_begin});
    std::vector<int64_t> map(P.n_ext);
    for (int c = 0; c < P.n_cells; ++c) {
        const int nr = (P.medium[c] == kFluid ? 3 : 5) * P.N;
        for (int r = 0; r < nr; ++r)
            map[P.ext_off[c] + r] = (int64_t)r * ctx->LT + (int64_t)P.ic_of_cell[c] * P.S;
    }
    if ((s = copy_in(ctx, ctx->link, P.link)) || (s = copy_in_real(ctx, ctx->c0, P.c0)) ||
        (s = copy_in_real(ctx, ctx->mat, P.mat)) || (s = upload_real(ctx, &ctx->tab, P.tables)) ||
        (s = upload(ctx, &ctx->emat, P.emat)) || (s = upload(ctx, &ctx->groups, gd)) ||
        (s = upload(ctx, &ctx->blk_group, P.blk_group)) || (s = upload(ctx, &ctx->map, map)) ||
        (s = dalloc(ctx, (void **)&ctx->staging, std::max<size_t>(1, P.n_ext) * 4 * sizeof(double))) ||
        (s = dalloc(ctx, (void **)&ctx->e_part, (size_t)ctx->n_blocks * P.S * sizeof(double))) ||
        (s = dalloc(ctx, (void **)&ctx->e_now, (size_t)P.S * sizeof(double))))
        return fail(s);
    *out = ctx;
    return HHO_OK;
}

void hho_destroy(hho_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : ctx->allocs) (void)hipFree(p);
    delete ctx;
}

hho_status hho_sizes(const hho_ctx *ctx, int64_t *n_dof, int32_t *n_cells, int32_t *n_faces) {
    if (!ctx) return HHO_ERR_ARG;
    if (n_dof) *n_dof = ctx->plan.n_ext;
    if (n_cells) *n_cells = ctx->plan.n_cells;
    if (n_faces) *n_faces = ctx->plan.n_faces;
    return HHO_OK;
}

hho_status hho_set_state(hho_ctx *ctx, int32_t shot, const double *U, int32_t on_device) {
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
}

hho_status hho_get_state(hho_ctx *ctx, int32_t shot, double *U, int32_t on_device) {
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
}

hho_status hho_set_sources(hho_ctx *ctx, int32_t shot, int32_t n, const double *xy, const double *dir,
                           const double *f0, const double *t0, const double *amp) {
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
    for (int i = 0; i < n; ++i) {
        const int c = locate_cell(ctx->plan, xy[2 * i], xy[2 * i + 1]);
        if (c < 0) {
            ctx->err = "set_sources: source " + std::to_string(i) + " lies outside the mesh";
            return HHO_ERR_ARG;
        }
        SrcDev e;
        std::memset(&e, 0, sizeof(e));
        e.ic = ctx->plan.ic_of_cell[c];
        e.shot = shot;
        e.dirx = dir[2 * i];
        e.diry = dir[2 * i + 1];
        e.f0 = f0[i];
        e.t0 = t0[i];
        e.amp = amp[i];
        eval_basis(ctx->plan, c, xy[2 * i], xy[2 * i + 1], e.phi);
        keep.push_back(e);
    }
    ctx->h_src = keep;
    return rebuild_sources(ctx);
}

hho_status hho_set_loads(hho_ctx *ctx, int32_t n_terms, const double *g, const double *omega,
                         const double *phase) {
    if (!ctx) return HHO_ERR_ARG;
    if (n_terms < 0 || n_terms > 4 || (n_terms > 0 && (!g || !omega || !phase))) {
        ctx->err = "set_loads: 0..4 terms with non-null arrays";
        return HHO_ERR_ARG;
    }
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return s;
    const Plan &P = ctx->plan;
    ctx->nterms = 0;
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
}

hho_status hho_receivers(hho_ctx *ctx, int32_t n, const double *xy, const int32_t *field) {
    if (!ctx) return HHO_ERR_ARG;
    if (n < 0 || (n > 0 && (!xy || !field))) {
        ctx->err = "receivers: bad arguments";
        return HHO_ERR_ARG;
    }
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return s;
    const Plan &P = ctx->plan;
    std::vector<RecDev> v;
    for (int i = 0; i < n; ++i) {
        const int c = locate_cell(P, xy[2 * i], xy[2 * i + 1]);
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
        eval_basis(P, c, xy[2 * i], xy[2 * i + 1], r.phi);
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
    return HHO_OK;
}

hho_status hho_erk_step(hho_ctx *ctx, double t0, double dt, int32_t n_steps) {
    if (!ctx) return HHO_ERR_ARG;
    if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(t0)) {
        ctx->err = "erk_step: n_steps >= 0 and dt > 0 required";
        return HHO_ERR_ARG;
    }
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return s;
    const int S = ctx->plan.S;
    if (ctx->nrec > 0) {
        const size_t need = (size_t)S * std::max(n_steps, 1) * ctx->nrec * 2;
        if (need > ctx->rec_cap) {
            if ((s = dalloc(ctx, (void **)&ctx->rec_out, need * sizeof(double)))) return s;
            ctx->rec_cap = need;
        }
    }
    if (ctx->record_energy) {
        const size_t need = (size_t)S * (std::max(n_steps, 1) + 1);
        if (need > ctx->e_hist_cap) {
            if ((s = dalloc(ctx, (void **)&ctx->e_hist, need * sizeof(double)))) return s;
            ctx->e_hist_cap = need;
        }
    }
    ctx->last_steps = n_steps;
    std::vector<double> E0(S);
    if (ctx->record_energy) {
        s = dispatch(ctx, [&](auto kc, auto *r) {
            using R = std::remove_pointer_t<decltype(r)>;
            return energy_now<decltype(kc)::value, R>(ctx, ctx->e_now);
        });
        if (s != HHO_OK) return s;
        HCK(hipMemcpyAsync(E0.data(), ctx->e_now, S * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    }
    s = dispatch(ctx, [&](auto kc, auto *r) {
        using R = std::remove_pointer_t<decltype(r)>;
        return run_steps<decltype(kc)::value, R>(ctx, t0, dt, n_steps);
    });
    if (s != HHO_OK) return s;
    if (ctx->record_energy && n_steps > 0) {
        std::vector<double> E((size_t)n_steps * S);
        HCK(hipMemcpyAsync(E.data(), ctx->e_hist, E.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HCK(hipStreamSynchronize(ctx->stream));
        const bool driven = !ctx->h_src.empty() || ctx->nterms > 0;
        for (int sh = 0; sh < S; ++sh) {
            double prev = E0[sh];
            for (int n = 0; n < n_steps; ++n) {
                const double e = E[(size_t)n * S + sh];
                if (!std::isfinite(e) ||
                    (!driven && (e > 1.05 * E0[sh] + 1e-300 || e > 1.05 * prev + 1e-300))) {
                    ctx->err = "energy of shot " + std::to_string(sh) + " grew by more than 5 % (or is not finite) at step " +
                               std::to_string(n);
                    return HHO_ERR_UNSTABLE;
                }
                prev = e;
            }
        }
    }
    return HHO_OK;
}

hho_status hho_synchronize(hho_ctx *ctx) {
    if (!ctx) return HHO_ERR_ARG;
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return s;
    HCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

hho_status hho_get_traces(hho_ctx *ctx, int32_t shot, double *out) {
    if (!ctx) return HHO_ERR_ARG;
    if (!out || shot < 0 || shot >= ctx->plan.S) {
        ctx->err = "get_traces: bad arguments";
        return HHO_ERR_ARG;
    }
    if (ctx->nrec == 0 || ctx->last_steps == 0) return HHO_OK;
    hho_status s = set_device(ctx);
    if (s != HHO_OK) return s;
    const size_t n = (size_t)ctx->last_steps * ctx->nrec * 2;
    HCK(hipMemcpyAsync(out, ctx->rec_out + (size_t)shot * n, n * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream));
    HCK(hipStreamSynchronize(ctx->stream));
    return HHO_OK;
}

hho_status hho_energy(hho_ctx *ctx, double *E) {
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
}

hho_status hho_energy_history(hho_ctx *ctx, int32_t shot, double *out) {
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
}

}  // extern "C"

// ----------------------------------------------------------------------------- host-only inspection
#include "../../include/hho_inspect.h"

struct hho_inspect {
    Plan plan;
};

extern "C" {

hho_status hho_inspect_create(const hho_mesh *mesh, const hho_params *prm, hho_inspect **out) {
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
}

void hho_inspect_destroy(hho_inspect *p) { delete p; }

hho_status hho_inspect_sizes(const hho_inspect *p, int64_t *sz) {
    if (!p || !sz) return HHO_ERR_ARG;
    const Plan &P = p->plan;
    const int64_t v[10] = {P.N, P.F, P.n_ic, P.max_nf, (int64_t)P.groups.size(), (int64_t)P.tables.size(),
                           P.n_cells, P.n_faces, P.cpb, (int64_t)P.blk_group.size()};
    std::memcpy(sz, v, sizeof(v));
    return HHO_OK;
}

hho_status hho_inspect_arrays(const hho_inspect *p, double *tables, int32_t *groups, int32_t *link, double *c0,
                              double *mat, int32_t *ic_of_cell) {
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
}

}  // extern "C"
