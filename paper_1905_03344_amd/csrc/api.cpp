// Host side of libsph: parameter validation, workspace layout, and the
// orchestration of the kernels behind each C ABI entry point.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "sph_internal.h"

// Intervals of (stage, start event, stop event) recorded while timing is on.
struct StageTimer {
    struct Interval {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Interval> open;
    std::vector<hipEvent_t> pool;
    double ms[SPH_NSTAGES] = {0};
    int64_t count[SPH_NSTAGES] = {0};
};

static hipEvent_t timer_event(StageTimer *t)
{
    if (!t->pool.empty()) {
        hipEvent_t e = t->pool.back();
        t->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// folds finished intervals into the totals (the caller synchronised)
static void timer_collect(StageTimer *t)
{
    for (auto &iv : t->open) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, iv.a, iv.b) == hipSuccess) {
            t->ms[iv.stage] += ms;
            t->count[iv.stage] += 1;
        }
        t->pool.push_back(iv.a);
        t->pool.push_back(iv.b);
    }
    t->open.clear();
}

// RAII bracket around one stage: records on the bound stream when enabled
struct StageScope {
    sph_ctx *c;
    int stage;
    hipEvent_t a = nullptr;
    StageScope(sph_ctx *c_, int st) : c(c_), stage(st)
    {
        if (c->timing && c->timer) {
            if (c->timer->open.size() > 4096) {
                (void)hipStreamSynchronize(c->stream);
                timer_collect(c->timer);
            }
            a = timer_event(c->timer);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~StageScope()
    {
        if (a) {
            hipEvent_t b = timer_event(c->timer);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->timer->open.push_back({stage, a, b});
            } else {
                c->timer->pool.push_back(a);
            }
        }
    }
};

static char g_params_error[256];

static int set_err(sph_ctx *c, int code, const char *msg)
{
    if (c) snprintf(c->err, sizeof(c->err), "%s", msg);
    return code;
}

static int hip_check(sph_ctx *c, hipError_t e, const char *where)
{
    if (e == hipSuccess) return SPH_OK;
    if (c) snprintf(c->err, sizeof(c->err), "%s: %s", where, hipGetErrorString(e));
    return SPH_EHIP;
}

extern "C" void sph_default_params(sph_params *p)
{
    memset(p, 0, sizeof(*p));
    p->list_stride = 128;
    p->extra_slots = 48;
    p->kernel = SPH_KERNEL_M4;
    p->n_target = 100;
    p->n_tol = 5;
    p->h_max_iter = 32;
    p->precision = SPH_FP64;
    p->gamma = 5.0 / 3.0;
    p->av_alpha = 1.0;
    p->av_beta = 2.0;
    p->av_eta2 = 0.01;
    p->cfl = 0.3;
    p->h_mode = SPH_H_PLAIN;
    p->check_finite = 0;
    p->max_level = 6;
    p->search_div = 2;
    p->walk_prefilter = SPH_PREFILTER_MATRIX;
    p->integrator = SPH_INTEGRATOR_KDK;
    p->volumes = SPH_VOLUMES_STANDARD;
    p->gve_exponent = 0.7;
}

extern "C" const char *sph_params_error(void) { return g_params_error; }

static const char *validate(const sph_params *p)
{
    if (p->n_max < 0 || p->n_max > (int64_t)INT32_MAX - 1) return "n_max out of range";
    if (p->list_stride < 1 || p->list_stride > 4096) return "list_stride out of range";
    if (p->extra_slots < 1 || p->extra_slots > 4096) return "extra_slots out of range";
    if (p->kernel != SPH_KERNEL_M4 && p->kernel != SPH_KERNEL_WENDLAND && p->kernel != SPH_KERNEL_SINC5)
        return "kernel must be SPH_KERNEL_M4, SPH_KERNEL_WENDLAND or SPH_KERNEL_SINC5";
    if (p->n_target < 1 || p->n_target > 1000) return "n_target out of range";
    if (p->n_tol < 0 || p->n_tol >= p->n_target) return "n_tol out of range";
    if (p->h_max_iter < 1 || p->h_max_iter > 256) return "h_max_iter out of range";
    if (p->precision != SPH_FP64 && p->precision != SPH_MIXED) return "unknown precision";
    if (p->h_mode != SPH_H_PLAIN && p->h_mode != SPH_H_LEARNED) return "unknown h_mode";
    if (p->max_level < 1 || p->max_level > 8) return "max_level must be in 1..8";
    if (p->search_div < 1 || p->search_div > 4) return "search_div must be in 1..4";
    if (p->integrator != SPH_INTEGRATOR_KDK && p->integrator != SPH_INTEGRATOR_AB2)
        return "integrator must be SPH_INTEGRATOR_KDK or SPH_INTEGRATOR_AB2";
    if (p->grad_h != 0 && p->grad_h != 1) return "grad_h must be 0 or 1";
    if (p->walk_defer_group < 0 || p->walk_defer_group > 64)
        return "walk_defer_group must be in 0..64";
    if (p->gradients != SPH_GRADIENTS_KERNEL && p->gradients != SPH_GRADIENTS_IAD)
        return "gradients must be SPH_GRADIENTS_KERNEL or SPH_GRADIENTS_IAD";
    if (p->walk_prefilter != SPH_PREFILTER_NONE && p->walk_prefilter != SPH_PREFILTER_MATRIX)
        return "walk_prefilter must be SPH_PREFILTER_NONE or SPH_PREFILTER_MATRIX";
    if (p->walk_strategy < SPH_WALK_AUTO || p->walk_strategy > SPH_WALK_WORKLIST)
        return "walk_strategy must be SPH_WALK_AUTO, SPH_WALK_SHELL_FIRST or SPH_WALK_WORKLIST";
    if (p->learned_try_shell < SPH_TRY_SHELL_AUTO || p->learned_try_shell > SPH_TRY_SHELL_ALWAYS)
        return "learned_try_shell must be SPH_TRY_SHELL_AUTO, SPH_TRY_SHELL_NEVER or "
               "SPH_TRY_SHELL_ALWAYS";
    if (p->volumes != SPH_VOLUMES_STANDARD && p->volumes != SPH_VOLUMES_GENERALIZED)
        return "volumes must be SPH_VOLUMES_STANDARD or SPH_VOLUMES_GENERALIZED";
    if (p->volumes == SPH_VOLUMES_GENERALIZED) {
        if (p->grad_h || p->gradients != SPH_GRADIENTS_KERNEL)
            return "generalized volume elements are not combined with grad_h or IAD gradients";
        if (!(p->gve_exponent >= 0.0 && p->gve_exponent <= 1.0))
            return "gve_exponent must be in [0, 1]";
    }
    if (!(p->gamma > 1.0)) return "gamma must exceed 1";
    if (!(p->cfl > 0.0)) return "cfl must be positive";
    if (!(p->av_eta2 > 0.0)) return "av_eta2 must be positive";
    for (int d = 0; d < 3; ++d)
        if (p->periodic[d] && !(p->box_hi[d] > p->box_lo[d])) return "periodic box has no extent";
    return nullptr;
}

// Carves the workspace; with base == nullptr only the size is computed.
size_t sph_layout(const sph_params *p, void *base, Workspace *w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = (off + 255) & ~(size_t)255;
        void *ptr = base ? (void *)((char *)base + off) : nullptr;
        off += bytes;
        return ptr;
    };
    int64_t n = p->n_max > 0 ? p->n_max : 1;
    int64_t nb_fine = ceil_div(n, SPH_BLOCK);
    int64_t nb_red = nb_fine < 2048 ? nb_fine : 2048;
    int64_t nb_sort = ceil_div(n, SPH_SORT_TILE);
    int64_t scan_n = 256 * nb_sort > n + 1 ? 256 * nb_sort : n + 1;
    int64_t scan_part = ceil_div(scan_n, SPH_SCAN_TILE) + 2;
    int64_t ncell = ((int64_t)1 << (3 * p->max_level)) + 1;
    // reduction partials: 8 per block of the reductions, one per block of
    // the force kernels (at least 32 particles each) and 256 slice minima
    const int64_t nb_pair = ceil_div(n, 32) + 256;
    int64_t red_len = nb_pair > 2048 * 8 ? nb_pair : 2048 * 8;
    Workspace t;
    t.bbox = (double *)take(6 * sizeof(double));
    t.bbox_part = (double *)take(nb_red * 6 * sizeof(double));
    t.key_a = (uint32_t *)take(n * sizeof(uint32_t));
    t.key_b = (uint32_t *)take(n * sizeof(uint32_t));
    t.val_a = (int32_t *)take(n * sizeof(int32_t));
    t.val_b = (int32_t *)take(n * sizeof(int32_t));
    t.hist = (uint32_t *)take(256 * nb_sort * sizeof(uint32_t));
    t.scan_part = (uint64_t *)take(scan_part * sizeof(uint64_t));
    t.cell_start = (int32_t *)take(ncell * sizeof(int32_t));
    t.hk = (double *)take(1024 * sizeof(double));
    t.status = (int64_t *)take(ST_COUNT * sizeof(int64_t));
    t.learn_step = (int64_t *)take(4 * sizeof(int64_t));
    t.dt_cur = (double *)take(sizeof(double));
    t.red_part = (double *)take(red_len * sizeof(double));
    t.refill = (uint8_t *)take(n);
    t.work = (int32_t *)take(n * sizeof(int32_t));
    t.woff = (int64_t *)take((n + 1) * sizeof(int64_t));
    t.wl = (int32_t *)take(n * sizeof(int32_t));
    t.hs_next = (double *)take(n * sizeof(double));
    t.hs_lo = (double *)take(n * sizeof(double));
    t.hs_hi = (double *)take(n * sizeof(double));
    t.hs_best_h = (double *)take(n * sizeof(double));
    t.hs_last_h = (double *)take(n * sizeof(double));
    t.hs_best_n = (int32_t *)take(n * sizeof(int32_t));
    t.hs_itk = (int32_t *)take(n * sizeof(int32_t));
    t.hs_bits = (int32_t *)take(n * sizeof(int32_t));
    t.shell_stride = ceil_div(n, 64) * 64;
    t.shell_e = (int2 *)take(SPH_SHELL_SLOTS * t.shell_stride * sizeof(int2));
    t.mixrec = p->precision == SPH_MIXED ? take(n * 64) : nullptr;
    t.mlp_master = (float *)take(SPH_MLP_ROW * sizeof(float));
    t.mlp_m = (float *)take(SPH_MLP_ROW * sizeof(float));
    t.mlp_v = (float *)take(SPH_MLP_ROW * sizeof(float));
    t.mlp_grad = (float *)take(SPH_MLP_ROW * sizeof(float));
    t.mlp_wb = (uint16_t *)take(SPH_MLP_ROW * sizeof(uint16_t));
    t.mlp_norm = (double *)take(12 * sizeof(double));
    t.mlp_part = (float *)take((size_t)SPH_MLP_TRAIN_WAVES * SPH_MLP_ROW * sizeof(float));
    t.h_try = p->h_mode == SPH_H_LEARNED ? (double *)take(n * sizeof(double)) : nullptr;
    t.pk64 = p->precision == SPH_FP64 ? take(n * 80) : nullptr;
    const bool ab2 = p->integrator == SPH_INTEGRATOR_AB2;
    t.du_prev[0] = ab2 ? (double *)take(n * sizeof(double)) : nullptr;
    t.du_prev[1] = ab2 ? (double *)take(n * sizeof(double)) : nullptr;
    t.dt_prev = (double *)take(sizeof(double));
    t.omega = p->grad_h ? (double *)take(n * sizeof(double)) : nullptr;
    t.iad = p->gradients == SPH_GRADIENTS_IAD ? (double2 *)take(n * 3 * sizeof(double2)) : nullptr;
    const bool gve = p->volumes == SPH_VOLUMES_GENERALIZED;
    t.gve_x = gve ? (double *)take(n * sizeof(double)) : nullptr;
    t.gve_y = gve ? (double *)take(n * sizeof(double)) : nullptr;
    t.nb_red = nb_red;
    t.nb_sort = nb_sort;
    t.scan_part_len = scan_part;
    if (w) *w = t;
    return off + 256;
}

// B_5 = 1 / (4 pi int_0^2 sinc^5(pi v / 2) v^2 dv): the normalisation of the
// sinc kernel (its volume integral is one), by 5-point Gauss-Legendre on 64
// equal subintervals
static double sinc5_norm()
{
    const double a = 2.0 * sqrt(10.0 / 7.0);
    const double xg[5] = {-sqrt(5.0 + a) / 3.0, -sqrt(5.0 - a) / 3.0, 0.0, sqrt(5.0 - a) / 3.0,
                          sqrt(5.0 + a) / 3.0};
    const double wo = (322.0 - 13.0 * sqrt(70.0)) / 900.0, wi = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
    const double wg[5] = {wo, wi, 128.0 / 225.0, wi, wo};
    const int m = 64;
    const double hsub = 2.0 / m;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
        const double mid = (k + 0.5) * hsub;
        for (int g = 0; g < 5; ++g) {
            const double v = mid + 0.5 * hsub * xg[g];
            const double xx = 0.5 * M_PI * v;
            const double sc = xx == 0.0 ? 1.0 : sin(xx) / xx;
            acc += wg[g] * 0.5 * hsub * (sc * sc * sc * sc * sc) * v * v;
        }
    }
    return 1.0 / (4.0 * M_PI * acc);
}

extern "C" int sph_create(const sph_params *p, sph_ctx **out)
{
    if (!p || !out) return SPH_EINVAL;
    *out = nullptr;
    const char *e = validate(p);
    if (e) {
        snprintf(g_params_error, sizeof(g_params_error), "%s", e);
        return SPH_EINVAL;
    }
    sph_ctx *c = new (std::nothrow) sph_ctx;
    if (!c) return SPH_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->p = *p;
    c->knorm = sinc5_norm();
    *out = c;
    return SPH_OK;
}

extern "C" void sph_destroy(sph_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->timer) {
        (void)hipStreamSynchronize(ctx->stream);
        for (auto &iv : ctx->timer->open) {
            (void)hipEventDestroy(iv.a);
            (void)hipEventDestroy(iv.b);
        }
        for (auto e : ctx->timer->pool) (void)hipEventDestroy(e);
        delete ctx->timer;
    }
    delete ctx;
}

extern "C" int sph_timing(sph_ctx *c, int enable)
{
    if (!c) return SPH_EINVAL;
    if (!c->timer) c->timer = new (std::nothrow) StageTimer;
    if (!c->timer) return SPH_ENOMEM;
    if (enable) {
        (void)hipStreamSynchronize(c->stream);
        timer_collect(c->timer);
        for (int k = 0; k < SPH_NSTAGES; ++k) {
            c->timer->ms[k] = 0.0;
            c->timer->count[k] = 0;
        }
    }
    c->timing = enable ? 1 : 0;
    return SPH_OK;
}

extern "C" int sph_timing_read(sph_ctx *c, double *ms, int64_t *count, int nstages)
{
    if (!c || nstages < 0) return SPH_EINVAL;
    if (!c->timer) c->timer = new (std::nothrow) StageTimer;
    if (!c->timer) return SPH_ENOMEM;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return set_err(c, SPH_EHIP, "sync");
    timer_collect(c->timer);
    for (int k = 0; k < nstages && k < SPH_NSTAGES; ++k) {
        if (ms) ms[k] = c->timer->ms[k];
        if (count) count[k] = c->timer->count[k];
    }
    return SPH_OK;
}

extern "C" int sph_workspace_size(const sph_params *p, size_t *bytes)
{
    if (!p || !bytes) return SPH_EINVAL;
    if (validate(p)) return SPH_EINVAL;
    *bytes = sph_layout(p, nullptr, nullptr);
    return SPH_OK;
}

// Hernquist & Katz (1989) factor table: T[0] = 2 and
// T[k] = clamp((1 + (n_target / k)^(1/3)) / 2, 1/2, 2).
static void hk_factors(int n_target, double *T)
{
    for (int k = 0; k < 1024; ++k) {
        double v = 2.0;
        if (k > 0) {
            v = 0.5 * (1.0 + cbrt((double)n_target / (double)k));
            v = v < 0.5 ? 0.5 : (v > 2.0 ? 2.0 : v);
        }
        T[k] = v;
    }
}

extern "C" int sph_bind(sph_ctx *c, void *workspace, size_t bytes, void *stream)
{
    if (!c || !workspace) return SPH_EINVAL;
    size_t need = sph_layout(&c->p, nullptr, nullptr);
    if (bytes < need) return set_err(c, SPH_ENOMEM, "workspace smaller than sph_workspace_size()");
    // align the base to 256 bytes inside the caller's buffer
    uintptr_t b = ((uintptr_t)workspace + 255) & ~(uintptr_t)255;
    if (b + (need - 256) > (uintptr_t)workspace + bytes)
        return set_err(c, SPH_ENOMEM, "workspace too small after alignment");
    c->ws_base = workspace;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)stream;
    sph_layout(&c->p, (void *)b, &c->w);
    double T[1024];
    hk_factors(c->p.n_target, T);
    int r = hip_check(c, hipMemcpyAsync(c->w.hk, T, sizeof(T), hipMemcpyHostToDevice, c->stream),
                      "upload factor table");
    if (r) return r;
    r = hip_check(c, hipMemsetAsync(c->w.status, 0, ST_COUNT * sizeof(int64_t), c->stream),
                  "clear status");
    if (r) return r;
    r = hip_check(c, hipMemsetAsync(c->w.learn_step, 0, 4 * sizeof(int64_t), c->stream),
                  "clear learned-try counters");
    if (r) return r;
    r = hip_check(c, hipMemsetAsync(c->w.dt_cur, 0, sizeof(double), c->stream), "clear dt");
    if (r) return r;
    r = hip_check(c, hipMemsetAsync(c->w.dt_prev, 0, sizeof(double), c->stream), "clear dt_prev");
    if (r) return r;
    // MLP state: zero parameters and moments, standardisation (0, 1)
    const double norm0[12] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1};
    r = hip_check(c, hipMemcpyAsync(c->w.mlp_norm, norm0, sizeof(norm0), hipMemcpyHostToDevice,
                                    c->stream), "upload standardisation");
    if (r) return r;
    for (float *q : {c->w.mlp_master, c->w.mlp_m, c->w.mlp_v, c->w.mlp_grad}) {
        r = hip_check(c, hipMemsetAsync(q, 0, SPH_MLP_ROW * sizeof(float), c->stream), "clear MLP");
        if (r) return r;
    }
    r = hip_check(c, hipMemsetAsync(c->w.mlp_wb, 0, SPH_MLP_ROW * sizeof(uint16_t), c->stream),
                  "clear MLP");
    if (r) return r;
    c->mlp_ready = 0;
    c->ab2_hist = 0;
    c->mlp_t = 0;
    c->harvest_feat = nullptr;
    c->harvest_target = nullptr;
    // the factor table lives in a host array: wait for the copy
    r = hip_check(c, hipStreamSynchronize(c->stream), "bind");
    if (r) return r;
    c->bound = 1;
    return SPH_OK;
}

static int check_particles(sph_ctx *c, const sph_particles *s)
{
    if (!c) return SPH_EINVAL;
    if (!c->bound) return set_err(c, SPH_ENOMEM, "no workspace bound");
    if (!s) return set_err(c, SPH_EINVAL, "particles is NULL");
    if (s->n < 0 || s->n > c->p.n_max) return set_err(c, SPH_EINVAL, "n outside [0, n_max]");
    if (s->cur != 0 && s->cur != 1) return set_err(c, SPH_EINVAL, "cur must be 0 or 1");
    if (s->n > 0) {
        for (int k = 0; k < 2; ++k) {
            const void *f[] = {s->x[k], s->y[k], s->z[k], s->vx[k], s->vy[k], s->vz[k],
                               s->m[k], s->h[k], s->u[k], s->ax[k], s->ay[k], s->az[k],
                               s->du[k], s->rho[k], s->divv[k], s->nc[k], s->id[k]};
            for (const void *q : f)
                if (!q) return set_err(c, SPH_EINVAL, "a carried field pointer is NULL");
        }
        const void *g[] = {s->pvx, s->pvy, s->pvz, s->pu, s->p, s->c, s->flags, s->key, s->perm};
        for (const void *q : g)
            if (!q) return set_err(c, SPH_EINVAL, "a single-buffer pointer is NULL");
    }
    return SPH_OK;
}

static int check_nlist(sph_ctx *c, const sph_particles *s, const sph_nlist *nl)
{
    if (!nl) return set_err(c, SPH_EINVAL, "nlist is NULL");
    if (s->n > 0 && (!nl->idx || !nl->ecnt || !nl->eidx))
        return set_err(c, SPH_EINVAL, "an nlist pointer is NULL");
    if (nl->stride < s->n || (nl->stride % 64) != 0)
        return set_err(c, SPH_EINVAL, "nlist stride must be >= n and a multiple of 64");
    return SPH_OK;
}

#define TRY(expr, where)                                  \
    do {                                                  \
        int _r = hip_check(c, (expr), where);             \
        if (_r) return _r;                                \
    } while (0)

extern "C" int sph_build_cells(sph_ctx *c, sph_particles *s)
{
    int r = check_particles(c, s);
    if (r) return r;
    int k = s->cur;
    StageScope scope(c, SPH_STAGE_CELLS);
    TRY(launch_bbox(c, s->x[k], s->y[k], s->z[k], s->n), "bbox");
    TRY(launch_keys(c, s->x[k], s->y[k], s->z[k], s->n), "keys");
    TRY(launch_radix_sort(c, s->n, s->key, s->perm), "radix sort");
    TRY(launch_permute(c, s, s->perm), "permute");
    s->cur = 1 - s->cur;
    TRY(launch_cell_table(c, s->key, s->n), "cell table");
    return SPH_OK;
}

// A5-A6; with_extra = false leaves the complement to the fused density pass
static int find_neighbors_impl(sph_ctx *c, sph_particles *s, sph_nlist *nl, const double *h_try,
                               bool with_extra)
{
    {
        StageScope scope(c, SPH_STAGE_HSOLVE);
        {
            StageScope walk(c, SPH_STAGE_HWALK);
            TRY(launch_hsolve(c, s, nl, h_try, 0), "h iteration (first counts)");
        }
        TRY(launch_hsolve(c, s, nl, h_try, 1), "h iteration");
    }
    if (with_extra) {
        StageScope scope(c, SPH_STAGE_EXTRA);
        TRY(launch_extra(c, s, nl), "complement lists");
    }
    return SPH_OK;
}

// learned mode: predicted smoothing lengths of this step into w.h_try
static int mlp_predict(sph_ctx *c, sph_particles *s, const double **h_try)
{
    *h_try = nullptr;
    if (c->p.h_mode != SPH_H_LEARNED) return SPH_OK;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "learned h mode: no MLP weights set");
    StageScope scope(c, SPH_STAGE_MLP);
    TRY(launch_mlp_predict(c, s, c->w.h_try), "MLP prediction");
    *h_try = c->w.h_try;
    return SPH_OK;
}

extern "C" int sph_find_neighbors(sph_ctx *c, sph_particles *s, sph_nlist *nl)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    const double *h_try = nullptr;
    r = mlp_predict(c, s, &h_try);
    if (r) return r;
    return find_neighbors_impl(c, s, nl, h_try, true);
}

extern "C" int sph_density(sph_ctx *c, sph_particles *s, const sph_nlist *nl)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    StageScope scope(c, SPH_STAGE_DENSITY);
    if (c->p.precision == SPH_MIXED) TRY(launch_density_mixed(c, s, nl, false), "density (mixed)");
    else TRY(launch_density(c, s, nl, false), "density");
    return SPH_OK;
}

extern "C" int sph_eos(sph_ctx *c, sph_particles *s)
{
    int r = check_particles(c, s);
    if (r) return r;
    StageScope scope(c, SPH_STAGE_EOS);
    if (c->p.precision == SPH_MIXED) TRY(launch_eos_mixed(c, s), "eos (mixed)");
    else TRY(launch_eos(c, s), "eos");
    return SPH_OK;
}

extern "C" int sph_momentum_energy(sph_ctx *c, sph_particles *s, const sph_nlist *nl, double *d_dt)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    {
        StageScope scope(c, SPH_STAGE_FORCES);
        if (c->p.precision == SPH_MIXED) TRY(launch_forces_mixed(c, s, nl), "forces (mixed)");
        else TRY(launch_forces(c, s, nl, d_dt), "forces");
    }
    TRY(launch_dt_min(c, s->n, d_dt), "dt minimum");
    return SPH_OK;
}

// A5-A9 on the sorted state with pv/pu already set
static int evaluate_sorted(sph_ctx *c, sph_particles *s, sph_nlist *nl, double *d_dt,
                           const double *h_try)
{
    int r = find_neighbors_impl(c, s, nl, h_try, false);
    if (r) return r;
    const bool mixed = c->p.precision == SPH_MIXED;
    {
        // density and divergence, with the complement E built in the same pass
        StageScope scope(c, SPH_STAGE_DENSITY);
        if (mixed) TRY(launch_density_mixed(c, s, nl, true), "density (mixed)");
        else TRY(launch_density(c, s, nl, true), "density");
    }
    {
        StageScope scope(c, SPH_STAGE_EOS);
        if (mixed) TRY(launch_eos_mixed(c, s), "eos (mixed)");
        else TRY(launch_eos(c, s), "eos");
    }
    {
        StageScope scope(c, SPH_STAGE_FORCES);
        if (mixed) TRY(launch_forces_mixed(c, s, nl), "forces (mixed)");
        else TRY(launch_forces(c, s, nl, d_dt), "forces");
    }
    TRY(launch_dt_min(c, s->n, d_dt), "dt minimum");
    return SPH_OK;
}

extern "C" int sph_evaluate(sph_ctx *c, sph_particles *s, sph_nlist *nl, double *d_dt)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    if (!d_dt) return set_err(c, SPH_EINVAL, "d_dt is NULL");
    r = sph_build_cells(c, s);
    if (r) return r;
    TRY(launch_copy_pred(c, s), "copy prediction");
    c->ab2_hist = 0;   // the integrator starts afresh from this state
    c->gve_fresh = 1;  // generalized weights from the standard density at this h
    r = evaluate_sorted(c, s, nl, d_dt, nullptr);
    c->gve_fresh = 0;
    return r;
}

extern "C" int sph_step(sph_ctx *c, sph_particles *s, sph_nlist *nl, double dt, double *d_dt)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    if (!d_dt) return set_err(c, SPH_EINVAL, "d_dt is NULL");
    if (!(dt > 0.0) && !(dt <= 0.0)) return set_err(c, SPH_EINVAL, "dt is NaN");
    {
        StageScope scope(c, SPH_STAGE_INTEGRATE);
        TRY(launch_set_dt(c, dt, d_dt), "set dt");
        TRY(launch_kick_drift(c, s), "kick-drift");
    }
    r = sph_build_cells(c, s);
    if (r) return r;
    {
        StageScope scope(c, SPH_STAGE_INTEGRATE);
        TRY(launch_predict(c, s), "predict");
    }
    if (c->harvest_feat) {
        StageScope scope(c, SPH_STAGE_MLP);
        TRY(launch_mlp_features(c, s, c->w.dt_cur, c->harvest_feat), "harvest features");
    }
    const double *h_try = nullptr;
    r = mlp_predict(c, s, &h_try);
    if (r) return r;
    r = evaluate_sorted(c, s, nl, d_dt, h_try);
    if (r) return r;
    if (c->harvest_feat) {
        StageScope scope(c, SPH_STAGE_MLP);
        TRY(launch_mlp_targets(c, s, c->harvest_feat, c->harvest_target,
                               c->harvest_mode == SPH_TARGET_CENTRED), "harvest targets");
    }
    {
        StageScope scope(c, SPH_STAGE_INTEGRATE);
        TRY(launch_kick(c, s), "kick");
    }
    c->ab2_hist = 1;
    return SPH_OK;
}

extern "C" int sph_conservation(sph_ctx *c, const sph_particles *s, double *d_out7)
{
    int r = check_particles(c, s);
    if (r) return r;
    if (!d_out7) return set_err(c, SPH_EINVAL, "d_out7 is NULL");
    TRY(launch_conservation(c, s, d_out7), "conservation");
    return SPH_OK;
}

extern "C" int sph_interaction_csr(sph_ctx *c, const sph_particles *s, const sph_nlist *nl,
                                   int64_t *d_off, int32_t *d_idx, int64_t capacity)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    if (!d_off) return set_err(c, SPH_EINVAL, "d_off is NULL");
    if (capacity < 0) return set_err(c, SPH_EINVAL, "capacity < 0");
    if (capacity > 0 && !d_idx) return set_err(c, SPH_EINVAL, "d_idx is NULL");
    TRY(launch_interaction_csr(c, s, nl, d_off, d_idx, capacity), "interaction csr");
    return SPH_OK;
}

extern "C" int sph_sync(sph_ctx *c, sph_stats *st)
{
    if (!c) return SPH_EINVAL;
    if (!c->bound) return set_err(c, SPH_ENOMEM, "no workspace bound");
    int64_t h[ST_COUNT];
    TRY(hipStreamSynchronize(c->stream), "sync");
    TRY(hipMemcpy(h, c->w.status, sizeof(h), hipMemcpyDeviceToHost), "read status");
    TRY(hipMemsetAsync(c->w.status, 0, sizeof(h), c->stream), "clear status");
    TRY(hipStreamSynchronize(c->stream), "sync");
    if (st) {
        memset(st, 0, sizeof(*st));
        st->nonconverged = h[ST_NONCONV];
        st->list_overflow = h[ST_LIST_OVERFLOW];
        st->extra_overflow = h[ST_EXTRA_OVERFLOW];
        st->nonfinite = h[ST_NONFINITE];
        st->h_counts = h[ST_HCOUNTS];
        st->learned_accepted = h[ST_LEARN_ACC];
        st->learned_fallback = h[ST_LEARN_FALLBACK];
        st->candidates = h[ST_CANDIDATES];
        st->extra_total = h[ST_EXTRA_TOTAL];
        st->candidates_first = h[ST_CANDIDATES_FIRST];
        st->iad_singular = h[ST_IAD_SINGULAR];
        st->csr_overflow = h[ST_CSR_OVERFLOW];
    }
    if (h[ST_LIST_OVERFLOW] || h[ST_EXTRA_OVERFLOW] || h[ST_CSR_OVERFLOW])
        return set_err(c, SPH_ECAPACITY, "a neighbour list exceeded its capacity");
    if (h[ST_NONFINITE]) return set_err(c, SPH_ENONFINITE, "non-finite field values");
    if (h[ST_IAD_SINGULAR]) return set_err(c, SPH_ENONFINITE, "singular IAD moment matrix");
    if (h[ST_NONCONV]) return SPH_WNOCONV;
    return SPH_OK;
}

extern "C" const char *sph_last_error(const sph_ctx *c) { return c ? c->err : "no context"; }

extern "C" int sph_copy_internal(sph_ctx *c, int which, void *dst, size_t bytes, size_t *needed)
{
    if (!c || !needed) return SPH_EINVAL;
    if (!c->bound) return set_err(c, SPH_ENOMEM, "no workspace bound");
    const void *src = nullptr;
    size_t sz = 0;
    if (which == 0) {
        src = c->w.cell_start;
        sz = (((size_t)1 << (3 * c->p.max_level)) + 1) * sizeof(int32_t);
    } else if (which == 1) {
        src = c->w.bbox;
        sz = 6 * sizeof(double);
    } else {
        return set_err(c, SPH_EINVAL, "unknown table");
    }
    *needed = sz;
    if (!dst) return SPH_OK;
    if (bytes < sz) return set_err(c, SPH_EINVAL, "destination too small");
    TRY(hipMemcpyAsync(dst, src, sz, hipMemcpyDeviceToDevice, c->stream), "copy internal");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// learned smoothing length
// ---------------------------------------------------------------------------
static int check_bound(sph_ctx *c)
{
    if (!c) return SPH_EINVAL;
    if (!c->bound) return set_err(c, SPH_ENOMEM, "no workspace bound");
    return SPH_OK;
}

extern "C" int sph_mlp_set_weights(sph_ctx *c, const float *params, const double *norm12)
{
    int r = check_bound(c);
    if (r) return r;
    if (!params) return set_err(c, SPH_EINVAL, "params is NULL");
    if (norm12)
        for (int k = 0; k < 6; ++k)
            if (!(norm12[6 + k] > 0.0) || !(norm12[k] == norm12[k]))
                return set_err(c, SPH_EINVAL, "standardisation std must be positive");
    TRY(hipMemcpyAsync(c->w.mlp_master, params, SPH_MLP_NPARAM * sizeof(float),
                       hipMemcpyHostToDevice, c->stream), "upload MLP parameters");
    if (norm12)
        TRY(hipMemcpyAsync(c->w.mlp_norm, norm12, 12 * sizeof(double), hipMemcpyHostToDevice,
                           c->stream), "upload standardisation");
    TRY(hipMemsetAsync(c->w.mlp_m, 0, SPH_MLP_ROW * sizeof(float), c->stream), "clear Adam");
    TRY(hipMemsetAsync(c->w.mlp_v, 0, SPH_MLP_ROW * sizeof(float), c->stream), "clear Adam");
    TRY(launch_mlp_refresh(c), "bf16 copy");
    TRY(hipStreamSynchronize(c->stream), "sync");   // host sources
    c->mlp_ready = 1;
    c->mlp_t = 0;
    return SPH_OK;
}

extern "C" int sph_mlp_get_weights(sph_ctx *c, float *params, double *norm12)
{
    int r = check_bound(c);
    if (r) return r;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "no MLP weights set");
    TRY(hipStreamSynchronize(c->stream), "sync");
    if (params)
        TRY(hipMemcpy(params, c->w.mlp_master, SPH_MLP_NPARAM * sizeof(float),
                      hipMemcpyDeviceToHost), "download MLP parameters");
    if (norm12)
        TRY(hipMemcpy(norm12, c->w.mlp_norm, 12 * sizeof(double), hipMemcpyDeviceToHost),
            "download standardisation");
    return SPH_OK;
}

extern "C" int sph_mlp_fit_norm(sph_ctx *c, const float *d_feat, int64_t n)
{
    int r = check_bound(c);
    if (r) return r;
    if (!d_feat || n < 1) return set_err(c, SPH_EINVAL, "need n >= 1 feature rows");
    TRY(launch_mlp_fit_norm(c, d_feat, n), "standardisation");
    return SPH_OK;
}

extern "C" int sph_get_features(sph_ctx *c, const sph_particles *s, const double *d_dt,
                                float *d_feat)
{
    int r = check_particles(c, s);
    if (r) return r;
    if (!d_dt || (s->n > 0 && !d_feat)) return set_err(c, SPH_EINVAL, "NULL pointer");
    TRY(launch_mlp_features(c, s, d_dt, d_feat), "features");
    return SPH_OK;
}

extern "C" int sph_get_omega(sph_ctx *c, const sph_particles *s, double *d_omega)
{
    int r = check_particles(c, s);
    if (r) return r;
    if (!c->p.grad_h) return set_err(c, SPH_EINVAL, "context created without grad_h");
    if (s->n > 0 && !d_omega) return set_err(c, SPH_EINVAL, "NULL pointer");
    if (s->n > 0)
        TRY(hipMemcpyAsync(d_omega, c->w.omega, s->n * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream), "copy omega");
    return SPH_OK;
}

extern "C" int sph_set_harvest(sph_ctx *c, float *d_feat, float *d_target, int32_t target_mode)
{
    int r = check_bound(c);
    if (r) return r;
    if ((d_feat == nullptr) != (d_target == nullptr))
        return set_err(c, SPH_EINVAL, "harvest needs both arrays or neither");
    if (target_mode != SPH_TARGET_SOLVED && target_mode != SPH_TARGET_CENTRED)
        return set_err(c, SPH_EINVAL, "unknown target mode");
    c->harvest_feat = d_feat;
    c->harvest_target = d_target;
    c->harvest_mode = target_mode;
    return SPH_OK;
}

extern "C" int sph_mlp_forward(sph_ctx *c, const float *d_feat, int64_t n, float *d_y,
                               uint16_t *d_h1, uint16_t *d_h2)
{
    int r = check_bound(c);
    if (r) return r;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "no MLP weights set");
    if (n < 0) return set_err(c, SPH_EINVAL, "n < 0");
    if (n > 0 && (!d_feat || !d_y)) return set_err(c, SPH_EINVAL, "NULL pointer");
    TRY(launch_mlp_forward(c, d_feat, n, d_y, d_h1, d_h2), "MLP forward");
    return SPH_OK;
}

extern "C" int sph_mlp_backward(sph_ctx *c, const float *d_feat, const float *d_target,
                                const int32_t *d_rows, int64_t row0, int64_t n, float *d_grad)
{
    int r = check_bound(c);
    if (r) return r;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "no MLP weights set");
    if (n < 1 || row0 < 0) return set_err(c, SPH_EINVAL, "need n >= 1 and row0 >= 0");
    if (!d_feat || !d_target || !d_grad) return set_err(c, SPH_EINVAL, "NULL pointer");
    TRY(launch_mlp_grad(c, d_feat, d_target, d_rows, row0, n, d_grad, nullptr), "MLP backward");
    return SPH_OK;
}

extern "C" int sph_mlp_adam_step(sph_ctx *c, const float *d_grad, double lr, double beta1,
                                 double beta2, double eps, int32_t t)
{
    int r = check_bound(c);
    if (r) return r;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "no MLP weights set");
    if (!d_grad || t < 1) return set_err(c, SPH_EINVAL, "need a gradient and t >= 1");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return set_err(c, SPH_EINVAL, "Adam constants out of range");
    TRY(launch_mlp_adam(c, d_grad, lr, beta1, beta2, eps, t), "Adam");
    return SPH_OK;
}

extern "C" int sph_mlp_train(sph_ctx *c, const float *d_feat, const float *d_target,
                             const int32_t *d_order, int64_t n, int32_t batch, int32_t epochs,
                             double lr, float *d_loss)
{
    int r = check_bound(c);
    if (r) return r;
    if (!c->mlp_ready) return set_err(c, SPH_EINVAL, "no MLP weights set");
    if (n < 1 || batch < 1 || epochs < 0) return set_err(c, SPH_EINVAL, "bad sizes");
    if (!d_feat || !d_target) return set_err(c, SPH_EINVAL, "NULL pointer");
    const int64_t nb = ceil_div(n, batch);
    for (int e = 0; e < epochs; ++e)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t row0 = b * batch;
            const int64_t cnt = n - row0 < batch ? n - row0 : batch;
            float *lo = d_loss ? d_loss + (int64_t)e * nb + b : nullptr;
            TRY(launch_mlp_grad(c, d_feat, d_target, d_order, row0, cnt, c->w.mlp_grad, lo),
                "MLP backward");
            TRY(launch_mlp_adam(c, c->w.mlp_grad, lr, 0.9, 0.999, 1e-8, ++c->mlp_t), "Adam");
        }
    return SPH_OK;
}
