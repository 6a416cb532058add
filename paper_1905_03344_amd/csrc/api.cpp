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
}

extern "C" const char *sph_params_error(void) { return g_params_error; }

static const char *validate(const sph_params *p)
{
    if (p->n_max < 0 || p->n_max > (int64_t)INT32_MAX - 1) return "n_max out of range";
    if (p->list_stride < 1 || p->list_stride > 4096) return "list_stride out of range";
    if (p->extra_slots < 1 || p->extra_slots > 4096) return "extra_slots out of range";
    if (p->kernel != SPH_KERNEL_M4) return "unsupported kernel";
    if (p->n_target < 1 || p->n_target > 1000) return "n_target out of range";
    if (p->n_tol < 0 || p->n_tol >= p->n_target) return "n_tol out of range";
    if (p->h_max_iter < 1 || p->h_max_iter > 256) return "h_max_iter out of range";
    if (p->precision != SPH_FP64 && p->precision != SPH_MIXED) return "unknown precision";
    if (p->h_mode != SPH_H_PLAIN && p->h_mode != SPH_H_LEARNED) return "unknown h_mode";
    if (p->max_level < 1 || p->max_level > 8) return "max_level must be in 1..8";
    if (p->search_div < 1 || p->search_div > 4) return "search_div must be in 1..4";
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
    int64_t red_len = nb_fine > 2048 * 8 ? nb_fine : 2048 * 8;
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
    t.shell_j = (int32_t *)take(48 * t.shell_stride * sizeof(int32_t));
    t.shell_r2 = (double *)take(48 * t.shell_stride * sizeof(double));
    t.mixrec = p->precision == SPH_MIXED ? take(n * 64) : nullptr;
    t.nb_red = nb_red;
    t.nb_sort = nb_sort;
    t.scan_part_len = scan_part;
    if (w) *w = t;
    return off + 256;
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
        TRY(launch_hsolve(c, s, nl, h_try), "h iteration");
    }
    if (with_extra) {
        StageScope scope(c, SPH_STAGE_EXTRA);
        TRY(launch_extra(c, s, nl), "complement lists");
    }
    return SPH_OK;
}

extern "C" int sph_find_neighbors(sph_ctx *c, sph_particles *s, sph_nlist *nl)
{
    int r = check_particles(c, s);
    if (r) return r;
    r = check_nlist(c, s, nl);
    if (r) return r;
    return find_neighbors_impl(c, s, nl, nullptr, true);
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
static int evaluate_sorted(sph_ctx *c, sph_particles *s, sph_nlist *nl, double *d_dt)
{
    int r = find_neighbors_impl(c, s, nl, nullptr, false);
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
    return evaluate_sorted(c, s, nl, d_dt);
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
    r = evaluate_sorted(c, s, nl, d_dt);
    if (r) return r;
    {
        StageScope scope(c, SPH_STAGE_INTEGRATE);
        TRY(launch_kick(c, s), "kick");
    }
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
    }
    if (h[ST_LIST_OVERFLOW] || h[ST_EXTRA_OVERFLOW])
        return set_err(c, SPH_ECAPACITY, "a neighbour list exceeded its capacity");
    if (h[ST_NONFINITE]) return set_err(c, SPH_ENONFINITE, "non-finite field values");
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
