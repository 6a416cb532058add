/*
 * sph_oracle.c -- slow, plain FP64 CPU reference of one SPH time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; both sides are
 * fed the same seeded input arrays and nothing else.
 *
 * What it computes (the paper prints only the two kernel formulas and the
 * square-patch initial conditions; every other equation is the standard
 * textbook form of the works the paper names, as listed per function):
 *   - M4 cubic-spline kernel and its radial derivative (kernel section,
 *     support 0 <= v <= 2 as in the Sinc and Wendland equations; M4 is the
 *     spline listed for ChaNGa in Table 1), and the kernel section's own
 *     two kernels: Wendland C2 and the sinc family (exponent 5);
 *   - cell keys: 10-bit-per-dimension Morton interleave of the cell index in
 *     the bounding box, stable sort by key (replaces the tree walk of
 *     Table 1 by a cell list);
 *   - neighbour counts and symmetric interaction lists by brute force and by
 *     a plain row-major uniform grid;
 *   - the smoothing-length iteration (Hernquist & Katz factor, then
 *     bisection once bracketed);
 *   - density sum with "standard" volume elements (Table 1), velocity
 *     divergence, ideal-gas EOS;
 *   - momentum equation (Rosswog 2009 kernel-averaged form, cited in the
 *     co-design section), Monaghan-Gingold artificial viscosity (Monaghan
 *     1983, same section), energy equation and a Courant time step;
 *   - kick-drift-kick leapfrog update and conservation sums (Neumaier);
 *     the paper's own energy update (second-order Adams-Bashforth) as the
 *     alternative integrator, positions and velocities as in KDK;
 *   - accuracy variants of the momentum and energy sums: grad-h factors
 *     (Springel & Hernquist 2002) and IAD gradients (Table 1; Garcia-Senz,
 *     Cabezon & Escartin 2012).
 *   - the learned smoothing-length MLP (6-64-64-1, tanh, bf16 operands)
 *     forward, analytic backward and Adam, in FP64 on bf16-rounded operands.
 *
 * Built with -O2 -ffp-contract=off -fno-fast-math so that every expression
 * is evaluated exactly as written, one IEEE operation at a time.
 *
 * Parity status: the paper publishes no numerical results for any of these
 * quantities; every function is pinned by closed forms, invariants and brute
 * force in the CPU test suite.  The MLP is pinned by finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Kernel: M4 cubic spline, support 2h.                                       */
/* W(r,h) = 1/(pi h^3) * { 1 - 1.5 q^2 + 0.75 q^3   (q<1)                     */
/*                         0.25 (2-q)^3             (1<=q<2)                  */
/*                         0                         (q>=2) },  q = r/h        */
/* ------------------------------------------------------------------------ */
double or_kernel_w(double r, double h)
{
    double q = r / h;
    double norm = 1.0 / (OR_PI * h * h * h);
    if (q < 1.0) return norm * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    if (q < 2.0) {
        double t = 2.0 - q;
        return norm * (0.25 * t * t * t);
    }
    return 0.0;
}

/* dW/dr = 1/(pi h^4) * { -3 q + 2.25 q^2 (q<1); -0.75 (2-q)^2 (1<=q<2); 0 } */
double or_kernel_dwdr(double r, double h)
{
    double q = r / h;
    double norm = 1.0 / (OR_PI * h * h * h * h);
    if (q < 1.0) return norm * (-3.0 * q + 2.25 * q * q);
    if (q < 2.0) {
        double t = 2.0 - q;
        return norm * (-0.75 * t * t);
    }
    return 0.0;
}

/* Wendland C2 in 3D, as printed in the kernel section with the 1/h^3 factor
 * the print omits: W = 21/(16 pi h^3) (1 - v/2)^4 (2 v + 1), 0 <= v <= 2.   */
double or_kernel_wendland(double r, double h)
{
    double v = r / h;
    if (v >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * v;
    return 21.0 / (16.0 * OR_PI * h * h * h) * (t * t * t * t) * (2.0 * v + 1.0);
}

/* dW/dr of the Wendland C2 kernel: d/dv [(1 - v/2)^4 (2v + 1)] = -5 v (1 - v/2)^3 */
double or_kernel_wendland_dwdr(double r, double h)
{
    double v = r / h;
    if (v >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * v;
    return 21.0 / (16.0 * OR_PI * h * h * h * h) * (-5.0 * v) * (t * t * t);
}

/* Sinc kernel of the kernel section, W = B_n / h^3 sinc^n(pi v / 2), 0 <= v <= 2,
 * sinc(x) = sin(x) / x.  The paper gives neither n nor B_n: n = 5 here, and B_n
 * follows from normalisation, B_n = 1 / (4 pi int_0^2 sinc^n(pi v/2) v^2 dv),
 * the integral by composite Simpson on 2^16 intervals.                       */
#define OR_SINC_N 5
static double sinc_val(double x)
{
    /* Taylor series below 1/2 (terms to x^16), sin(x)/x above */
    if (x < 0.5) {
        double x2 = x * x, term = 1.0, s = 1.0;
        for (int k = 1; k <= 8; ++k) {
            term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
            s += term;
        }
        return s;
    }
    return sin(x) / x;
}
static double sinc_deriv(double x)
{
    /* d/dx sin(x)/x = (x cos x - sin x) / x^2; series -x/3 + x^3/30 - ... below 1/2 */
    if (x < 0.5) {
        double x2 = x * x, term = 1.0, s = 0.0;
        for (int k = 1; k <= 8; ++k) {
            term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));   /* (-1)^k x^2k / (2k+1)! */
            s += 2.0 * k * term;
        }
        return s / x;   /* x > 0 here: callers handle x = 0 */
    }
    return (x * cos(x) - sin(x)) / (x * x);
}
static double sinc_pow(double s)
{
    double s2 = s * s;
    return s2 * s2 * s;   /* n = 5 */
}
double or_sinc_norm(void)
{
    static double bn = 0.0;
    if (bn == 0.0) {
        const int m = 1 << 16;
        const double dv = 2.0 / m;
        double acc = 0.0;
        for (int k = 0; k <= m; ++k) {
            double v = k * dv;
            double f = sinc_pow(sinc_val(0.5 * OR_PI * v)) * v * v;
            double wgt = (k == 0 || k == m) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
            acc += wgt * f;
        }
        double integral = acc * dv / 3.0;
        bn = 1.0 / (4.0 * OR_PI * integral);
    }
    return bn;
}
double or_kernel_sinc(double r, double h)
{
    double v = r / h;
    if (v >= 2.0) return 0.0;
    return or_sinc_norm() / (h * h * h) * sinc_pow(sinc_val(0.5 * OR_PI * v));
}
/* dW/dr = B_n / h^4 * n sinc^(n-1)(x) sinc'(x) * pi/2,  x = pi v / 2 */
double or_kernel_sinc_dwdr(double r, double h)
{
    double v = r / h;
    if (v >= 2.0 || v <= 0.0) return 0.0;
    double x = 0.5 * OR_PI * v;
    double s = sinc_val(x);
    double s4 = (s * s) * (s * s);
    return or_sinc_norm() / (h * h * h * h) * (OR_SINC_N * s4 * sinc_deriv(x) * (0.5 * OR_PI));
}

/* kernel selection: 0 = M4, 1 = Wendland C2, 2 = sinc (n = 5) */
static double kern(int kernel, double r, double h)
{
    if (kernel == 1) return or_kernel_wendland(r, h);
    if (kernel == 2) return or_kernel_sinc(r, h);
    return or_kernel_w(r, h);
}
static double kern_dr(int kernel, double r, double h)
{
    if (kernel == 1) return or_kernel_wendland_dwdr(r, h);
    if (kernel == 2) return or_kernel_sinc_dwdr(r, h);
    return or_kernel_dwdr(r, h);
}

/* dW/dh at fixed r: W = h^-3 w(r/h) gives dW/dh = -(3 W + r dW/dr) / h */
double or_kernel_dwdh(int kernel, double r, double h)
{
    return -(3.0 * kern(kernel, r, h) + r * kern_dr(kernel, r, h)) / h;
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *x, *y, *z;
    int per[3];
    double L[3], halfL[3];
} or_geom;

static void geom_init(or_geom *g, const double *x, const double *y, const double *z,
                      const int *periodic, const double *box_lo, const double *box_hi)
{
    g->x = x; g->y = y; g->z = z;
    for (int d = 0; d < 3; ++d) {
        g->per[d] = periodic ? periodic[d] : 0;
        g->L[d] = g->per[d] ? (box_hi[d] - box_lo[d]) : 0.0;
        g->halfL[d] = 0.5 * g->L[d];
    }
}

/* minimum-image component of b - a in dimension d */
static double min_image(const or_geom *g, int d, double a, double b)
{
    double t = b - a;
    if (g->per[d]) {
        if (t > g->halfL[d]) t -= g->L[d];
        else if (t < -g->halfL[d]) t += g->L[d];
    }
    return t;
}

/* r^2 between i and j, evaluated as (dx*dx + dy*dy) + dz*dz with dx = x_j - x_i */
static double pair_r2(const or_geom *g, int64_t i, int64_t j, double *dx, double *dy, double *dz)
{
    double a = min_image(g, 0, g->x[i], g->x[j]);
    double b = min_image(g, 1, g->y[i], g->y[j]);
    double c = min_image(g, 2, g->z[i], g->z[j]);
    if (dx) { *dx = a; *dy = b; *dz = c; }
    double ab = a * a + b * b;
    return ab + c * c;
}

/* ------------------------------------------------------------------------ */
/* Bounding box and cell keys                                                 */
/* ------------------------------------------------------------------------ */
void or_bbox(int64_t n, const double *x, const double *y, const double *z,
             const int *periodic, const double *box_lo, const double *box_hi,
             double *lo, double *hi)
{
    const double *c[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        if (periodic[d]) { lo[d] = box_lo[d]; hi[d] = box_hi[d]; continue; }
        double a = INFINITY, b = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            if (c[d][i] < a) a = c[d][i];
            if (c[d][i] > b) b = c[d][i];
        }
        if (n == 0) { a = 0.0; b = 0.0; }
        lo[d] = a; hi[d] = b;
    }
}

/* integer cell index in [0, 1023] of coordinate v in [lo, lo+L] */
static int cell10(double v, double lo, double L)
{
    double w = L / 1024.0;
    if (!(w > 0.0)) return 0;
    double t = (v - lo) / w;
    if (!(t >= 0.0)) return 0;           /* negative or NaN */
    if (!(t < 1024.0)) return 1023;
    return (int)t;                        /* truncation == floor for t >= 0 */
}

/* Morton interleave, written bit by bit: x bit b -> 3b, y -> 3b+1, z -> 3b+2 */
static uint32_t morton3(int gx, int gy, int gz)
{
    uint32_t key = 0;
    for (int b = 0; b < 10; ++b) {
        key |= (uint32_t)((gx >> b) & 1) << (3 * b);
        key |= (uint32_t)((gy >> b) & 1) << (3 * b + 1);
        key |= (uint32_t)((gz >> b) & 1) << (3 * b + 2);
    }
    return key;
}

void or_cell_keys(int64_t n, const double *x, const double *y, const double *z,
                  const double *lo, const double *hi, uint32_t *key)
{
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        key[i] = morton3(cell10(x[i], lo[0], L[0]), cell10(y[i], lo[1], L[1]),
                         cell10(z[i], lo[2], L[2]));
}

typedef struct { uint32_t key; int64_t pos; } kp_t;
static int kp_cmp(const void *a, const void *b)
{
    const kp_t *p = (const kp_t *)a, *q = (const kp_t *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->pos < q->pos ? -1 : (p->pos > q->pos);
}

/* Stable sort by key: perm[k] = position (in the input order) of the k-th
 * smallest key; equal keys keep their input order. */
void or_sort_perm(int64_t n, const uint32_t *key, int32_t *perm)
{
    kp_t *a = (kp_t *)malloc(sizeof(kp_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { a[i].key = key[i]; a[i].pos = i; }
    qsort(a, (size_t)n, sizeof(kp_t), kp_cmp);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)a[i].pos;
    free(a);
}

/* start[c] = first sorted position whose key lies in level-l cell c, c in
 * [0, 8^l]; keys must be sorted ascending. Found by binary search. */
void or_cell_start(int64_t n, const uint32_t *sorted_key, int level, int32_t *start)
{
    int shift = 3 * (10 - level);
    int64_t ncell = (int64_t)1 << (3 * level);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c <= ncell; ++c) {
        uint64_t target = (uint64_t)c << shift;
        int64_t a = 0, b = n;
        while (a < b) {
            int64_t mid = a + (b - a) / 2;
            if ((uint64_t)sorted_key[mid] < target) a = mid + 1; else b = mid;
        }
        start[c] = (int32_t)a;
    }
}

/* ------------------------------------------------------------------------ */
/* Plain uniform grid (row-major cells), used for neighbour queries.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nc[3];
    double lo[3], cs[3];
    int per[3];
    int64_t *start;  /* ncells + 1 */
    int64_t *item;   /* particle ids grouped by cell */
} or_grid;

static int grid_coord(const or_grid *G, int d, double v)
{
    if (!(G->cs[d] > 0.0)) return 0;
    double t = (v - G->lo[d]) / G->cs[d];
    if (!(t >= 0.0)) return 0;
    if (!(t < (double)G->nc[d])) return G->nc[d] - 1;
    return (int)t;
}

static void grid_build(or_grid *G, int64_t n, const double *x, const double *y, const double *z,
                       const int *periodic, const double *box_lo, const double *box_hi,
                       double target_cell)
{
    double lo[3], hi[3];
    or_bbox(n, x, y, z, periodic, box_lo, box_hi, lo, hi);
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        double L = hi[d] - lo[d];
        int k = (target_cell > 0.0 && L > 0.0) ? (int)floor(L / target_cell) : 1;
        if (k < 1) k = 1;
        if (k > 256) k = 256;
        G->nc[d] = k;
        G->lo[d] = lo[d];
        G->cs[d] = L / k;
        G->per[d] = periodic[d];
        total *= k;
    }
    G->start = (int64_t *)calloc((size_t)total + 1, sizeof(int64_t));
    G->item = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    const double *c[3] = {x, y, z};
    for (int64_t i = 0; i < n; ++i) {
        int g[3];
        for (int d = 0; d < 3; ++d) g[d] = grid_coord(G, d, c[d][i]);
        cell[i] = ((int64_t)g[2] * G->nc[1] + g[1]) * G->nc[0] + g[0];
        G->start[cell[i] + 1]++;
    }
    for (int64_t k = 0; k < total; ++k) G->start[k + 1] += G->start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)total);
    memcpy(fill, G->start, sizeof(int64_t) * (size_t)total);
    for (int64_t i = 0; i < n; ++i) G->item[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
}

static void grid_free(or_grid *G) { free(G->start); free(G->item); }

/* Visit every particle in the cells overlapping [p - R, p + R] (one spare
 * cell on each side).  Calls fn(j, ctx) for each j; periodic dimensions wrap
 * and never visit a cell twice. */
typedef void (*visit_fn)(int64_t j, void *ctx);

static void grid_visit(const or_grid *G, const double p[3], double R, visit_fn fn, void *ctx)
{
    int cnt[3], first[3];
    for (int d = 0; d < 3; ++d) {
        int a, b;
        if (G->cs[d] > 0.0) {
            a = (int)floor((p[d] - R - G->lo[d]) / G->cs[d]) - 1;
            b = (int)floor((p[d] + R - G->lo[d]) / G->cs[d]) + 1;
        } else { a = 0; b = 0; }
        if (G->per[d]) {
            if (b - a + 1 >= G->nc[d]) { a = 0; b = G->nc[d] - 1; }
        } else {
            if (a < 0) a = 0;
            if (b > G->nc[d] - 1) b = G->nc[d] - 1;
        }
        first[d] = a;
        cnt[d] = b - a + 1;
    }
    for (int kz = 0; kz < cnt[2]; ++kz) {
        int gz = first[2] + kz;
        if (G->per[2]) gz = ((gz % G->nc[2]) + G->nc[2]) % G->nc[2];
        for (int ky = 0; ky < cnt[1]; ++ky) {
            int gy = first[1] + ky;
            if (G->per[1]) gy = ((gy % G->nc[1]) + G->nc[1]) % G->nc[1];
            for (int kx = 0; kx < cnt[0]; ++kx) {
                int gx = first[0] + kx;
                if (G->per[0]) gx = ((gx % G->nc[0]) + G->nc[0]) % G->nc[0];
                int64_t cell = ((int64_t)gz * G->nc[1] + gy) * G->nc[0] + gx;
                for (int64_t k = G->start[cell]; k < G->start[cell + 1]; ++k) fn(G->item[k], ctx);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour counts: N_i(h) = #{ j != i : r_ij^2 < (2h)^2 }                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_geom *g;
    int64_t i;
    double r2max;
    int64_t count;
} count_ctx;

static void count_visit(int64_t j, void *vctx)
{
    count_ctx *c = (count_ctx *)vctx;
    if (j == c->i) return;
    if (pair_r2(c->g, c->i, j, NULL, NULL, NULL) < c->r2max) c->count++;
}

static int64_t count_one(const or_geom *g, const or_grid *G, int64_t n, int64_t i, double h)
{
    double twoh = 2.0 * h;
    count_ctx c = {g, i, twoh * twoh, 0};
    if (G) {
        double p[3] = {g->x[i], g->y[i], g->z[i]};
        grid_visit(G, p, twoh, count_visit, &c);
    } else {
        for (int64_t j = 0; j < n; ++j) count_visit(j, &c);
    }
    return c.count;
}

static double grid_target(int64_t n, const double *x, const double *y, const double *z,
                          const int *periodic, const double *box_lo, const double *box_hi)
{
    double lo[3], hi[3];
    or_bbox(n, x, y, z, periodic, box_lo, box_hi, lo, hi);
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= (hi[d] - lo[d] > 0.0 ? hi[d] - lo[d] : 1.0);
    return cbrt(vol * 32.0 / (double)(n > 0 ? n : 1));
}

/* method: 0 = brute force O(N^2), 1 = uniform grid */
void or_count(int64_t n, const double *x, const double *y, const double *z, const double *h,
              const int *periodic, const double *box_lo, const double *box_hi, int method,
              int32_t *count)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    or_grid G;
    if (method == 1)
        grid_build(&G, n, x, y, z, periodic, box_lo, box_hi,
                   grid_target(n, x, y, z, periodic, box_lo, box_hi));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        count[i] = (int32_t)count_one(&g, method == 1 ? &G : NULL, n, i, h[i]);
    if (method == 1) grid_free(&G);
}

/* ------------------------------------------------------------------------ */
/* Smoothing-length iteration                                                 */
/* ------------------------------------------------------------------------ */
/* Hernquist & Katz (1989) update factor table: T[0] = 2,
 * T[k] = clamp(0.5 (1 + (n_target/k)^(1/3)), 0.5, 2), k = 1..1023. */
void or_hk_table(int n_target, double *T)
{
    T[0] = 2.0;
    for (int k = 1; k < 1024; ++k) {
        double v = 0.5 * (1.0 + cbrt((double)n_target / (double)k));
        if (v < 0.5) v = 0.5;
        if (v > 2.0) v = 2.0;
        T[k] = v;
    }
}

/* Per particle, from h_in:
 *   repeat up to max_iter times:
 *     N = count at h; keep the best (h, N) by |N - target| (ties: smaller h);
 *     stop when |N - target| <= tol;
 *     N below the band raises the lower bracket to h, above it lowers the
 *     upper bracket to h;
 *     with both brackets set h = (lo + hi)/2, else h = h * T[min(N, 1023)].
 *   without convergence the best (h, N) is returned and flag bit 0 is set.
 * Returns the number of particles that did not converge; iters (optional)
 * receives the number of counts taken per particle. */
int64_t or_hsolve(int64_t n, const double *x, const double *y, const double *z,
                  const double *h_in, const int *periodic, const double *box_lo,
                  const double *box_hi, int n_target, int n_tol, int max_iter, int method,
                  double *h_out, int32_t *nc_out, uint8_t *flag_out, int32_t *iters)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    double T[1024];
    or_hk_table(n_target, T);
    or_grid G;
    if (method == 1)
        grid_build(&G, n, x, y, z, periodic, box_lo, box_hi,
                   grid_target(n, x, y, z, periodic, box_lo, box_hi));
    int64_t nonconv = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nonconv)
    for (int64_t i = 0; i < n; ++i) {
        double h = h_in[i];
        double lo = 0.0, hi = 0.0;
        int have_lo = 0, have_hi = 0;
        double best_h = h;
        int64_t best_n = -1;
        int done = 0, k;
        for (k = 0; k < max_iter; ++k) {
            int64_t N = count_one(&g, method == 1 ? &G : NULL, n, i, h);
            int64_t dev = N > n_target ? N - n_target : n_target - N;
            int64_t bdev = best_n > n_target ? best_n - n_target : n_target - best_n;
            if (best_n < 0 || dev < bdev || (dev == bdev && h < best_h)) { best_h = h; best_n = N; }
            if (dev <= n_tol) { done = 1; ++k; break; }
            if (N < n_target - n_tol) {
                if (!have_lo || h > lo) lo = h;
                have_lo = 1;
            } else {
                if (!have_hi || h < hi) hi = h;
                have_hi = 1;
            }
            if (have_lo && have_hi) h = 0.5 * (lo + hi);
            else h = h * T[N < 1023 ? N : 1023];
        }
        if (iters) iters[i] = k;
        h_out[i] = best_h;
        nc_out[i] = (int32_t)best_n;
        flag_out[i] = done ? 0 : 1;
        if (!done) nonconv++;
    }
    if (method == 1) grid_free(&G);
    return nonconv;
}

/* ------------------------------------------------------------------------ */
/* Interaction lists S_i = L_i U { j : i in L_j },  L_i = { j!=i : r^2 < 4h_i^2 } */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_geom *g;
    int64_t i;
    double r2max;
    int64_t *buf;
    int64_t cnt, cap;
} gather_ctx;

static void gather_visit(int64_t j, void *vctx)
{
    gather_ctx *c = (gather_ctx *)vctx;
    if (j == c->i) return;
    if (pair_r2(c->g, c->i, j, NULL, NULL, NULL) < c->r2max) {
        if (c->cnt == c->cap) {
            c->cap = c->cap ? 2 * c->cap : 256;
            c->buf = (int64_t *)realloc(c->buf, sizeof(int64_t) * (size_t)c->cap);
        }
        c->buf[c->cnt++] = j;
    }
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t p = *(const int64_t *)a, q = *(const int64_t *)b;
    return p < q ? -1 : (p > q);
}

/* Builds S (symmetric = 1) or the gather sets L (symmetric = 0), ascending
 * per row. off has n+1 entries; *idx_out is malloc'ed (release with
 * or_free). Returns the total number of entries. */
int64_t or_lists(int64_t n, const double *x, const double *y, const double *z, const double *h,
                 const int *periodic, const double *box_lo, const double *box_hi, int method,
                 int symmetric, int64_t *off, int32_t **idx_out)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    or_grid G;
    if (method == 1)
        grid_build(&G, n, x, y, z, periodic, box_lo, box_hi,
                   grid_target(n, x, y, z, periodic, box_lo, box_hi));
    /* gather sets L_i */
    int64_t **Lrow = (int64_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t *));
    int64_t *Lcnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double twoh = 2.0 * h[i];
        gather_ctx c = {&g, i, twoh * twoh, NULL, 0, 0};
        if (method == 1) {
            double p[3] = {x[i], y[i], z[i]};
            grid_visit(&G, p, twoh, gather_visit, &c);
        } else {
            for (int64_t j = 0; j < n; ++j) gather_visit(j, &c);
        }
        qsort(c.buf, (size_t)c.cnt, sizeof(int64_t), cmp_i64);
        Lrow[i] = c.buf;
        Lcnt[i] = c.cnt;
    }
    if (method == 1) grid_free(&G);
    /* transpose: T_j = { i : j in L_i }, filled with i ascending (empty when
     * only the gather sets are asked for) */
    int64_t *Toff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; symmetric && i < n; ++i)
        for (int64_t k = 0; k < Lcnt[i]; ++k) Toff[Lrow[i][k] + 1]++;
    for (int64_t j = 0; j < n; ++j) Toff[j + 1] += Toff[j];
    int64_t *Tidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Toff[n] > 0 ? Toff[n] : 1));
    int64_t *Tfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) Tfill[j] = Toff[j];
    for (int64_t i = 0; symmetric && i < n; ++i)
        for (int64_t k = 0; k < Lcnt[i]; ++k) Tidx[Tfill[Lrow[i][k]]++] = i;
    free(Tfill);
    /* merge the two ascending rows without duplicates */
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = 0, b = Toff[i], cnt = 0;
        while (a < Lcnt[i] || b < Toff[i + 1]) {
            int64_t va = a < Lcnt[i] ? Lrow[i][a] : INT64_MAX;
            int64_t vb = b < Toff[i + 1] ? Tidx[b] : INT64_MAX;
            if (va < vb) ++a; else if (vb < va) ++b; else { ++a; ++b; }
            ++cnt;
        }
        off[i + 1] = off[i] + cnt;
    }
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = 0, b = Toff[i], w = off[i];
        while (a < Lcnt[i] || b < Toff[i + 1]) {
            int64_t va = a < Lcnt[i] ? Lrow[i][a] : INT64_MAX;
            int64_t vb = b < Toff[i + 1] ? Tidx[b] : INT64_MAX;
            int64_t v;
            if (va < vb) { v = va; ++a; } else if (vb < va) { v = vb; ++b; } else { v = va; ++a; ++b; }
            idx[w++] = (int32_t)v;
        }
    }
    for (int64_t i = 0; i < n; ++i) free(Lrow[i]);
    free(Lrow); free(Lcnt); free(Toff); free(Tidx);
    *idx_out = idx;
    return off[n];
}

void or_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Density and velocity divergence                                            */
/*   rho_i  = m_i W(0,h_i) + sum_{j in L_i} m_j W(r_ij, h_i)                  */
/*   divv_i = (1/rho_i) sum_{j in L_i} m_j (v_j - v_i) . grad_i W(r_ij, h_i)  */
/* entries of S_i outside L_i are skipped (their kernel value is zero).       */
/* Generalized volume elements (X non-NULL; Table 1 lists them for SPHYNX,   */
/* and as in development for the mini-app; read as Hopkins 2013 and          */
/* Cabezon et al. 2017): the weighted sum                                    */
/*   Y_i = X_i W(0,h_i) + sum_{j in L_i} X_j W(r_ij, h_i)                    */
/* gives the volume V_i = X_i / Y_i and the density rho_i = m_i Y_i / X_i    */
/* (X = m is the standard sum); Y_i is returned in ysum when non-NULL.       */
/* ------------------------------------------------------------------------ */
void or_density(int64_t n, const double *x, const double *y, const double *z,
                const double *vx, const double *vy, const double *vz, const double *m,
                const double *h, const int *periodic, const double *box_lo,
                const double *box_hi, const int64_t *off, const int32_t *idx,
                double *rho, double *divv, double *divv_mag, int kernel, double *omega,
                const double *X, double *ysum)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    const double *wgt = X ? X : m;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double hi = h[i];
        double twoh = 2.0 * hi;
        double r2max = twoh * twoh;
        double s = wgt[i] * kern(kernel, 0.0, hi);
        double sh = m[i] * or_kernel_dwdh(kernel, 0.0, hi);   /* sum of m_j dW/dh */
        double dv = 0.0, dvm = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            int64_t j = idx[k];
            double dx, dy, dz;
            double r2 = pair_r2(&g, i, j, &dx, &dy, &dz);
            if (!(r2 < r2max)) continue;
            double r = sqrt(r2);
            s += wgt[j] * kern(kernel, r, hi);
            sh += m[j] * or_kernel_dwdh(kernel, r, hi);
            if (r > 0.0) {
                /* grad_i W = dW/dr (x_i - x_j)/r, and x_i - x_j = -(dx,dy,dz) */
                double gw = kern_dr(kernel, r, hi) / r;
                double vdot = (vx[j] - vx[i]) * (-dx) + (vy[j] - vy[i]) * (-dy) + (vz[j] - vz[i]) * (-dz);
                dv += m[j] * vdot * gw;
                /* condition of the dot product: sum of |component products| */
                double vabs = fabs((vx[j] - vx[i]) * dx) + fabs((vy[j] - vy[i]) * dy) +
                              fabs((vz[j] - vz[i]) * dz);
                dvm += fabs(m[j] * gw) * vabs;
            }
        }
        double rh = X ? m[i] * s / X[i] : s;
        rho[i] = rh;
        if (ysum) ysum[i] = s;
        divv[i] = dv / rh;
        if (divv_mag) divv_mag[i] = dvm / rh;
        /* grad-h factor (Springel & Hernquist 2002) for h proportional to
         * rho^(-1/3): Omega = 1 - (dh/drho) sum_j m_j dW/dh = 1 + h/(3 rho) sum */
        if (omega) omega[i] = 1.0 + hi / (3.0 * rh) * sh;
    }
}

/* Ideal gas: P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u) */
void or_eos(int64_t n, const double *rho, const double *u, double gamma, double *p, double *c)
{
    for (int64_t i = 0; i < n; ++i) {
        p[i] = (gamma - 1.0) * rho[i] * u[i];
        c[i] = sqrt(gamma * (gamma - 1.0) * u[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Momentum, energy, artificial viscosity, Courant time step                 */
/*   x_ij = x_i - x_j, v_ij = v_i - v_j, w = v_ij . x_ij                     */
/*   AV (w < 0): mu = hb w / (r^2 + eta2 hb^2),                              */
/*               Pi = (-alpha cb mu + beta mu^2) / rhob   (else Pi = 0)      */
/*   gradWbar = 1/2 [grad_i W(r,h_i) + grad_i W(r,h_j)]                      */
/*   a_i  = - sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) gradWbar         */
/*   du_i =   sum_j m_j (P_i/rho_i^2 + Pi_ij/2) v_ij . gradWbar              */
/*   dt_i = cfl h_i / (c_i + 1.2 (alpha c_i + beta max_j |mu_ij|))           */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* IAD: integral approach to derivatives (Garcia-Senz, Cabezon & Escartin     */
/* 2012; Table 1 lists it for SPHYNX and, in development, the mini-app).      */
/*   tau_i = sum_{j in L_i} (m_j/rho_j) d d^T W(r_ij, h_i),  d = x_j - x_i,  */
/*   c_i = tau_i^{-1}, stored as (xx, xy, xz, yy, yz, zz).                    */
/* The inverse by Gauss-Jordan elimination with partial pivoting.  Returns   */
/* the number of particles whose tau is singular (their c is set to NaN).    */
/* ------------------------------------------------------------------------ */
static int invert3(double a[3][3], double out[3][3])
{
    double m[3][6];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) { m[r][k] = a[r][k]; m[r][k + 3] = (r == k); }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
        if (!(fabs(m[piv][col]) > 0.0)) return 1;
        if (piv != col)
            for (int k = 0; k < 6; ++k) { double t = m[col][k]; m[col][k] = m[piv][k]; m[piv][k] = t; }
        double inv = 1.0 / m[col][col];
        for (int k = 0; k < 6; ++k) m[col][k] *= inv;
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            double f = m[r][col];
            for (int k = 0; k < 6; ++k) m[r][k] -= f * m[col][k];
        }
    }
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) out[r][k] = m[r][k + 3];
    return 0;
}

int64_t or_iad(int64_t n, const double *x, const double *y, const double *z, const double *m,
               const double *rho, const double *h, const int *periodic, const double *box_lo,
               const double *box_hi, const int64_t *off, const int32_t *idx, int kernel,
               double *c6)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
    for (int64_t i = 0; i < n; ++i) {
        double r2max = 4.0 * h[i] * h[i];
        double t[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            int64_t j = idx[k];
            double d[3];
            double r2 = pair_r2(&g, i, j, &d[0], &d[1], &d[2]);
            if (!(r2 < r2max)) continue;
            double vw = m[j] / rho[j] * kern(kernel, sqrt(r2), h[i]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) t[a][b] += vw * d[a] * d[b];
        }
        double ci[3][3];
        if (invert3(t, ci)) {
            ++bad;
            for (int k = 0; k < 6; ++k) c6[6 * i + k] = NAN;
            continue;
        }
        /* tau is symmetric; its computed inverse is symmetric up to rounding:
         * keep the mean of the two off-diagonal halves */
        c6[6 * i + 0] = ci[0][0];
        c6[6 * i + 1] = 0.5 * (ci[0][1] + ci[1][0]);
        c6[6 * i + 2] = 0.5 * (ci[0][2] + ci[2][0]);
        c6[6 * i + 3] = ci[1][1];
        c6[6 * i + 4] = 0.5 * (ci[1][2] + ci[2][1]);
        c6[6 * i + 5] = ci[2][2];
    }
    return bad;
}

/* c d for the symmetric c stored as (xx, xy, xz, yy, yz, zz) */
static void sym_apply(const double *c, const double d[3], double out[3])
{
    out[0] = c[0] * d[0] + c[1] * d[1] + c[2] * d[2];
    out[1] = c[1] * d[0] + c[3] * d[1] + c[4] * d[2];
    out[2] = c[2] * d[0] + c[4] * d[1] + c[5] * d[2];
}

typedef struct {
    double gamma, alpha, beta, eta2, cfl;
    int kernel;
    const double *omega;   /* grad-h factors, or NULL for the averaged-gradient form */
    const double *iad;     /* IAD matrices c (6 per particle), or NULL for kernel gradients */
    const double *gve_r;   /* generalized volume elements: X_i / m_i, or NULL */
    const double *gve_g;   /* and P_i / Y_i^2 */
} or_phys;

/* the pair term of particle i from neighbour j: writes the acceleration
 * contribution (before the factor m_j is applied: per unit m_j) */
static void pair_force(const or_geom *g, int64_t i, int64_t j, const double *vx,
                       const double *vy, const double *vz, const double *h, const double *rho,
                       const double *p, const double *c, const or_phys *ph,
                       double *fx, double *fy, double *fz, double *de, double *mu_abs,
                       double *de_abs)
{
    double dx, dy, dz;
    double r2 = pair_r2(g, i, j, &dx, &dy, &dz);
    *fx = *fy = *fz = *de = *mu_abs = 0.0;
    if (de_abs) *de_abs = 0.0;
    if (!(r2 > 0.0)) return;
    double r = sqrt(r2);
    double xij = -dx, yij = -dy, zij = -dz;
    double vxij = vx[i] - vx[j], vyij = vy[i] - vy[j], vzij = vz[i] - vz[j];
    double w = vxij * xij + vyij * yij + vzij * zij;
    double gwi = kern_dr(ph->kernel, r, h[i]) / r;
    double gwj = kern_dr(ph->kernel, r, h[j]) / r;
    double gbar = 0.5 * (gwi + gwj);
    double Pi = 0.0;
    if (w < 0.0) {
        double hb = 0.5 * (h[i] + h[j]);
        double cb = 0.5 * (c[i] + c[j]);
        double rb = 0.5 * (rho[i] + rho[j]);
        double mu = hb * w / (r2 + ph->eta2 * hb * hb);
        Pi = (-ph->alpha * cb * mu + ph->beta * mu * mu) / rb;
        *mu_abs = fabs(mu);
    }
    if (ph->iad) {
        /* IAD: grad_i W(h_i) becomes A_i = c_i d W(r, h_i) and grad_i W(h_j)
         * becomes A_j = c_j d W(r, h_j), d = x_j - x_i; pressure terms with
         * their own particle's A, the viscosity with the mean of the two */
        double d[3] = {dx, dy, dz}, Ai[3], Aj[3];
        sym_apply(ph->iad + 6 * i, d, Ai);
        sym_apply(ph->iad + 6 * j, d, Aj);
        double wi = kern(ph->kernel, r, h[i]), wj = kern(ph->kernel, r, h[j]);
        double fi = p[i] / ((ph->omega ? ph->omega[i] : 1.0) * rho[i] * rho[i]);
        double fj = p[j] / ((ph->omega ? ph->omega[j] : 1.0) * rho[j] * rho[j]);
        double G[3], Ab[3];
        for (int a = 0; a < 3; ++a) {
            Ai[a] *= wi;
            Aj[a] *= wj;
            Ab[a] = 0.5 * (Ai[a] + Aj[a]);
            G[a] = (fi * Ai[a] + fj * Aj[a]) + Pi * Ab[a];
        }
        *fx = -G[0];
        *fy = -G[1];
        *fz = -G[2];
        double v[3] = {vxij, vyij, vzij};
        double e1 = 0.0, e2 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            e1 += v[a] * Ai[a];
            e2 += v[a] * Ab[a];
            a1 += fabs(v[a] * Ai[a]);
            a2 += fabs(v[a] * Ab[a]);
        }
        *de = fi * e1 + 0.5 * Pi * e2;
        if (de_abs) *de_abs = fabs(fi) * a1 + fabs(0.5 * Pi) * a2;
        return;
    }
    if (ph->gve_r) {
        /* generalized volume elements: from the Lagrangian with V_i = X_i/Y_i
         * (X held fixed), m_i a_i = -sum_j X_i X_j [P_i/Y_i^2 grad_i W(h_i)
         * + P_j/Y_j^2 grad_i W(h_j)] and du_i = (X_i P_i/(m_i Y_i^2)) sum_j
         * X_j v_ij . grad_i W(h_i); per unit m_j with r = X/m, g = P/Y^2:
         * r_i r_j (g_i grad_i W(h_i) + g_j grad_i W(h_j)); the viscosity
         * keeps the averaged gradient */
        double rr = ph->gve_r[i] * ph->gve_r[j];
        double fi = rr * ph->gve_g[i], fj = rr * ph->gve_g[j];
        double gg = (fi * gwi + fj * gwj) + Pi * gbar;
        *fx = -gg * xij;
        *fy = -gg * yij;
        *fz = -gg * zij;
        double e = fi * gwi + 0.5 * Pi * gbar;
        *de = e * w;
        if (de_abs)
            *de_abs = fabs(e) * (fabs(vxij * xij) + fabs(vyij * yij) + fabs(vzij * zij));
        return;
    }
    if (ph->omega) {
        /* grad-h form: each pressure term with its own particle's gradient
         * and grad-h factor, the viscosity with the averaged gradient */
        double fi = p[i] / (ph->omega[i] * rho[i] * rho[i]);
        double fj = p[j] / (ph->omega[j] * rho[j] * rho[j]);
        double g = (fi * gwi + fj * gwj) + Pi * gbar;
        *fx = -g * xij;
        *fy = -g * yij;
        *fz = -g * zij;
        double e = fi * gwi + 0.5 * Pi * gbar;
        *de = e * w;
        if (de_abs)
            *de_abs = fabs(e) * (fabs(vxij * xij) + fabs(vyij * yij) + fabs(vzij * zij));
        return;
    }
    double pi_term = p[i] / (rho[i] * rho[i]);
    double pj_term = p[j] / (rho[j] * rho[j]);
    double sfac = (pi_term + pj_term) + Pi;
    *fx = -sfac * gbar * xij;
    *fy = -sfac * gbar * yij;
    *fz = -sfac * gbar * zij;
    *de = (pi_term + 0.5 * Pi) * gbar * w;
    /* condition of the energy term: w is a dot product */
    if (de_abs)
        *de_abs = fabs((pi_term + 0.5 * Pi) * gbar) *
                  (fabs(vxij * xij) + fabs(vyij * yij) + fabs(vzij * zij));
}

void or_forces(int64_t n, const double *x, const double *y, const double *z,
               const double *vx, const double *vy, const double *vz, const double *m,
               const double *h, const double *rho, const double *p, const double *c,
               const int *periodic, const double *box_lo, const double *box_hi,
               const int64_t *off, const int32_t *idx, double alpha, double beta, double eta2,
               double cfl, double *ax, double *ay, double *az, double *du, double *dt_i,
               double *amag, double *dumag, int kernel, const double *omega, const double *iad,
               const double *gve_r, const double *gve_g)
{
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    or_phys ph = {0.0, alpha, beta, eta2, cfl, kernel, omega, iad, gve_r, gve_g};
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double sx = 0.0, sy = 0.0, sz = 0.0, se = 0.0, mumax = 0.0, mag = 0.0, emag = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            int64_t j = idx[k];
            double fx, fy, fz, de, mua, dea;
            pair_force(&g, i, j, vx, vy, vz, h, rho, p, c, &ph, &fx, &fy, &fz, &de, &mua, &dea);
            sx += m[j] * fx;
            sy += m[j] * fy;
            sz += m[j] * fz;
            se += m[j] * de;
            if (mua > mumax) mumax = mua;
            mag += m[j] * sqrt(fx * fx + fy * fy + fz * fz);
            emag += m[j] * dea;
        }
        ax[i] = sx; ay[i] = sy; az[i] = sz; du[i] = se;
        if (amag) amag[i] = mag;
        if (dumag) dumag[i] = emag;
        if (dt_i) dt_i[i] = cfl * h[i] / (c[i] + 1.2 * (alpha * c[i] + beta * mumax));
    }
}

/* m_i m_j times the pair acceleration term of i from j (used by the
 * antisymmetry check): written as (m_i m_j) * f */
void or_pair_term(int64_t n, const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz, const double *m,
                  const double *h, const double *rho, const double *p, const double *c,
                  const int *periodic, const double *box_lo, const double *box_hi,
                  int64_t i, int64_t j, double alpha, double beta, double eta2, double *out4,
                  int kernel, const double *omega, const double *iad, const double *gve_r,
                  const double *gve_g)
{
    (void)n;
    or_geom g;
    geom_init(&g, x, y, z, periodic, box_lo, box_hi);
    or_phys ph = {0.0, alpha, beta, eta2, 0.0, kernel, omega, iad, gve_r, gve_g};
    double fx, fy, fz, de, mua;
    pair_force(&g, i, j, vx, vy, vz, h, rho, p, c, &ph, &fx, &fy, &fz, &de, &mua, NULL);
    double mm = m[i] * m[j];
    out4[0] = mm * fx; out4[1] = mm * fy; out4[2] = mm * fz; out4[3] = mua;
}

/* ------------------------------------------------------------------------ */
/* Conservation sums with Neumaier compensated summation                      */
/*   out = [Px, Py, Pz, Lx, Ly, Lz, E],  P = sum m v,  L = sum m x cross v,    */
/*   E = sum m (v.v/2 + u)                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } neu_t;
static void neu_add(neu_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

void or_conservation(int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *m,
                     const double *u, double *out7)
{
    neu_t acc[7];
    memset(acc, 0, sizeof(acc));
    for (int64_t i = 0; i < n; ++i) {
        neu_add(&acc[0], m[i] * vx[i]);
        neu_add(&acc[1], m[i] * vy[i]);
        neu_add(&acc[2], m[i] * vz[i]);
        neu_add(&acc[3], m[i] * (y[i] * vz[i] - z[i] * vy[i]));
        neu_add(&acc[4], m[i] * (z[i] * vx[i] - x[i] * vz[i]));
        neu_add(&acc[5], m[i] * (x[i] * vy[i] - y[i] * vx[i]));
        double ke = 0.5 * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        neu_add(&acc[6], m[i] * (ke + u[i]));
    }
    for (int k = 0; k < 7; ++k) out7[k] = acc[k].s + acc[k].c;
}

/* ------------------------------------------------------------------------ */
/* Kick-drift-kick leapfrog pieces                                            */
/* ------------------------------------------------------------------------ */
/* first half: v += dt/2 a, u += dt/2 du, x += dt v (periodic wrap into [lo,hi)) */
void or_kick_drift(int64_t n, double dt, double *x, double *y, double *z, double *vx,
                   double *vy, double *vz, double *u, const double *ax, const double *ay,
                   const double *az, const double *du, const int *periodic,
                   const double *box_lo, const double *box_hi)
{
    double hdt = 0.5 * dt;
    double *pos[3] = {x, y, z};
    double *vel[3] = {vx, vy, vz};
    const double *acc[3] = {ax, ay, az};
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            vel[d][i] = vel[d][i] + hdt * acc[d][i];
            double q = pos[d][i] + dt * vel[d][i];
            if (periodic[d]) {
                double L = box_hi[d] - box_lo[d];
                if (q >= box_hi[d]) q -= L;
                else if (q < box_lo[d]) q += L;
            }
            pos[d][i] = q;
        }
        u[i] = u[i] + hdt * du[i];
    }
}

/* predicted values for the force evaluation: v* = v_half + dt/2 a, u* likewise */
void or_predict(int64_t n, double dt, const double *vx, const double *vy, const double *vz,
                const double *u, const double *ax, const double *ay, const double *az,
                const double *du, double *pvx, double *pvy, double *pvz, double *pu)
{
    double hdt = 0.5 * dt;
    for (int64_t i = 0; i < n; ++i) {
        pvx[i] = vx[i] + hdt * ax[i];
        pvy[i] = vy[i] + hdt * ay[i];
        pvz[i] = vz[i] + hdt * az[i];
        pu[i] = u[i] + hdt * du[i];
    }
}

/* second half kick: v += dt/2 a_new, u += dt/2 du_new */
void or_kick(int64_t n, double dt, double *vx, double *vy, double *vz, double *u,
             const double *ax, const double *ay, const double *az, const double *du)
{
    double hdt = 0.5 * dt;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] = vx[i] + hdt * ax[i];
        vy[i] = vy[i] + hdt * ay[i];
        vz[i] = vz[i] + hdt * az[i];
        u[i] = u[i] + hdt * du[i];
    }
}

/* Energy by the second-order Adams-Bashforth method with a variable step
 * (the paper names Adams-Bashforth for the energy update next to the
 * Courant step; it prints no formula):
 *   u^{n+1} = u^n + dt_n [(1 + r/2) du^n - (r/2) du^{n-1}],  r = dt_n / dt_{n-1},
 * i.e. du extrapolated linearly to the middle of the step; with no previous
 * step (hist = 0) the Euler step u^{n+1} = u^n + dt_n du^n.                 */
void or_ab2_energy(int64_t n, double dt, double dt_prev, int hist, double *u, const double *du,
                   const double *du_prev)
{
    if (!hist) {
        for (int64_t i = 0; i < n; ++i) u[i] = u[i] + dt * du[i];
        return;
    }
    double r = dt / dt_prev;
    double c1 = 1.0 + 0.5 * r, c0 = 0.5 * r;
    for (int64_t i = 0; i < n; ++i) u[i] = u[i] + dt * (c1 * du[i] - c0 * du_prev[i]);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the later parallel loops (timing the oracle on one core
 * and on all of them); n < 1 is ignored. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Learned smoothing length: MLP 6 -> 64 -> 64 -> 1, tanh hidden layers.      */
/* Weights are row-major [out][in].  Operands entering each layer (inputs,   */
/* hidden activations, weights) are rounded to bfloat16 with round-to-       */
/* nearest-even; biases stay FP32; sums are exact-ish FP64 here.             */
/* ------------------------------------------------------------------------ */
static double bf16_round(double v)
{
    /* round a double directly to the nearest value with 8 significant bits
     * (the bfloat16 significand), ties to even: keep the top 7 stored
     * fraction bits of the 52.  The bfloat16 subnormal range is not
     * modelled (values that small do not occur here). */
    uint64_t b;
    memcpy(&b, &v, 8);
    if ((b & 0x7ff0000000000000ull) == 0x7ff0000000000000ull) return v;  /* inf/nan */
    uint64_t lsb = (b >> 45) & 1ull;
    b += 0x00000FFFFFFFFFFFull + lsb;
    b &= ~0x00001FFFFFFFFFFFull;
    memcpy(&v, &b, 8);
    return v;
}

void or_bf16_round(int64_t n, const double *in, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_round(in[i]);
}

/* forward for a batch: x [B][6] standardised features.
 * z1, a1, z2, a2 (each [B][64], optional) and y [B] are written. */
void or_mlp_forward(int64_t B, const double *x, const double *W1, const double *b1,
                    const double *W2, const double *b2, const double *W3, const double *b3,
                    int use_bf16, double *z1, double *a1, double *z2, double *a2, double *y)
{
#define RB(v) (use_bf16 ? bf16_round(v) : (v))
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < B; ++s) {
        double xin[6], h1[64], h2[64];
        for (int k = 0; k < 6; ++k) xin[k] = RB(x[s * 6 + k]);
        for (int o = 0; o < 64; ++o) {
            double acc = b1[o];
            for (int k = 0; k < 6; ++k) acc += RB(W1[o * 6 + k]) * xin[k];
            if (z1) z1[s * 64 + o] = acc;
            h1[o] = tanh(acc);
            if (a1) a1[s * 64 + o] = h1[o];
            h1[o] = RB(h1[o]);
        }
        for (int o = 0; o < 64; ++o) {
            double acc = b2[o];
            for (int k = 0; k < 64; ++k) acc += RB(W2[o * 64 + k]) * h1[k];
            if (z2) z2[s * 64 + o] = acc;
            h2[o] = tanh(acc);
            if (a2) a2[s * 64 + o] = h2[o];
            h2[o] = RB(h2[o]);
        }
        double acc = b3[0];
        for (int k = 0; k < 64; ++k) acc += RB(W3[k]) * h2[k];
        y[s] = acc;
    }
}

/* Loss L = (1/B) sum (y - t)^2 and its gradient with respect to every
 * parameter, by the chain rule through the forward above (the bf16
 * roundings are treated as identity in the backward, straight-through).
 * Gradients g* have the shapes of the parameters. Returns the loss. */
double or_mlp_loss_grad(int64_t B, const double *x, const double *t, const double *W1,
                        const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3, int use_bf16, double *gW1,
                        double *gb1, double *gW2, double *gb2, double *gW3, double *gb3)
{
    memset(gW1, 0, sizeof(double) * 64 * 6);
    memset(gb1, 0, sizeof(double) * 64);
    memset(gW2, 0, sizeof(double) * 64 * 64);
    memset(gb2, 0, sizeof(double) * 64);
    memset(gW3, 0, sizeof(double) * 64);
    gb3[0] = 0.0;
    double loss = 0.0;
    for (int64_t s = 0; s < B; ++s) {
        double xin[6], a1[64], h1[64], a2[64], h2[64];
        for (int k = 0; k < 6; ++k) xin[k] = RB(x[s * 6 + k]);
        for (int o = 0; o < 64; ++o) {
            double acc = b1[o];
            for (int k = 0; k < 6; ++k) acc += RB(W1[o * 6 + k]) * xin[k];
            a1[o] = tanh(acc);
            h1[o] = RB(a1[o]);
        }
        for (int o = 0; o < 64; ++o) {
            double acc = b2[o];
            for (int k = 0; k < 64; ++k) acc += RB(W2[o * 64 + k]) * h1[k];
            a2[o] = tanh(acc);
            h2[o] = RB(a2[o]);
        }
        double y = b3[0];
        for (int k = 0; k < 64; ++k) y += RB(W3[k]) * h2[k];
        double e = y - t[s];
        loss += e * e;
        double dy = 2.0 * e / (double)B;
        /* layer 3 */
        double d2[64];
        for (int k = 0; k < 64; ++k) {
            gW3[k] += dy * h2[k];
            d2[k] = dy * RB(W3[k]) * (1.0 - a2[k] * a2[k]);
        }
        gb3[0] += dy;
        /* layer 2 */
        double d1[64];
        for (int k = 0; k < 64; ++k) d1[k] = 0.0;
        for (int o = 0; o < 64; ++o) {
            gb2[o] += d2[o];
            for (int k = 0; k < 64; ++k) {
                gW2[o * 64 + k] += d2[o] * h1[k];
                d1[k] += d2[o] * RB(W2[o * 64 + k]);
            }
        }
        for (int k = 0; k < 64; ++k) d1[k] *= (1.0 - a1[k] * a1[k]);
        /* layer 1 */
        for (int o = 0; o < 64; ++o) {
            gb1[o] += d1[o];
            for (int k = 0; k < 6; ++k) gW1[o * 6 + k] += d1[o] * xin[k];
        }
    }
    return loss / (double)B;
}

#undef RB

/* Adam (Kingma & Ba 2015) on one parameter tensor, step t >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) */
void or_adam(int64_t n, double *p, double *m, double *v, const double *g, double lr,
             double beta1, double beta2, double eps, int t)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t k = 0; k < n; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        double mh = m[k] / c1;
        double vh = v[k] / c2;
        p[k] -= lr * mh / (sqrt(vh) + eps);
    }
}
