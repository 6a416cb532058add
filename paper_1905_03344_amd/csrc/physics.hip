// Density and divergence, equation of state, momentum / energy / viscosity
// with the Courant step, kick-drift-kick integrator and conservation sums.
#include <mutex>

#include "sph_internal.h"

// rho_i = m_i W(0,h_i) + sum_{L_i} m_j W(r_ij,h_i);
// divv_i = (1/rho_i) sum_{L_i} m_j (v_j - v_i) . grad_i W(r_ij,h_i).
// With EXTRA the same pass appends i to E_j for every one-sided pair.
// Pair loops run with SPH_GROUP lanes per particle: the gather set of a
// particle lies in ascending index order (neighbouring cells in Morton
// order), so the lanes of a group load short runs of consecutive particles
// and each load touches a few cache lines instead of one per lane.  Each
// lane sums its share of the pairs (k = lane, lane + SPH_GROUP, ...) and the
// group adds the partial sums in a fixed butterfly order, so results are
// reproducible.  Block b treats the T = SPH_PTILE_D (density) or
// SPH_PTILE_F (forces) particles [T b, T (b+1)): in round r its
// G = SPH_BLOCK / SPH_GROUP groups take particles T b + G r + group.
// Eight lanes per particle (eight particles per
// wave) measured best of 4, 8, 16, 32 and 64: a wave load then spans the
// short row segments of eight consecutive particles, whose neighbours
// overlap, and rows of ~100 entries keep the lanes busy.
#ifndef SPH_GROUP
#define SPH_GROUP 8
#endif
// pairs per lane per batch of the density pass: 3 keeps it at 113 VGPRs (4
// waves/SIMD; 4 pairs take 131, 3 waves): 64M density 37.7 -> 36.0 ms, 8M
// 4.97 -> 4.72 (2 pairs: 37.3 ms at 5 waves)
#ifndef SPH_BATCH
#define SPH_BATCH 3
#endif
#ifndef SPH_FBATCH
#define SPH_FBATCH 2
#endif
// rounds per block of the density (D) and force (F) kernels: a block takes
// SPH_PTILE_* = SPH_PROUNDS_* * SPH_BLOCK / SPH_GROUP consecutive particles.
// Measured (8M / 64M patch, ms per launch): forces 8 rounds 6.02 / 47.2,
// 4 rounds 5.77 / 45.2, 2 rounds 5.69 / 44.5 (a narrower window of
// particles in flight per XCD); density 8 rounds 4.86 / 37.1, 4 rounds
// 4.90 / 37.6, 2 rounds 5.07 / 39.1.  Non-temporal row loads (keeping the
// rows out of L2) made the forces slower (47.2 -> 51.4 ms), and so did a
// direct-mapped LDS cache of neighbour records in the density kernel
// (37 -> 53 ms with 512 slots, 71 with 1024: its fill phases serialise on
// load latency at two blocks per CU).
#ifndef SPH_PROUNDS_D
#define SPH_PROUNDS_D 8
#endif
#ifndef SPH_PROUNDS_F
#define SPH_PROUNDS_F 2
#endif
#define SPH_PTILE_D (SPH_PROUNDS_D * (SPH_BLOCK / SPH_GROUP))
#define SPH_PTILE_F (SPH_PROUNDS_F * (SPH_BLOCK / SPH_GROUP))

__device__ __forceinline__ double group_sum(double v)
{
    for (int o = SPH_GROUP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SPH_GROUP);
    return v;
}
__device__ __forceinline__ double group_max(double v)
{
    for (int o = SPH_GROUP / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, SPH_GROUP));
    return v;
}

static Pk64 ctx_pk64(sph_ctx *c)
{
    const int64_t n = c->p.n_max;
    double2 *b = (double2 *)c->w.pk64;
    return Pk64{b, b + n, b + 2 * n, b + 3 * n, b + 4 * n};
}

__global__ __launch_bounds__(SPH_BLOCK) void k_pack64(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ h, const double *__restrict__ vx,
    const double *__restrict__ vy, const double *__restrict__ vz, const double *__restrict__ m,
    Pk64 P)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    P.xy[i] = make_double2(x[i], y[i]);
    P.zh[i] = make_double2(z[i], h[i]);
    P.vxy[i] = make_double2(vx[i], vy[i]);
    P.vzm[i] = make_double2(vz[i], m[i]);
}

// GH: also the grad-h factor Omega_i = 1 - (1/(3 rho_i)) sum_j m_j (3 W + r dW/dr).
// GV: generalized volume elements, Y_i = X_i W(0,h_i) + sum_{L_i} X_j W(r_ij,h_i)
// (stored in ysum) and rho_i = m_i Y_i / X_i; the divergence keeps m_j.
template <int PM, bool EXTRA, int KER, bool GH, bool GV>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_D void k_density(
    int64_t n, Pk64 P, const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K, Geo g,
    double knorm,
    double *__restrict__ rho, double *__restrict__ divv, double *__restrict__ omega,
    int32_t *__restrict__ ecnt,
    int32_t *__restrict__ eidx, int slots, int64_t *__restrict__ status,
    const double *__restrict__ X, double *__restrict__ ysum)
{
    const int lane = threadIdx.x & (SPH_GROUP - 1);
    const int grp = threadIdx.x / SPH_GROUP;
    const int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SPH_PTILE_D;
    int64_t appended = 0, dropped = 0;
    for (int r = 0; r < SPH_PROUNDS_D; ++r) {   // SPH_BLOCK / SPH_GROUP groups per round
        const int64_t i = base + (int64_t)r * (SPH_BLOCK / SPH_GROUP) + grp;
        double s = 0.0, dv = 0.0, t = 0.0, inv_h = 0.0, mi = 0.0;
        if (i < n) {
            const double2 pxy = P.xy[i], pzh = P.zh[i], pv = P.vxy[i], pvm = P.vzm[i];
            const double xi = pxy.x, yi = pxy.y, zi = pzh.x;
            const double vxi = pv.x, vyi = pv.y, vzi = pvm.x;
            mi = pvm.y;
            inv_h = 1.0 / pzh.y;
            const int cnt = min(nc[i], K);
            const int32_t *row = idx + i * (int64_t)K;
            // batches of SPH_BATCH pairs per lane: indices first, then every
            // gather of the batch, then the arithmetic (slots past the end
            // point at particle i itself and are skipped)
            for (int k0 = lane; k0 < cnt; k0 += SPH_BATCH * SPH_GROUP) {
                int jb[SPH_BATCH];
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    const int k = k0 + q * SPH_GROUP;
                    jb[q] = k < cnt ? row[k] : (int)i;
                }
                double xb[SPH_BATCH], yb[SPH_BATCH], zb[SPH_BATCH], hb[SPH_BATCH], mb[SPH_BATCH];
                double ub[SPH_BATCH], vb[SPH_BATCH], wb[SPH_BATCH], qb[SPH_BATCH];
                int ek[SPH_BATCH];   // complement slot taken for pair q (-1: none)
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    const int j = jb[q];
                    const double2 a = P.xy[j], b = P.zh[j], cv = P.vxy[j], d = P.vzm[j];
                    xb[q] = a.x; yb[q] = a.y; zb[q] = b.x; hb[q] = b.y;
                    ub[q] = cv.x; vb[q] = cv.y; wb[q] = d.x; mb[q] = d.y;
                    qb[q] = GV ? X[j] : 0.0;
                    ek[q] = -1;
                }
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    if (k0 + q * SPH_GROUP >= cnt) break;
                    const int j = jb[q];
                    double dx = mimg<PM, 0>(xi, xb[q], g);
                    double dy = mimg<PM, 1>(yi, yb[q], g);
                    double dz = mimg<PM, 2>(zi, zb[q], g);
                    double r2 = exact_r2(dx, dy, dz);
                    if (EXTRA) {
#pragma clang fp contract(off)
                        double twoh = 2.0 * hb[q];
                        if (!(r2 < twoh * twoh)) ek[q] = extra_take(j, ecnt);
                    }
                    const double rinv = r2 > 0.0 ? rsqrt_nr(r2) : 0.0;
                    double rr = r2 * rinv;
                    double mj = mb[q];
                    const double wk = kern_w<KER>(rr, inv_h, knorm);
                    s += (GV ? qb[q] : mj) * wk;
                    if (rr > 0.0) {
                        const double dw = kern_dwdr<KER>(rr, inv_h, knorm);
                        double gw = dw * rinv;
                        double vdot = (ub[q] - vxi) * (-dx) + (vb[q] - vyi) * (-dy) + (wb[q] - vzi) * (-dz);
                        dv += mj * vdot * gw;
                        if (GH) t += mj * (3.0 * wk + rr * dw);
                    } else if (GH) {
                        t += mj * 3.0 * wk;
                    }
                }
                if (EXTRA) {
#pragma unroll
                    for (int q = 0; q < SPH_BATCH; ++q)
                        if (ek[q] >= 0) extra_put(jb[q], ek[q], (int)i, eidx, slots, appended, dropped);
                }
            }
        }
        s = group_sum(s);
        dv = group_sum(dv);
        if (GH) t = group_sum(t);
        if (i < n && lane == 0) {
            const double w0 = kern_w<KER>(0.0, inv_h, knorm);
            double rh;
            if (GV) {
                const double xi_w = X[i];
                const double yv = xi_w * w0 + s;
                rh = mi * yv / xi_w;
                ysum[i] = yv;
            } else {
                rh = mi * w0 + s;
            }
            rho[i] = rh;
            divv[i] = dv / rh;
            if (GH) omega[i] = 1.0 - (3.0 * mi * w0 + t) / (3.0 * rh);
        }
    }
    if (EXTRA) {
        block_add_i64(appended, status + ST_EXTRA_TOTAL);
        block_add_i64(dropped, status + ST_EXTRA_OVERFLOW);
    }
}

// E rows in ascending order (their slots were taken by atomics), one thread
// per row, for row capacities above SPH_ELDS (the force kernels rank shorter
// rows themselves): rows of up to 16 entries through a sorting network in
// registers, longer ones by insertion sort in place
#define SPH_ESORT 16
__device__ __forceinline__ void cmp_swap(int &a, int &b)
{
    const int lo = min(a, b), hi = max(a, b);
    a = lo;
    b = hi;
}

__global__ __launch_bounds__(SPH_BLOCK) void k_sort_extra(int64_t n, const int32_t *__restrict__ ecnt,
                                                          int32_t *__restrict__ eidx, int slots)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ne = min(ecnt[i], slots);
    if (ne < 2) return;
    int32_t *row = eidx + i * (int64_t)slots;
    if (ne <= SPH_ESORT && (((uintptr_t)row) & 15) == 0) {
        int v[SPH_ESORT];
        // 16-byte loads of the row's first ceil(ne/4) quads
#pragma unroll
        for (int q = 0; q < SPH_ESORT / 4; ++q) {
            int4 w = make_int4(0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff);
            if (4 * q < ne) w = reinterpret_cast<const int4 *>(row)[q];
            v[4 * q] = 4 * q < ne ? w.x : 0x7fffffff;
            v[4 * q + 1] = 4 * q + 1 < ne ? w.y : 0x7fffffff;
            v[4 * q + 2] = 4 * q + 2 < ne ? w.z : 0x7fffffff;
            v[4 * q + 3] = 4 * q + 3 < ne ? w.w : 0x7fffffff;
        }
        // bitonic sorting network on 16 values
#pragma unroll
        for (int sz = 2; sz <= SPH_ESORT; sz <<= 1)
#pragma unroll
            for (int st = sz >> 1; st > 0; st >>= 1)
#pragma unroll
                for (int k = 0; k < SPH_ESORT; ++k) {
                    const int l = k ^ st;
                    if (l > k) {
                        if ((k & sz) == 0) cmp_swap(v[k], v[l]);
                        else cmp_swap(v[l], v[k]);
                    }
                }
#pragma unroll
        for (int q = 0; q < SPH_ESORT / 4; ++q) {
            if (4 * q + 3 < ne) {
                reinterpret_cast<int4 *>(row)[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2],
                                                             v[4 * q + 3]);
            } else {
#pragma unroll
                for (int k = 4 * q; k < 4 * q + 4; ++k)
                    if (k < ne) row[k] = v[k];
            }
        }
        return;
    }
    for (int a = 1; a < ne; ++a) {
        const int x = row[a];
        int b = a - 1;
        while (b >= 0 && row[b] > x) {
            row[b + 1] = row[b];
            --b;
        }
        row[b + 1] = x;
    }
}

hipError_t launch_sort_extra(sph_ctx *c, const sph_nlist *nl, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_extra, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, nl->ecnt, nl->eidx, c->p.extra_slots);
    return hipGetLastError();
}

// generalized volume elements: X_i = (m_i / rho_i)^p from the density held
__global__ __launch_bounds__(SPH_BLOCK) void k_gve_weights(int64_t n, const double *__restrict__ m,
                                                           const double *__restrict__ rho,
                                                           double p, double *__restrict__ X)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) X[i] = pow(m[i] / rho[i], p);
}

hipError_t launch_density(sph_ctx *c, sph_particles *s, const sph_nlist *nl, bool build_extra)
{
    int64_t n = s->n;
    if (build_extra) {
        hipError_t e = launch_zero_i32(c, nl->ecnt, n);
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    int cur = s->cur;
    Geo g = make_geo(c->p);
    unsigned nb = (unsigned)ceil_div(n, SPH_BLOCK);
    const unsigned nbt = (unsigned)ceil_div(n, SPH_PTILE_D);
    const Pk64 P = ctx_pk64(c);
    hipLaunchKernelGGL(k_pack64, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur], s->y[cur],
                       s->z[cur], s->h[cur], s->pvx, s->pvy, s->pvz, s->m[cur], P);
#define SPH_DENSITY_ARGS                                                                        \
    dim3(nbt), dim3(SPH_BLOCK), 0, c->stream, n, P, s->nc[cur], nl->idx, c->p.list_stride, g,     \
        c->knorm, s->rho[cur], s->divv[cur], c->w.omega, nl->ecnt, nl->eidx, c->p.extra_slots,  \
        c->w.status, c->w.gve_x, c->w.gve_y
#define SPH_DENSITY(EX, GHV, GVV)                                                               \
    SPH_DISPATCH_KER(c->p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                             \
        hipLaunchKernelGGL((k_density<PM, EX, KER, GHV, GVV>), SPH_DENSITY_ARGS)))
    if (c->p.volumes == SPH_VOLUMES_GENERALIZED) {
        // the weights come from the density of the previous evaluation; an
        // evaluation that starts a run forms the standard density first
        bool extra = build_extra;
        if (c->gve_fresh) {
            if (extra) { SPH_DENSITY(true, false, false) }
            else { SPH_DENSITY(false, false, false) }
            extra = false;
        }
        hipLaunchKernelGGL(k_gve_weights, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->m[cur],
                           s->rho[cur], c->p.gve_exponent, c->w.gve_x);
        if (extra) { SPH_DENSITY(true, false, true) }
        else { SPH_DENSITY(false, false, true) }
    } else if (c->p.grad_h) {
        if (build_extra) { SPH_DENSITY(true, true, false) }
        else { SPH_DENSITY(false, true, false) }
    } else if (build_extra) {
        SPH_DENSITY(true, false, false)
    } else {
        SPH_DENSITY(false, false, false)
    }
#undef SPH_DENSITY
#undef SPH_DENSITY_ARGS
    return hipGetLastError();
}

// ideal gas; the neighbour record carries P / (Omega rho^2) (Omega = 1
// without grad-h terms, omega NULL), or with generalized volume elements
// (X non-NULL) q = (X/m) P / Y^2
__global__ __launch_bounds__(SPH_BLOCK) void k_eos(int64_t n, const double *__restrict__ rho,
                                                   const double *__restrict__ u, double gamma,
                                                   const double *__restrict__ omega,
                                                   double *__restrict__ p, double *__restrict__ c,
                                                   double2 *__restrict__ rp, int check,
                                                   int64_t *__restrict__ status,
                                                   const double *__restrict__ X,
                                                   const double *__restrict__ m,
                                                   const double *__restrict__ ysum)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t bad = 0;
    if (i < n) {
        const double rh = rho[i];
        double pv = (gamma - 1.0) * rh * u[i];
        double cv = sqrt(gamma * (gamma - 1.0) * u[i]);
        p[i] = pv;
        c[i] = cv;
        if (X) {
            const double yv = ysum[i];
            rp[i] = make_double2(rh, X[i] / m[i] * pv / (yv * yv));
        } else {
            const double den = omega ? omega[i] * (rh * rh) : rh * rh;
            rp[i] = make_double2(rh, pv / den);   // P / (Omega rho^2) once per particle
        }
        if (check && !(isfinite(pv) && isfinite(cv) && isfinite(rho[i]))) bad = 1;
    }
    if (check) block_add_i64(bad, status + ST_NONFINITE);
}

hipError_t launch_eos(sph_ctx *c, sph_particles *s)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eos, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, s->rho[s->cur], s->pu, c->p.gamma,
                       c->p.grad_h ? c->w.omega : nullptr, s->p, s->c, ctx_pk64(c).rp,
                       c->p.check_finite, c->w.status, c->w.gve_x, s->m[s->cur], c->w.gve_y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// momentum, energy, artificial viscosity, Courant step
// ---------------------------------------------------------------------------
// gradient forms of the pair sums (template argument GR)
#define SPH_GR_AVG 0   // averaged kernel gradient
#define SPH_GR_OWN 1   // each pressure term with its own kernel gradient (grad-h)
#define SPH_GR_IAD 2   // each pressure term with its own IAD gradient
#define SPH_GR_GVE 3   // generalized volume elements: r_i r_j (g_i grad W(h_i) + g_j grad W(h_j))

struct ForceAcc {
    double ax, ay, az, du, mumax;
};

// neighbour fields of one pair, gathered ahead of the arithmetic
struct NbrF {
    double x, y, z, vx, vy, vz, m, h, rho, p, c;   // p holds P / (Omega rho^2), or q = r g
    double xw;                                     // generalized volumes: X_j
    double cm[6];                                  // IAD: c_j (xx, xy, xz, yy, yz, zz)
};

// the three IAD arrays of n_max double2 each
struct IadC {
    double2 *a, *b, *c;   // (xx, xy), (xz, yy), (yz, zz)
};

static IadC ctx_iad(sph_ctx *c)
{
    double2 *b = c->w.iad;
    const int64_t n = c->p.n_max;
    return IadC{b, b ? b + n : nullptr, b ? b + 2 * n : nullptr};
}

// IAD moment matrix over the gather set and its inverse, one group of
// SPH_GROUP lanes per particle (as the density kernel): tau accumulates
// (m_j/rho_j) W(r_ij,h_i) d d^T, d = x_j - x_i; c = adj(tau)/det(tau)
template <int PM, int KER>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_D void k_iad(
    int64_t n, Pk64 P, const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K,
    Geo g, double knorm, IadC out, int64_t *__restrict__ status)
{
    const int lane = threadIdx.x & (SPH_GROUP - 1);
    const int grp = threadIdx.x / SPH_GROUP;
    const int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SPH_BLOCK;
    int64_t bad = 0;
    for (int r = 0; r < SPH_GROUP; ++r) {
        const int64_t i = base + (int64_t)r * (SPH_BLOCK / SPH_GROUP) + grp;
        double txx = 0.0, txy = 0.0, txz = 0.0, tyy = 0.0, tyz = 0.0, tzz = 0.0;
        if (i < n) {
            const double2 pxy = P.xy[i], pzh = P.zh[i];
            const double xi = pxy.x, yi = pxy.y, zi = pzh.x;
            const double inv_h = 1.0 / pzh.y;
            const int cnt = min(nc[i], K);
            const int32_t *row = idx + i * (int64_t)K;
            for (int k0 = lane; k0 < cnt; k0 += SPH_BATCH * SPH_GROUP) {
                int jb[SPH_BATCH];
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    const int k = k0 + q * SPH_GROUP;
                    jb[q] = k < cnt ? row[k] : (int)i;
                }
                double2 ab[SPH_BATCH], zb[SPH_BATCH], mb[SPH_BATCH], rb[SPH_BATCH];
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    const int j = jb[q];
                    ab[q] = P.xy[j]; zb[q] = P.zh[j]; mb[q] = P.vzm[j]; rb[q] = P.rp[j];
                }
#pragma unroll
                for (int q = 0; q < SPH_BATCH; ++q) {
                    if (k0 + q * SPH_GROUP >= cnt) break;
                    const double dx = mimg<PM, 0>(xi, ab[q].x, g);
                    const double dy = mimg<PM, 1>(yi, ab[q].y, g);
                    const double dz = mimg<PM, 2>(zi, zb[q].x, g);
                    const double r2 = exact_r2(dx, dy, dz);
                    const double rr = r2 > 0.0 ? r2 * rsqrt_nr(r2) : 0.0;
                    const double vw = mb[q].y / rb[q].x * kern_w<KER>(rr, inv_h, knorm);
                    txx += vw * dx * dx; txy += vw * dx * dy; txz += vw * dx * dz;
                    tyy += vw * dy * dy; tyz += vw * dy * dz; tzz += vw * dz * dz;
                }
            }
        }
        txx = group_sum(txx); txy = group_sum(txy); txz = group_sum(txz);
        tyy = group_sum(tyy); tyz = group_sum(tyz); tzz = group_sum(tzz);
        if (i < n && lane == 0) {
            const double axx = tyy * tzz - tyz * tyz;
            const double axy = txz * tyz - txy * tzz;
            const double axz = txy * tyz - txz * tyy;
            const double det = txx * axx + txy * axy + txz * axz;
            if (!(det > 0.0) || !isfinite(det)) ++bad;
            const double id = 1.0 / det;
            const double ayy = txx * tzz - txz * txz;
            const double ayz = txy * txz - txx * tyz;
            const double azz = txx * tyy - txy * txy;
            out.a[i] = make_double2(axx * id, axy * id);
            out.b[i] = make_double2(axz * id, ayy * id);
            out.c[i] = make_double2(ayz * id, azz * id);
        }
    }
    block_add_i64(bad, status + ST_IAD_SINGULAR);
}

hipError_t launch_iad(sph_ctx *c, sph_particles *s, const sph_nlist *nl)
{
    const int64_t n = s->n;
    if (n == 0) return hipSuccess;
    Geo g = make_geo(c->p);
    const IadC I = ctx_iad(c);
    SPH_DISPATCH_KER(c->p.kernel, SPH_DISPATCH_PM(periodic_mask(g),
        hipLaunchKernelGGL((k_iad<PM, KER>), dim3((unsigned)ceil_div(n, SPH_BLOCK)),
                           dim3(SPH_BLOCK), 0, c->stream, n, ctx_pk64(c), s->nc[s->cur], nl->idx,
                           c->p.list_stride, g, c->knorm, I, c->w.status)))
    return hipGetLastError();
}

template <int GR>
__device__ __forceinline__ NbrF load_nbr(int j, const Pk64 &P, const double *__restrict__ c,
                                         const IadC &I, const double *__restrict__ Xw)
{
    NbrF b;
    const double2 a = P.xy[j], zh = P.zh[j], v = P.vxy[j], vm = P.vzm[j], rp = P.rp[j];
    b.x = a.x; b.y = a.y; b.z = zh.x; b.h = zh.y;
    b.vx = v.x; b.vy = v.y; b.vz = vm.x; b.m = vm.y;
    // the plain form's sound speed follows from the record (ideal gas:
    // c^2 = gamma P / rho = gamma (P / rho^2) rho), one gather fewer per pair
    b.rho = rp.x; b.p = rp.y; b.c = GR == SPH_GR_AVG ? 0.0 : c[j];
    b.xw = GR == SPH_GR_GVE ? Xw[j] : 0.0;
    if (GR == SPH_GR_IAD) {
        const double2 p0 = I.a[j], p1 = I.b[j], p2 = I.c[j];
        b.cm[0] = p0.x; b.cm[1] = p0.y; b.cm[2] = p1.x;
        b.cm[3] = p1.y; b.cm[4] = p2.x; b.cm[5] = p2.y;
    }
    return b;
}

// GR: SPH_GR_AVG everything with the averaged kernel gradient; SPH_GR_OWN
// pressure terms with each particle's own kernel gradient (grad-h form), the
// viscosity with the average; SPH_GR_IAD pressure terms with each particle's
// own IAD gradient A = c d W, the viscosity with their mean (ci: c_i);
// SPH_GR_GVE the generalized-volume pressure terms (pi_term = q_i = r_i g_i,
// b.p = q_j, ri = X_i / m_i, b.xw = X_j), the viscosity with the average
template <int PM, int KER, int GR>
__device__ __forceinline__ void force_pair(const NbrF &b, double xi, double yi, double zi,
                                           double vxi, double vyi, double vzi, double hi,
                                           double inv_hi, double rhoi, double ci, double pi_term,
                                           const double *cmi, double ri, const Geo &g,
                                           double knorm, double alpha, double beta, double eta2,
                                           double gamma, ForceAcc &A)
{
    double dx = mimg<PM, 0>(xi, b.x, g);
    double dy = mimg<PM, 1>(yi, b.y, g);
    double dz = mimg<PM, 2>(zi, b.z, g);
    double r2 = dx * dx + dy * dy + dz * dz;
    // a pair at r = 0 adds zero to every sum (1/r taken as 0 zeroes the
    // kernel gradients, the offset zeroes the IAD ones); no early exit, so
    // that the compiler issues all of a batch's gathers before its arithmetic
    const double inv_r = r2 > 0.0 ? rsqrt_nr(r2) : 0.0;
    const double r = r2 * inv_r;
    double hj = b.h;
    double xij = -dx, yij = -dy, zij = -dz;
    double vxij = vxi - b.vx, vyij = vyi - b.vy, vzij = vzi - b.vz;
    double w = vxij * xij + vyij * yij + vzij * zij;
    if (GR == SPH_GR_IAD) {
        double Pi = 0.0;
        if (w < 0.0) {
            double hb = 0.5 * (hi + b.h);
            double cb = 0.5 * (ci + b.c);
            double rb = 0.5 * (rhoi + b.rho);
            // mu = hb w / den and Pi = (..) / rb from one reciprocal of den rb
            const double den = r2 + eta2 * hb * hb;
            const double rq = rcp_nr(den * rb);
            const double mu = hb * w * (rb * rq);
            Pi = (-alpha * cb * mu + beta * mu * mu) * (den * rq);
            A.mumax = fmax(A.mumax, fabs(mu));
        }
        const double wi = kern_w<KER>(r, inv_hi, knorm);
        const double wj = kern_w<KER>(r, rcp_nr(b.h), knorm);
        // A = c d W with d = x_j - x_i = (dx, dy, dz)
        const double aix = (cmi[0] * dx + cmi[1] * dy + cmi[2] * dz) * wi;
        const double aiy = (cmi[1] * dx + cmi[3] * dy + cmi[4] * dz) * wi;
        const double aiz = (cmi[2] * dx + cmi[4] * dy + cmi[5] * dz) * wi;
        const double ajx = (b.cm[0] * dx + b.cm[1] * dy + b.cm[2] * dz) * wj;
        const double ajy = (b.cm[1] * dx + b.cm[3] * dy + b.cm[4] * dz) * wj;
        const double ajz = (b.cm[2] * dx + b.cm[4] * dy + b.cm[5] * dz) * wj;
        const double abx = 0.5 * (aix + ajx), aby = 0.5 * (aiy + ajy), abz = 0.5 * (aiz + ajz);
        const double mj = b.m, pj_term = b.p;
        A.ax -= mj * ((pi_term * aix + pj_term * ajx) + Pi * abx);
        A.ay -= mj * ((pi_term * aiy + pj_term * ajy) + Pi * aby);
        A.az -= mj * ((pi_term * aiz + pj_term * ajz) + Pi * abz);
        A.du += mj * (pi_term * (vxij * aix + vyij * aiy + vzij * aiz) +
                      0.5 * Pi * (vxij * abx + vyij * aby + vzij * abz));
        return;
    }
    double gwi = kern_dwdr<KER>(r, inv_hi, knorm) * inv_r;
    double gwj = kern_dwdr<KER>(r, rcp_nr(hj), knorm) * inv_r;
    double gbar = 0.5 * (gwi + gwj);
    double rhoj = b.rho;
    double Pi = 0.0;
    if (w < 0.0) {
        double hb = 0.5 * (hi + hj);
        double cj = b.c;
        if (GR == SPH_GR_AVG) {
            const double c2 = gamma * b.p * rhoj;
            cj = c2 > 0.0 ? c2 * rsqrt_nr(c2) : 0.0;
        }
        double cb = 0.5 * (ci + cj);
        double rb = 0.5 * (rhoi + rhoj);
        const double den = r2 + eta2 * hb * hb;
        const double rq = rcp_nr(den * rb);
        const double mu = hb * w * (rb * rq);
        Pi = (-alpha * cb * mu + beta * mu * mu) * (den * rq);
        A.mumax = fmax(A.mumax, fabs(mu));
    }
    double pj_term = b.p;
    double mj = b.m;
    if (GR == SPH_GR_GVE) {
        // m_j r_i r_j g_i = X_j q_i and m_j r_i r_j g_j = r_i m_j q_j
        const double ti = b.xw * pi_term * gwi;
        double f = (ti + ri * mj * pj_term * gwj) + mj * Pi * gbar;
        A.ax -= f * xij;
        A.ay -= f * yij;
        A.az -= f * zij;
        A.du += (ti + 0.5 * mj * Pi * gbar) * w;
        return;
    }
    if (GR == SPH_GR_OWN) {
        double f = mj * ((pi_term * gwi + pj_term * gwj) + Pi * gbar);
        A.ax -= f * xij;
        A.ay -= f * yij;
        A.az -= f * zij;
        A.du += mj * (pi_term * gwi + 0.5 * Pi * gbar) * w;
        return;
    }
    double sfac = (pi_term + pj_term) + Pi;
    double f = mj * sfac * gbar;
    A.ax -= f * xij;
    A.ay -= f * yij;
    A.az -= f * zij;
    A.du += mj * (pi_term + 0.5 * Pi) * gbar * w;
}

// S_i = L_i (row order) then E_i (ascending) in groups of SPH_GROUP lanes;
// ELDS: E rows ranked in LDS here (capacity <= SPH_ELDS), else sorted already
template <int PM, bool ELDS, int KER, int GR>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_F void k_forces(
    int64_t n, Pk64 P, IadC I, const double *__restrict__ Xw, const double *__restrict__ c,
    const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K,
    const int32_t *__restrict__ ecnt, const int32_t *__restrict__ eidx, int slots, Geo g,
    double knorm, double alpha, double beta, double eta2, double gamma, double cfl,
    double *__restrict__ ax,
    double *__restrict__ ay, double *__restrict__ az, double *__restrict__ du,
    double *__restrict__ dt_part)
{
    const int lane = threadIdx.x & (SPH_GROUP - 1);
    const int grp = threadIdx.x / SPH_GROUP;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = blk * SPH_PTILE_F;
    __shared__ int32_t e_raw[ELDS ? SPH_BLOCK / SPH_GROUP : 1][ELDS ? SPH_ELDS : 1];
    __shared__ int32_t e_srt[ELDS ? SPH_BLOCK / SPH_GROUP : 1][ELDS ? SPH_ELDS : 1];
    double dti = INFINITY;
    for (int r = 0; r < SPH_PROUNDS_F; ++r) {   // SPH_BLOCK / SPH_GROUP groups per round
        const int64_t i = base + (int64_t)r * (SPH_BLOCK / SPH_GROUP) + grp;
        ForceAcc A = {0.0, 0.0, 0.0, 0.0, 0.0};
        double hi = 0.0, ci = 0.0;
        if (i < n) {
            const NbrF me = load_nbr<GR>((int)i, P, c, I, Xw);
            const double xi = me.x, yi = me.y, zi = me.z;
            const double vxi = me.vx, vyi = me.vy, vzi = me.vz;
            hi = me.h;
            const double inv_hi = 1.0 / hi, rhoi = me.rho;
            ci = c[i];
            const double pi_term = me.p;
            const double ri = GR == SPH_GR_GVE ? me.xw / me.m : 0.0;
            const int cnt = min(nc[i], K);
            const int ne = min(ecnt[i], slots);
            const int32_t *lrow = idx + i * (int64_t)K;
            const int32_t *erow = eidx + i * (int64_t)slots;
            if (ELDS && ne > 0) erow_sort_lds<SPH_GROUP>(erow, ne, lane, e_raw[grp], e_srt[grp]);
            const int tot = cnt + ne;
            for (int k0 = lane; k0 < tot; k0 += SPH_FBATCH * SPH_GROUP) {
                int jb[SPH_FBATCH];
#pragma unroll
                for (int q = 0; q < SPH_FBATCH; ++q) {
                    const int k = k0 + q * SPH_GROUP;
                    jb[q] = k < cnt ? lrow[k]
                                    : (k < tot ? (ELDS ? e_srt[grp][k - cnt] : erow[k - cnt]) : (int)i);
                }
                NbrF nb[SPH_FBATCH];
#pragma unroll
                for (int q = 0; q < SPH_FBATCH; ++q)
                    nb[q] = load_nbr<GR>(jb[q], P, c, I, Xw);
#pragma unroll
                for (int q = 0; q < SPH_FBATCH; ++q) {
                    if (k0 + q * SPH_GROUP >= tot) break;
                    force_pair<PM, KER, GR>(nb[q], xi, yi, zi, vxi, vyi, vzi, hi, inv_hi, rhoi, ci,
                                            pi_term, me.cm, ri, g, knorm, alpha, beta, eta2,
                                            gamma, A);
                }
            }
        }
        A.ax = group_sum(A.ax);
        A.ay = group_sum(A.ay);
        A.az = group_sum(A.az);
        A.du = group_sum(A.du);
        A.mumax = group_max(A.mumax);
        if (i < n && lane == 0) {
            ax[i] = A.ax;
            ay[i] = A.ay;
            az[i] = A.az;
            du[i] = A.du;
            dti = fmin(dti, cfl * hi / (ci + 1.2 * (alpha * ci + beta * A.mumax)));
        }
    }
    // block minimum of dt_i (min is exact and order independent)
    __shared__ double sh[SPH_BLOCK];
    sh[threadIdx.x] = dti;
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dt_part[blk] = sh[0];
}

__global__ __launch_bounds__(SPH_BLOCK) void k_min_final(const double *__restrict__ part, int64_t nb,
                                                         double *__restrict__ out)
{
    __shared__ double sh[SPH_BLOCK];
    double v = INFINITY;
    for (int64_t k = threadIdx.x; k < nb; k += SPH_BLOCK) v = fmin(v, part[k]);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_forces(sph_ctx *c, sph_particles *s, const sph_nlist *nl, double *d_dt)
{
    int64_t n = s->n;
    int cur = s->cur;
    const sph_params &p = c->p;
    int64_t nb = ceil_div(n > 0 ? n : 1, SPH_PTILE_F);
    // dt partials live in the reduction area (sized for n_max / 32 blocks)
    double *part = c->w.red_part;
    c->dt_parts = nb;
    Geo g = make_geo(p);
#define SPH_FORCE_ARGS                                                                          \
    dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, n, ctx_pk64(c), I, c->w.gve_x, s->c,      \
        s->nc[cur],                                                                             \
        nl->idx, p.list_stride, nl->ecnt, nl->eidx, p.extra_slots, g, c->knorm, p.av_alpha,     \
        p.av_beta, p.av_eta2, p.gamma, p.cfl, s->ax[cur], s->ay[cur], s->az[cur], s->du[cur],   \
        part
    if (p.extra_slots > SPH_ELDS) {
        hipError_t e = launch_sort_extra(c, nl, n);
        if (e != hipSuccess) return e;
    }
    const IadC I = ctx_iad(c);
    const bool elds = p.extra_slots <= SPH_ELDS;
#define SPH_FORCE_GR(GRV)                                                                       \
    if (elds) {                                                                                 \
        SPH_DISPATCH_KER(p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                            \
            hipLaunchKernelGGL((k_forces<PM, true, KER, GRV>), SPH_FORCE_ARGS)))                \
    } else {                                                                                    \
        SPH_DISPATCH_KER(p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                            \
            hipLaunchKernelGGL((k_forces<PM, false, KER, GRV>), SPH_FORCE_ARGS)))               \
    }
    if (p.gradients == SPH_GRADIENTS_IAD) {
        hipError_t e = launch_iad(c, s, nl);
        if (e != hipSuccess) return e;
        SPH_FORCE_GR(SPH_GR_IAD)
    } else if (p.grad_h) {
        SPH_FORCE_GR(SPH_GR_OWN)
    } else if (p.volumes == SPH_VOLUMES_GENERALIZED) {
        SPH_FORCE_GR(SPH_GR_GVE)
    } else {
        SPH_FORCE_GR(SPH_GR_AVG)
    }
#undef SPH_FORCE_GR
#undef SPH_FORCE_ARGS
    return hipGetLastError();
}

// minimum over slices of the dt partials, one per block (min is exact, so
// the two stages give the value of one)
#define SPH_DT_SLICES 256
__global__ __launch_bounds__(SPH_BLOCK) void k_min_slices(const double *__restrict__ part, int64_t nb,
                                                          double *__restrict__ out)
{
    const int64_t per = (nb + SPH_DT_SLICES - 1) / SPH_DT_SLICES;
    const int64_t lo = blockIdx.x * per, hi = min(nb, lo + per);
    __shared__ double sh[SPH_BLOCK];
    double v = INFINITY;
    for (int64_t k = lo + threadIdx.x; k < hi; k += SPH_BLOCK) v = fmin(v, part[k]);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

hipError_t launch_dt_min(sph_ctx *c, int64_t n, double *d_dt)
{
    (void)n;
    if (!d_dt) return hipSuccess;
    const int64_t nb = c->dt_parts;
    if (nb > 4 * SPH_DT_SLICES) {
        // the slice minima go behind the partials (the area holds n_max / 32
        // partials, at least 16384, and at most n_max / 64 are written)
        double *slices = c->w.red_part + nb;
        hipLaunchKernelGGL(k_min_slices, dim3(SPH_DT_SLICES), dim3(SPH_BLOCK), 0, c->stream,
                           c->w.red_part, nb, slices);
        hipLaunchKernelGGL(k_min_final, dim3(1), dim3(SPH_BLOCK), 0, c->stream, slices,
                           (int64_t)SPH_DT_SLICES, d_dt);
    } else {
        hipLaunchKernelGGL(k_min_final, dim3(1), dim3(SPH_BLOCK), 0, c->stream, c->w.red_part,
                           nb, d_dt);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// kick-drift-kick pieces; dt read from the device scalar of the step
// ---------------------------------------------------------------------------
__global__ void k_set_dt(double dt, const double *__restrict__ src, double *__restrict__ dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = (dt > 0.0) ? dt : *src;
}

hipError_t launch_set_dt(sph_ctx *c, double dt, const double *d_dt)
{
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, c->stream, dt, d_dt, c->w.dt_cur);
    return hipGetLastError();
}

// ab2: 0 = KDK half kick of u; 1 = Euler u + dt du; 2 = Adams-Bashforth
// u + dt [(1 + r/2) du - (r/2) du_prev], r = dt / dt_prev.  With ab2 > 0 the
// kernel also moves du into du_prev (the previous step's du is read first).
__global__ __launch_bounds__(SPH_BLOCK) void k_kick_drift(
    int64_t n, const double *__restrict__ dtp, double *__restrict__ x, double *__restrict__ y,
    double *__restrict__ z, double *__restrict__ vx, double *__restrict__ vy,
    double *__restrict__ vz, double *__restrict__ u, const double *__restrict__ ax,
    const double *__restrict__ ay, const double *__restrict__ az, const double *__restrict__ du,
    Geo g, double lo0, double lo1, double lo2, double hi0, double hi1, double hi2, int ab2,
    double *__restrict__ du_prev, const double *__restrict__ dt_prev)
{
#pragma clang fp contract(off)
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dt = *dtp;
    double hdt = 0.5 * dt;
    double *pos[3] = {x, y, z};
    double *vel[3] = {vx, vy, vz};
    const double *acc[3] = {ax, ay, az};
    const double blo[3] = {lo0, lo1, lo2}, bhi[3] = {hi0, hi1, hi2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double v = vel[d][i] + hdt * acc[d][i];
        vel[d][i] = v;
        double q = pos[d][i] + dt * v;
        if (g.per[d]) {
            if (q >= bhi[d]) q -= g.L[d];
            else if (q < blo[d]) q += g.L[d];
        }
        pos[d][i] = q;
    }
    if (ab2 == 0) {
        u[i] = u[i] + hdt * du[i];
    } else {
        const double dun = du[i];
        if (ab2 == 1) {
            u[i] = u[i] + dt * dun;
        } else {
            const double r = dt / *dt_prev;
            const double c1 = 1.0 + 0.5 * r, c0 = 0.5 * r;
            u[i] = u[i] + dt * (c1 * dun - c0 * du_prev[i]);
        }
        du_prev[i] = dun;
    }
}

hipError_t launch_kick_drift(sph_ctx *c, sph_particles *s)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    const sph_params &p = c->p;
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, c->w.dt_cur, s->x[k], s->y[k], s->z[k], s->vx[k], s->vy[k],
                       s->vz[k], s->u[k], s->ax[k], s->ay[k], s->az[k], s->du[k], make_geo(p),
                       p.box_lo[0], p.box_lo[1], p.box_lo[2], p.box_hi[0], p.box_hi[1],
                       p.box_hi[2], p.integrator == SPH_INTEGRATOR_AB2 ? (c->ab2_hist ? 2 : 1) : 0,
                       c->w.du_prev[k], c->w.dt_prev);
    return hipGetLastError();
}

// pv = v + dt/2 a, pu = u + dt/2 du   (mode 0)
// pv = v, pu = u                      (mode 1: evaluation at the stored state)
// pv = v + dt/2 a, pu = u             (mode 2: Adams-Bashforth energy, final)
__global__ __launch_bounds__(SPH_BLOCK) void k_predict(
    int64_t n, const double *__restrict__ dtp, int mode, const double *__restrict__ vx,
    const double *__restrict__ vy, const double *__restrict__ vz, const double *__restrict__ u,
    const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ az,
    const double *__restrict__ du, double *__restrict__ pvx, double *__restrict__ pvy,
    double *__restrict__ pvz, double *__restrict__ pu)
{
#pragma clang fp contract(off)
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == 1) {
        pvx[i] = vx[i]; pvy[i] = vy[i]; pvz[i] = vz[i]; pu[i] = u[i];
        return;
    }
    double hdt = 0.5 * (*dtp);
    pvx[i] = vx[i] + hdt * ax[i];
    pvy[i] = vy[i] + hdt * ay[i];
    pvz[i] = vz[i] + hdt * az[i];
    pu[i] = mode == 2 ? u[i] : u[i] + hdt * du[i];
}

static hipError_t predict(sph_ctx *c, sph_particles *s, int mode)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, c->w.dt_cur, mode, s->vx[k], s->vy[k], s->vz[k], s->u[k],
                       s->ax[k], s->ay[k], s->az[k], s->du[k], s->pvx, s->pvy, s->pvz, s->pu);
    return hipGetLastError();
}

hipError_t launch_predict(sph_ctx *c, sph_particles *s)
{
    return predict(c, s, c->p.integrator == SPH_INTEGRATOR_AB2 ? 2 : 0);
}
hipError_t launch_copy_pred(sph_ctx *c, sph_particles *s) { return predict(c, s, 1); }

// second half kick; with ab2 the energy is already final, and the step's dt
// is kept for the next Adams-Bashforth step
__global__ __launch_bounds__(SPH_BLOCK) void k_kick(int64_t n, const double *__restrict__ dtp,
                                                    double *__restrict__ vx,
                                                    double *__restrict__ vy,
                                                    double *__restrict__ vz,
                                                    double *__restrict__ u,
                                                    const double *__restrict__ ax,
                                                    const double *__restrict__ ay,
                                                    const double *__restrict__ az,
                                                    const double *__restrict__ du, int ab2,
                                                    double *__restrict__ dt_prev)
{
#pragma clang fp contract(off)
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (ab2 && i == 0) *dt_prev = *dtp;
    if (i >= n) return;
    double hdt = 0.5 * (*dtp);
    vx[i] = vx[i] + hdt * ax[i];
    vy[i] = vy[i] + hdt * ay[i];
    vz[i] = vz[i] + hdt * az[i];
    if (!ab2) u[i] = u[i] + hdt * du[i];
}

hipError_t launch_kick(sph_ctx *c, sph_particles *s)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    hipLaunchKernelGGL(k_kick, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, c->w.dt_cur, s->vx[k], s->vy[k], s->vz[k], s->u[k], s->ax[k],
                       s->ay[k], s->az[k], s->du[k], c->p.integrator == SPH_INTEGRATOR_AB2 ? 1 : 0,
                       c->w.dt_prev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// conservation sums: per-block tree sums, then one block over the partials
// in index order; the same inputs give the same bits every run
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_cons_partial(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ vz, const double *__restrict__ m, const double *__restrict__ u,
    double *__restrict__ part)
{
    __shared__ double sh[7][SPH_BLOCK];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double mi = m[i];
        a[0] += mi * vx[i];
        a[1] += mi * vy[i];
        a[2] += mi * vz[i];
        a[3] += mi * (y[i] * vz[i] - z[i] * vy[i]);
        a[4] += mi * (z[i] * vx[i] - x[i] * vz[i]);
        a[5] += mi * (x[i] * vy[i] - y[i] * vx[i]);
        a[6] += mi * (0.5 * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) + u[i]);
    }
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 7) part[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(SPH_BLOCK) void k_cons_final(const double *__restrict__ part,
                                                          int64_t nb, double *__restrict__ out)
{
    __shared__ double sh[7][SPH_BLOCK];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nb; b += SPH_BLOCK)
        for (int k = 0; k < 7; ++k) a[k] += part[b * 8 + k];
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 7) out[threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_conservation(sph_ctx *c, const sph_particles *s, double *out7)
{
    int64_t n = s->n;
    int k = s->cur;
    int64_t nb = 1024;
    if (nb > c->w.nb_red) nb = c->w.nb_red;
    if (n < nb * SPH_BLOCK) nb = ceil_div(n > 0 ? n : 1, SPH_BLOCK);
    hipLaunchKernelGGL(k_cons_partial, dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, n,
                       s->x[k], s->y[k], s->z[k], s->vx[k], s->vy[k], s->vz[k], s->m[k], s->u[k],
                       c->w.red_part);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(SPH_BLOCK), 0, c->stream, c->w.red_part, nb,
                       out7);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free conservation sums.  The block partials live in `scratch`,
// a file-scope device array (each GPU the library runs on holds its own copy
// until the process ends) instead of the bound workspace; the same kernels
// and the same block count as sph_conservation, so the same bits.  Host code
// must not pass `scratch` itself to a kernel (in host code the name stands
// for a host-side symbol): its device address is looked up once per device
// with hipGetSymbolAddress and kept in g_scratch_dev.
// ---------------------------------------------------------------------------
#define SPH_CONS_MAX_BLOCKS 1024
#define SPH_NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) double scratch[SPH_CONS_MAX_BLOCKS * 8];

static std::mutex g_scratch_mu;
static double *g_scratch_dev[SPH_NOALLOC_MAX_DEVICES];

// device address of this GPU's scratch (the current device's), looked up on
// the first call on that device
static hipError_t scratch_on_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SPH_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

extern "C" int sph_conservation_noalloc(const sph_particles *s, double *d_out7, void *stream)
{
    if (!s || !d_out7) return SPH_EINVAL;
    if (s->n < 0 || (s->cur != 0 && s->cur != 1)) return SPH_EINVAL;
    const int k = s->cur;
    const int64_t n = s->n;
    if (n > 0) {
        const void *f[] = {s->x[k], s->y[k], s->z[k], s->vx[k], s->vy[k], s->vz[k], s->m[k],
                           s->u[k]};
        for (const void *q : f)
            if (!q) return SPH_EINVAL;
    }
    double *part = nullptr;
    if (scratch_on_current_device(&part) != hipSuccess) return SPH_EHIP;
    // at most SPH_CONS_MAX_BLOCKS blocks stride over any n, so the partials
    // always fit; the block count is sph_conservation's
    int64_t nb = ceil_div(n > 0 ? n : 1, SPH_BLOCK);
    if (nb > SPH_CONS_MAX_BLOCKS) nb = SPH_CONS_MAX_BLOCKS;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_cons_partial, dim3((unsigned)nb), dim3(SPH_BLOCK), 0, st, n, s->x[k],
                       s->y[k], s->z[k], s->vx[k], s->vy[k], s->vz[k], s->m[k], s->u[k], part);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(SPH_BLOCK), 0, st, part, nb, d_out7);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}
