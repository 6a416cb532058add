// Neighbour search on the Morton cell table: the per-particle smoothing-
// length iteration with the gather set written in the same pass, and the
// one-sided complement E that makes the interaction sets symmetric.
#include "sph_internal.h"

// Search geometry of one launch.  Cells of level l are aligned blocks of
// 2^(10-l) key cells per dimension; the table holds level lmax, a level-l
// cell c spans table entries [c << 3(lmax-l), (c+1) << 3(lmax-l)).
struct Search {
    const int32_t *cs;
    int lmax;
    int div;
    double lo[3], L[3];
    double margin;
    Geo g;
};

__device__ __forceinline__ Search make_search(const int32_t *cs, int lmax, int div,
                                              const double *bbox, Geo g)
{
    Search S;
    S.cs = cs;
    S.lmax = lmax;
    S.div = div;
    double mx = 0.0;
    for (int d = 0; d < 3; ++d) {
        S.lo[d] = bbox[d];
        S.L[d] = bbox[3 + d] - bbox[d];
        mx = fmax(mx, S.L[d]);
    }
    // absolute widening of every search box: far above the rounding of the
    // cell arithmetic, far below a cell
    S.margin = ldexp(mx, -20);
    S.g = g;
    return S;
}

// Calls f(s0, s1) for merged, non-empty ranges of sorted particles covering
// every cell that overlaps the box [p - R, p + R] (widened by the margin).
template <typename F>
__device__ __forceinline__ void visit_ranges(const Search &S, double px, double py, double pz,
                                             double R, F &&f)
{
    double Rs = R + S.margin;
    int l = S.lmax;
    while (l > 0) {
        bool ok = true;
        for (int d = 0; d < 3; ++d)
            if (S.L[d] > 0.0 && ldexp(S.L[d], -l) * S.div < Rs) ok = false;
        if (ok) break;
        --l;
    }
    const int nl = 1 << l;
    int a[3], cnt[3];
    const double p[3] = {px, py, pz};
    for (int d = 0; d < 3; ++d) {
        if (!(S.L[d] > 0.0)) { a[d] = 0; cnt[d] = 1; continue; }
        double w = ldexp(S.L[d], -l);
        double ta = floor((p[d] - Rs - S.lo[d]) / w);
        double tb = floor((p[d] + Rs - S.lo[d]) / w);
        ta = fmin(fmax(ta, -2.0 * nl), 3.0 * nl);
        tb = fmin(fmax(tb, -2.0 * nl), 3.0 * nl);
        int ia = (int)ta, ib = (int)tb;
        if (S.g.per[d]) {
            if (ib - ia + 1 >= nl) { ia = 0; ib = nl - 1; }
        } else {
            ia = max(ia, 0);
            ib = min(ib, nl - 1);
        }
        a[d] = ia;
        cnt[d] = ib - ia + 1;
    }
    const int sh = 3 * (S.lmax - l);
    int rs = 0, re = 0;
    // cell coordinates are reduced modulo nl (only periodic dimensions can
    // leave [0, nl); the others were clamped above)
    const int m = nl - 1;  // nl is a power of two
    for (int kz = 0; kz < cnt[2]; ++kz) {
        int cz = (a[2] + kz) & m;
        for (int ky = 0; ky < cnt[1]; ++ky) {
            int cy = (a[1] + ky) & m;
            for (int kx = 0; kx < cnt[0]; ++kx) {
                int cx = (a[0] + kx) & m;
                uint32_t code = morton((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
                int s0 = S.cs[(int64_t)code << sh];
                int s1 = S.cs[((int64_t)code + 1) << sh];
                if (s0 == s1) continue;
                if (s0 == re) {
                    re = s1;
                } else {
                    if (re > rs) f(rs, re);
                    rs = s0;
                    re = s1;
                }
            }
        }
    }
    if (re > rs) f(rs, re);
}

// Count of L_i(h) = { j != i : r^2 < (2h)^2 }, writing up to K entries of
// the set into idx (slot-major).
__device__ __forceinline__ int count_fill(const Search &S, const double *__restrict__ x,
                                          const double *__restrict__ y,
                                          const double *__restrict__ z, int64_t i, double xi,
                                          double yi, double zi, double h,
                                          int32_t *__restrict__ idx, int64_t stride, int K,
                                          bool write, int64_t &tested)
{
#pragma clang fp contract(off)
    double twoh = 2.0 * h;
    double r2max = twoh * twoh;
    int cnt = 0;
    const Geo &g = S.g;
    visit_ranges(S, xi, yi, zi, twoh, [&](int s0, int s1) {
        tested += s1 - s0;
        for (int j = s0; j < s1; ++j) {
            double dx = min_image(xi, x[j], g.per[0], g.L[0], g.halfL[0]);
            double dy = min_image(yi, y[j], g.per[1], g.L[1], g.halfL[1]);
            double dz = min_image(zi, z[j], g.per[2], g.L[2], g.halfL[2]);
            double r2 = exact_r2(dx, dy, dz);
            if (r2 < r2max && j != (int)i) {
                if (write && cnt < K) idx[(int64_t)cnt * stride + i] = j;
                ++cnt;
            }
        }
    });
    return cnt;
}

// Smoothing-length iteration, one thread per particle:
//   N = count at h; keep the best (h, N) by |N - target| (ties: smaller h);
//   stop when |N - target| <= tol; below the band raise the lower bracket,
//   above it lower the upper bracket; bisect once both are set, else
//   h *= T[min(N, 1023)].  The gather set of the last counted h is written.
// With h_try (learned mode) the first count is taken at h_try[i]; if it is
// in the band it is accepted, otherwise the iteration restarts from h[i].
__global__ __launch_bounds__(SPH_BLOCK) void k_hsolve(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, double *__restrict__ h, int32_t *__restrict__ nc,
    uint8_t *__restrict__ flags, uint8_t *__restrict__ refill, int32_t *__restrict__ idx,
    int64_t stride, int K, const int32_t *__restrict__ cs, const double *__restrict__ bbox,
    Geo g, int lmax, int div, const double *__restrict__ hk, int target, int tol, int maxit,
    const double *__restrict__ h_try, int64_t *__restrict__ status)
{
#pragma clang fp contract(off)
    int64_t i = global_index();
    bool valid = i < n;
    int64_t counts = 0, nonconv = 0, overflow = 0, acc = 0, fallback = 0, tested = 0;
    if (valid) {
        Search S = make_search(cs, lmax, div, bbox, g);
        double xi = x[i], yi = y[i], zi = z[i];
        double hcur = h[i];
        bool done = false;
        double best_h = hcur, last_h = hcur;
        int best_n = -1;
        uint8_t fl = 0;
        if (h_try) {
            double ht = h_try[i];
            int N = count_fill(S, x, y, z, i, xi, yi, zi, ht, idx, stride, K, true, tested);
            ++counts;
            int dev = N > target ? N - target : target - N;
            if (dev <= tol) {
                done = true;
                best_h = ht;
                last_h = ht;
                best_n = N;
                fl = SPH_FLAG_LEARNED;
                ++acc;
            } else {
                ++fallback;
            }
        }
        if (!done) {
            double lo = 0.0, hi = 0.0;
            bool have_lo = false, have_hi = false;
            for (int k = 0; k < maxit; ++k) {
                int N = count_fill(S, x, y, z, i, xi, yi, zi, hcur, idx, stride, K, true, tested);
                ++counts;
                last_h = hcur;
                int dev = N > target ? N - target : target - N;
                int bdev = best_n > target ? best_n - target : target - best_n;
                if (best_n < 0 || dev < bdev || (dev == bdev && hcur < best_h)) {
                    best_h = hcur;
                    best_n = N;
                }
                if (dev <= tol) { done = true; break; }
                if (N < target - tol) {
                    if (!have_lo || hcur > lo) lo = hcur;
                    have_lo = true;
                } else {
                    if (!have_hi || hcur < hi) hi = hcur;
                    have_hi = true;
                }
                if (have_lo && have_hi) hcur = 0.5 * (lo + hi);
                else hcur = hcur * hk[N < 1023 ? N : 1023];
            }
        }
        if (!done) { fl |= SPH_FLAG_NOCONV; ++nonconv; }
        h[i] = best_h;
        nc[i] = best_n;
        flags[i] = fl;
        bool again = best_h != last_h;
        refill[i] = again ? 1 : 0;
        if (!again && best_n > K) ++overflow;
    }
    block_add_i64(counts, status + ST_HCOUNTS);
    block_add_i64(tested, status + ST_CANDIDATES);
    block_add_i64(nonconv, status + ST_NONCONV);
    block_add_i64(overflow, status + ST_LIST_OVERFLOW);
    if (h_try) {
        block_add_i64(acc, status + ST_LEARN_ACC);
        block_add_i64(fallback, status + ST_LEARN_FALLBACK);
    }
}

// rewrite the gather set of particles whose kept h is not the last counted one
__global__ __launch_bounds__(SPH_BLOCK) void k_refill(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ h, const int32_t *__restrict__ nc,
    const uint8_t *__restrict__ refill, int32_t *__restrict__ idx, int64_t stride, int K,
    const int32_t *__restrict__ cs, const double *__restrict__ bbox, Geo g, int lmax, int div,
    int64_t *__restrict__ status)
{
    int64_t i = global_index();
    int64_t overflow = 0, tested = 0;
    if (i < n && refill[i]) {
        Search S = make_search(cs, lmax, div, bbox, g);
        int N = count_fill(S, x, y, z, i, x[i], y[i], z[i], h[i], idx, stride, K, true, tested);
        if (N > K) ++overflow;
        (void)nc;
    }
    block_add_i64(overflow, status + ST_LIST_OVERFLOW);
}

hipError_t launch_hsolve(sph_ctx *c, sph_particles *s, sph_nlist *nl, const double *h_try)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    const sph_params &p = c->p;
    int cur = s->cur;
    unsigned nb = (unsigned)ceil_div(n, SPH_BLOCK);
    Geo g = make_geo(p);
    hipLaunchKernelGGL(k_hsolve, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur], s->y[cur],
                       s->z[cur], s->h[cur], s->nc[cur], s->flags, c->w.refill, nl->idx,
                       nl->stride, p.list_stride, c->w.cell_start, c->w.bbox, g, p.max_level,
                       p.search_div, c->w.hk, p.n_target, p.n_tol, p.h_max_iter, h_try,
                       c->w.status);
    hipLaunchKernelGGL(k_refill, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur], s->y[cur],
                       s->z[cur], s->h[cur], s->nc[cur], c->w.refill, nl->idx, nl->stride,
                       p.list_stride, c->w.cell_start, c->w.bbox, g, p.max_level, p.search_div,
                       c->w.status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// complement E: j in L_i with i not in L_j  =>  i belongs to E_j
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_zero_i32(int32_t *__restrict__ a, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

template <bool FILL>
__global__ __launch_bounds__(SPH_BLOCK) void k_extra(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ h, const int32_t *__restrict__ nc,
    const int32_t *__restrict__ idx, int64_t stride, int K, Geo g, int32_t *__restrict__ cnt,
    const int64_t *__restrict__ eoff, int32_t *__restrict__ eidx, int64_t ecap)
{
#pragma clang fp contract(off)
    int64_t i = global_index();
    if (i >= n) return;
    double xi = x[i], yi = y[i], zi = z[i];
    int m = min(nc[i], K);
    for (int k = 0; k < m; ++k) {
        int j = idx[(int64_t)k * stride + i];
        double dx = min_image(xi, x[j], g.per[0], g.L[0], g.halfL[0]);
        double dy = min_image(yi, y[j], g.per[1], g.L[1], g.halfL[1]);
        double dz = min_image(zi, z[j], g.per[2], g.L[2], g.halfL[2]);
        double r2 = exact_r2(dx, dy, dz);
        double twoh = 2.0 * h[j];
        if (!(r2 < twoh * twoh)) {
            int pos = atomicAdd(&cnt[j], 1);
            if (FILL) {
                int64_t at = eoff[j] + pos;
                if (at < ecap && at < eoff[j + 1]) eidx[at] = (int32_t)i;
            }
        }
    }
}

// ascending order inside each row of E (fills came in arbitrary order)
__global__ __launch_bounds__(SPH_BLOCK) void k_extra_sort(int64_t n, const int64_t *__restrict__ eoff,
                                                          int32_t *__restrict__ eidx, int64_t ecap,
                                                          int64_t *__restrict__ status)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j == 0 && eoff[n] > ecap) status[ST_EXTRA_OVERFLOW] = 1;
    if (j >= n) return;
    int64_t a = eoff[j], b = eoff[j + 1];
    if (b > ecap) b = ecap;
    for (int64_t p = a + 1; p < b; ++p) {
        int32_t v = eidx[p];
        int64_t q = p - 1;
        while (q >= a && eidx[q] > v) {
            eidx[q + 1] = eidx[q];
            --q;
        }
        eidx[q + 1] = v;
    }
}

hipError_t launch_extra(sph_ctx *c, sph_particles *s, sph_nlist *nl)
{
    int64_t n = s->n;
    const sph_params &p = c->p;
    int cur = s->cur;
    unsigned nb = (unsigned)ceil_div(n > 0 ? n : 1, SPH_BLOCK);
    Geo g = make_geo(p);
    hipLaunchKernelGGL(k_zero_i32, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, c->w.ecnt, n);
    hipLaunchKernelGGL(k_zero_i32, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, c->w.efill, n);
    if (n > 0)
        hipLaunchKernelGGL((k_extra<false>), dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur],
                           s->y[cur], s->z[cur], s->h[cur], s->nc[cur], nl->idx, nl->stride,
                           p.list_stride, g, c->w.ecnt, (const int64_t *)nullptr,
                           (int32_t *)nullptr, (int64_t)0);
    hipError_t e = launch_scan_i32_to_i64(c, c->w.ecnt, nl->eoff, n);
    if (e != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL((k_extra<true>), dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur],
                           s->y[cur], s->z[cur], s->h[cur], s->nc[cur], nl->idx, nl->stride,
                           p.list_stride, g, c->w.efill, nl->eoff, nl->eidx, nl->ecap);
        hipLaunchKernelGGL(k_extra_sort, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, nl->eoff,
                           nl->eidx, nl->ecap, c->w.status);
    }
    return hipGetLastError();
}
