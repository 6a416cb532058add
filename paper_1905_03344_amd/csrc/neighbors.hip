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
    // cell coordinates are reduced modulo nl (only periodic dimensions can
    // leave [0, nl); the others were clamped above).  Every lane calls f once
    // per cell, empty or not, so lanes of a wave stay in step.
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
                f(s0, s1);
            }
        }
    }
}

// Count of L_i(h) = { j != i : r^2 < (2h)^2 }, writing up to K entries of
// the set into idx (slot-major).
template <int PM>
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
            double dx = mimg<PM, 0>(xi, x[j], g);
            double dy = mimg<PM, 1>(yi, y[j], g);
            double dz = mimg<PM, 2>(zi, z[j], g);
            double r2 = exact_r2(dx, dy, dz);
            if (r2 < r2max && j != (int)i) {
                if (write && cnt < K) idx[(int64_t)cnt * stride + i] = j;
                ++cnt;
            }
        }
    });
    return cnt;
}

// ---------------------------------------------------------------------------
// Smoothing-length iteration, wave-cooperative.
// A wave owns 64 consecutive (Morton-sorted) particles.  Per count it builds
// the union of its members' search boxes, walks the cells of that box in
// batches of 64 (one cell per lane, prefix sums of the cell sizes), streams
// the candidates in tiles of 64 through LDS and lets every lane test every
// candidate of the tile against its own particle (broadcast LDS reads), so
// control flow is uniform across the wave and candidate loads are coalesced.
// Per particle the arithmetic is the iteration of the paper's reading:
//   N = count at h; keep the best (h, N) by |N - target| (ties: smaller h);
//   stop when |N - target| <= tol; below the band raise the lower bracket,
//   above it lower the upper bracket; bisect once both are set, else
//   h *= T[min(N, 1023)]; at most maxit counts.
// The gather set of the last counted h is written (slot-major).
// With h_try (learned mode) the first count is taken at h_try[i]; in band it
// is accepted, otherwise the plain iteration starts from h[i].
// ---------------------------------------------------------------------------
struct Cand {
    double x, y, z;
    int j;
    int pad;
};

__device__ __forceinline__ double wave_min_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_min_u(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_incl_scan_i(int v)
{
    int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}
// orders this wave's LDS writes before its later LDS reads (LDS is in order
// within a wave; this keeps the compiler from moving accesses across)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define WAVES_PER_BLOCK (SPH_BLOCK / 64)

template <int PM>
__global__ __launch_bounds__(SPH_BLOCK) void k_hsolve(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const uint32_t *__restrict__ key, double *__restrict__ h,
    int32_t *__restrict__ nc, uint8_t *__restrict__ flags, uint8_t *__restrict__ refill,
    int32_t *__restrict__ idx, int64_t stride, int K, const int32_t *__restrict__ cs,
    const double *__restrict__ bbox, Geo g, int lmax, int div, const double *__restrict__ hk,
    int target, int tol, int maxit, const double *__restrict__ h_try,
    int64_t *__restrict__ status)
{
#pragma clang fp contract(off)
    __shared__ Cand s_c[WAVES_PER_BLOCK][64];
    __shared__ int s_start[WAVES_PER_BLOCK][64];
    __shared__ int s_pre[WAVES_PER_BLOCK][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t grp = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + w;
    const int64_t i = grp * 64 + lane;
    const bool valid = i < n;
    const Search S = make_search(cs, lmax, div, bbox, g);

    double xi = 0.0, yi = 0.0, zi = 0.0, hcur = 0.0, hnext = 0.0;
    uint32_t ki = 0;
    if (valid) {
        xi = x[i]; yi = y[i]; zi = z[i];
        hcur = h[i];
        ki = key[i];
    }
    bool tried = (h_try == nullptr);
    hnext = (!tried && valid) ? h_try[i] : hcur;   // h of the next count
    bool stop = !valid, conv = false;
    double lo_b = 0.0, hi_b = 0.0, best_h = hcur, last_h = hcur;
    bool have_lo = false, have_hi = false;
    int best_n = -1, itk = 0;
    uint8_t fl = 0;
    int64_t counts = 0, tested = 0, acc = 0, fallback = 0;

    uint64_t pending = __ballot(valid);
    while (pending) {
        // sub-group: the pending lanes, split by Morton prefix while their
        // positions spread over more than 1.5 search diameters (a group that
        // straddles a large Morton jump would otherwise scan the gap)
        uint64_t members = pending;
        for (int sp = 0; sp < 32; ++sp) {
            bool mem = (members >> lane) & 1ull;
            double Rm = wave_max_d(mem ? 2.0 * hnext : 0.0);
            double ext = 0.0;
            const double p3[3] = {xi, yi, zi};
            for (int d = 0; d < 3; ++d) {
                double a = wave_min_d(mem ? p3[d] : INFINITY);
                double b = wave_max_d(mem ? p3[d] : -INFINITY);
                ext = fmax(ext, b - a);
            }
            if (!(ext > 3.0 * Rm) || __popcll(members) == 1) break;
            uint32_t kmin = wave_min_u(mem ? ki : 0xFFFFFFFFu);
            uint32_t kmax = wave_max_u(mem ? ki : 0u);
            if (kmin == kmax) break;
            int hb = 31 - __clz(kmin ^ kmax);
            int leader = __ffsll((unsigned long long)members) - 1;
            uint32_t lk = (uint32_t)__shfl((int)ki, leader, 64);
            members &= __ballot(((ki ^ lk) >> hb) == 0u);
        }
        pending &= ~members;
        const bool mem = (members >> lane) & 1ull;

        while (true) {
            const bool act = mem && !stop;
            if (!__ballot(act)) break;
            const double hc = hnext;
            const double twoh = 2.0 * hc;
            const double r2max = twoh * twoh;
            // union box of the active lanes
            double Rmax = wave_max_d(act ? twoh : 0.0);
            double blo[3], bhi[3];
            {
                const double p3[3] = {xi, yi, zi};
                for (int d = 0; d < 3; ++d) {
                    blo[d] = wave_min_d(act ? p3[d] - twoh : INFINITY) - S.margin;
                    bhi[d] = wave_max_d(act ? p3[d] + twoh : -INFINITY) + S.margin;
                }
            }
            double span = fmax(fmax(bhi[0] - blo[0], bhi[1] - blo[1]), bhi[2] - blo[2]);
            int l = S.lmax;
            while (l > 0) {
                bool ok = true;
                for (int d = 0; d < 3; ++d) {
                    double cw = ldexp(S.L[d], -l);
                    if (S.L[d] > 0.0 && (cw * S.div < Rmax + S.margin || cw * 16.0 < span)) ok = false;
                }
                if (ok) break;
                --l;
            }
            const int nl = 1 << l;
            const int msk = nl - 1;
            int a[3], cnt[3];
            for (int d = 0; d < 3; ++d) {
                if (!(S.L[d] > 0.0)) { a[d] = 0; cnt[d] = 1; continue; }
                double wd = ldexp(S.L[d], -l);
                double ta = floor((blo[d] - S.lo[d]) / wd);
                double tb = floor((bhi[d] - S.lo[d]) / wd);
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
                cnt[d] = max(ib - ia + 1, 0);
            }
            const int sh = 3 * (S.lmax - l);
            const int ncell = cnt[0] * cnt[1] * cnt[2];
            int N = 0;
            int32_t *wp = idx + i;   // slot N of this particle's gather set
            for (int cb = 0; cb < ncell; cb += 64) {
                int c = cb + lane;
                int s0 = 0, len = 0;
                if (c < ncell) {
                    int kx = c % cnt[0];
                    int ky = (c / cnt[0]) % cnt[1];
                    int kz = c / (cnt[0] * cnt[1]);
                    uint32_t code = morton((uint32_t)((a[0] + kx) & msk),
                                           (uint32_t)((a[1] + ky) & msk),
                                           (uint32_t)((a[2] + kz) & msk));
                    s0 = S.cs[(int64_t)code << sh];
                    len = S.cs[((int64_t)code + 1) << sh] - s0;
                }
                int incl = wave_incl_scan_i(len);
                int total = __shfl(incl, 63, 64);
                wave_lds_sync();
                s_start[w][lane] = s0;
                s_pre[w][lane] = incl - len;
                wave_lds_sync();
                if (act) tested += total;
                for (int base = 0; base < total; base += 64) {
                    int v = base + lane;
                    if (v < total) {
                        int r = 0;
                        for (int st = 32; st > 0; st >>= 1)
                            if (s_pre[w][r + st] <= v) r += st;
                        int j = s_start[w][r] + (v - s_pre[w][r]);
                        Cand cd;
                        cd.x = x[j];
                        cd.y = y[j];
                        cd.z = z[j];
                        cd.j = j;
                        cd.pad = 0;
                        s_c[w][lane] = cd;
                    }
                    wave_lds_sync();
                    const int m = min(64, total - base);
                    if (act) {
#pragma unroll 4
                        for (int t = 0; t < m; ++t) {
                            const Cand cd = s_c[w][t];
                            double dx = mimg<PM, 0>(xi, cd.x, g);
                            double dy = mimg<PM, 1>(yi, cd.y, g);
                            double dz = mimg<PM, 2>(zi, cd.z, g);
                            double r2 = exact_r2(dx, dy, dz);
                            if (r2 < r2max && cd.j != (int)i) {
                                if (N < K) *wp = cd.j;
                                wp += stride;
                                ++N;
                            }
                        }
                    }
                    wave_lds_sync();
                }
            }
            if (act) {
                ++counts;
                last_h = hc;
                int dev = N > target ? N - target : target - N;
                if (!tried) {
                    tried = true;
                    if (dev <= tol) {
                        stop = conv = true;
                        best_h = hc;
                        best_n = N;
                        fl = SPH_FLAG_LEARNED;
                        ++acc;
                    } else {
                        ++fallback;
                        hnext = hcur;
                    }
                } else {
                    int bdev = best_n > target ? best_n - target : target - best_n;
                    if (best_n < 0 || dev < bdev || (dev == bdev && hc < best_h)) {
                        best_h = hc;
                        best_n = N;
                    }
                    if (dev <= tol) {
                        stop = conv = true;
                    } else {
                        if (N < target - tol) {
                            if (!have_lo || hc > lo_b) lo_b = hc;
                            have_lo = true;
                        } else {
                            if (!have_hi || hc < hi_b) hi_b = hc;
                            have_hi = true;
                        }
                        ++itk;
                        if (itk >= maxit) stop = true;
                        else if (have_lo && have_hi) hnext = 0.5 * (lo_b + hi_b);
                        else hnext = hc * hk[N < 1023 ? N : 1023];
                    }
                }
            }
        }
    }
    int64_t nonconv = 0, overflow = 0;
    if (valid) {
        if (!conv) { fl |= SPH_FLAG_NOCONV; ++nonconv; }
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
template <int PM>
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
        int N = count_fill<PM>(S, x, y, z, i, x[i], y[i], z[i], h[i], idx, stride, K, true, tested);
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
    SPH_DISPATCH_PM(periodic_mask(g),
        hipLaunchKernelGGL(k_hsolve<PM>, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur],
                           s->y[cur], s->z[cur], s->key, s->h[cur], s->nc[cur], s->flags,
                           c->w.refill, nl->idx, nl->stride, p.list_stride, c->w.cell_start,
                           c->w.bbox, g, p.max_level, p.search_div, c->w.hk, p.n_target, p.n_tol,
                           p.h_max_iter, h_try, c->w.status);
        hipLaunchKernelGGL(k_refill<PM>, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur],
                           s->y[cur], s->z[cur], s->h[cur], s->nc[cur], c->w.refill, nl->idx,
                           nl->stride, p.list_stride, c->w.cell_start, c->w.bbox, g, p.max_level,
                           1, c->w.status))
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

hipError_t launch_zero_i32(sph_ctx *c, int32_t *a, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, a, n);
    return hipGetLastError();
}

template <int PM>
__global__ __launch_bounds__(SPH_BLOCK) void k_extra(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ h, const int32_t *__restrict__ nc,
    const int32_t *__restrict__ idx, int64_t stride, int K, Geo g, int32_t *__restrict__ ecnt,
    int32_t *__restrict__ eidx, int slots, int64_t *__restrict__ status)
{
#pragma clang fp contract(off)
    int64_t i = global_index();
    int64_t appended = 0, dropped = 0;
    if (i < n) {
        double xi = x[i], yi = y[i], zi = z[i];
        int m = min(nc[i], K);
        for (int k = 0; k < m; ++k) {
            int j = idx[(int64_t)k * stride + i];
            double dx = mimg<PM, 0>(xi, x[j], g);
            double dy = mimg<PM, 1>(yi, y[j], g);
            double dz = mimg<PM, 2>(zi, z[j], g);
            double r2 = exact_r2(dx, dy, dz);
            double twoh = 2.0 * h[j];
            if (!(r2 < twoh * twoh)) extra_append(j, (int)i, ecnt, eidx, stride, slots, appended, dropped);
        }
    }
    block_add_i64(appended, status + ST_EXTRA_TOTAL);
    block_add_i64(dropped, status + ST_EXTRA_OVERFLOW);
}

hipError_t launch_extra(sph_ctx *c, sph_particles *s, sph_nlist *nl)
{
    int64_t n = s->n;
    const sph_params &p = c->p;
    int cur = s->cur;
    hipError_t e = launch_zero_i32(c, nl->ecnt, n);
    if (e != hipSuccess || n == 0) return e;
    Geo g = make_geo(p);
    unsigned nb = (unsigned)ceil_div(n, SPH_BLOCK);
    SPH_DISPATCH_PM(periodic_mask(g),
        hipLaunchKernelGGL(k_extra<PM>, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->x[cur],
                           s->y[cur], s->z[cur], s->h[cur], s->nc[cur], nl->idx, nl->stride,
                           p.list_stride, g, nl->ecnt, nl->eidx, p.extra_slots, c->w.status))
    return hipGetLastError();
}
