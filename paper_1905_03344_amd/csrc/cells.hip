// Cell list construction: bounding box, Morton keys, stable LSD radix sort,
// permutation of the particle fields, cell-start table; device-wide scans.
#include "sph_internal.h"

// ---------------------------------------------------------------------------
// bounding box: exact min / max per dimension (order independent)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_bbox_partial(const double *__restrict__ x,
                                                            const double *__restrict__ y,
                                                            const double *__restrict__ z,
                                                            int64_t n, double *__restrict__ part)
{
    __shared__ double sh[6][SPH_BLOCK];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v[3] = {x[i], y[i], z[i]};
        for (int d = 0; d < 3; ++d) {
            mn[d] = fmin(mn[d], v[d]);
            mx[d] = fmax(mx[d], v[d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = mn[d];
        sh[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + s]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(SPH_BLOCK) void k_bbox_final(const double *__restrict__ part,
                                                          int64_t nb, int64_t n, Geo g,
                                                          double lo0, double lo1, double lo2,
                                                          double hi0, double hi1, double hi2,
                                                          double *__restrict__ bbox)
{
    __shared__ double sh[6][SPH_BLOCK];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = threadIdx.x; k < nb; k += SPH_BLOCK)
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], part[k * 6 + d]);
            v[3 + d] = fmax(v[3 + d], part[k * 6 + 3 + d]);
        }
    for (int d = 0; d < 6; ++d) sh[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + s]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        int d = threadIdx.x;
        double a = sh[d][0], b = sh[3 + d][0];
        if (n == 0) { a = 0.0; b = 0.0; }
        double blo[3] = {lo0, lo1, lo2}, bhi[3] = {hi0, hi1, hi2};
        if (g.per[d]) { a = blo[d]; b = bhi[d]; }
        bbox[d] = a;
        bbox[3 + d] = b;
    }
}

hipError_t launch_bbox(sph_ctx *c, const double *x, const double *y, const double *z, int64_t n)
{
    int64_t nb = c->w.nb_red;
    if (n < nb * SPH_BLOCK) nb = ceil_div(n > 0 ? n : 1, SPH_BLOCK);
    hipLaunchKernelGGL(k_bbox_partial, dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, x, y, z,
                       n, c->w.bbox_part);
    const sph_params &p = c->p;
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(SPH_BLOCK), 0, c->stream, c->w.bbox_part, nb, n,
                       make_geo(p), p.box_lo[0], p.box_lo[1], p.box_lo[2], p.box_hi[0],
                       p.box_hi[1], p.box_hi[2], c->w.bbox);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// keys: 10 bits per dimension of the cell index in the bounding box
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_keys(const double *__restrict__ x,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ z, int64_t n,
                                                    const double *__restrict__ bbox,
                                                    uint32_t *__restrict__ key,
                                                    int32_t *__restrict__ val)
{
#pragma clang fp contract(off)
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double lo0 = bbox[0], lo1 = bbox[1], lo2 = bbox[2];
    double L0 = bbox[3] - lo0, L1 = bbox[4] - lo1, L2 = bbox[5] - lo2;
    key[i] = morton((uint32_t)cell10(x[i], lo0, L0), (uint32_t)cell10(y[i], lo1, L1),
                    (uint32_t)cell10(z[i], lo2, L2));
    val[i] = (int32_t)i;
}

hipError_t launch_keys(sph_ctx *c, const double *x, const double *y, const double *z, int64_t n)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, x, y, z, n, c->w.bbox, c->w.key_a, c->w.val_a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// device-wide exclusive scans (fixed order, deterministic)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan of the per-thread totals of one block; returns the
// exclusive prefix of this thread and writes the block total to *total
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total)
{
    __shared__ T wsum[SPH_BLOCK / 64];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    T before = 0, all = 0;
    for (int k = 0; k < SPH_BLOCK / 64; ++k) {
        if (k < wv) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(SPH_BLOCK) void k_scan_reduce(const TI *__restrict__ in, int64_t n,
                                                           uint64_t *__restrict__ part)
{
    int64_t base = blockIdx.x * (int64_t)SPH_SCAN_TILE + threadIdx.x * SPH_SCAN_ITEMS;
    uint64_t s = 0;
    for (int k = 0; k < SPH_SCAN_ITEMS; ++k)
        if (base + k < n) s += (uint64_t)(TO)in[base + k];
    uint64_t tot;
    block_excl_scan<uint64_t>(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of nb partials in place, grand total at part[nb]
__global__ __launch_bounds__(SPH_BLOCK) void k_scan_partials(uint64_t *__restrict__ part,
                                                             int64_t nb)
{
    int64_t per = ceil_div(nb, SPH_BLOCK);
    int64_t b0 = threadIdx.x * per;
    uint64_t s = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) s += part[b0 + k];
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t>(s, &tot);
    for (int64_t k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            uint64_t v = part[b0 + k];
            part[b0 + k] = ex;
            ex += v;
        }
    }
    if (threadIdx.x == 0) part[nb] = tot;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(SPH_BLOCK) void k_scan_apply(const TI *__restrict__ in, int64_t n,
                                                          const uint64_t *__restrict__ part,
                                                          int64_t nb, TO *__restrict__ out,
                                                          int write_total)
{
    int64_t base = blockIdx.x * (int64_t)SPH_SCAN_TILE + threadIdx.x * SPH_SCAN_ITEMS;
    TO v[SPH_SCAN_ITEMS];
    uint64_t s = 0;
    for (int k = 0; k < SPH_SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? (TO)in[base + k] : (TO)0;
        s += (uint64_t)v[k];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t>(s, &tot) + part[blockIdx.x];
    for (int k = 0; k < SPH_SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = (TO)ex;
        ex += (uint64_t)v[k];
    }
    if (write_total && blockIdx.x == 0 && threadIdx.x == 0) out[n] = (TO)part[nb];
}

template <typename TI, typename TO>
static hipError_t scan_impl(sph_ctx *c, const TI *in, TO *out, int64_t n, int write_total)
{
    int64_t nb = ceil_div(n > 0 ? n : 1, SPH_SCAN_TILE);
    if (nb + 1 > c->w.scan_part_len) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream,
                       in, n, c->w.scan_part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SPH_BLOCK), 0, c->stream, c->w.scan_part, nb);
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream,
                       in, n, c->w.scan_part, nb, out, write_total);
    return hipGetLastError();
}

// out has n+1 entries: out[n] = total
hipError_t launch_scan_i32_to_i64(sph_ctx *c, const int32_t *in, int64_t *out, int64_t n)
{
    return scan_impl<int32_t, int64_t>(c, in, out, n, 1);
}

hipError_t launch_scan_u32(sph_ctx *c, const uint32_t *in, uint32_t *out, int64_t n)
{
    return scan_impl<uint32_t, uint32_t>(c, in, out, n, 0);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, 4 passes over the 30-bit keys.
// Pass = per-tile digit histogram, exclusive scan over (digit, tile), and a
// stable scatter that ranks equal digits by wave ballots in index order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_sort_hist(const uint32_t *__restrict__ key,
                                                         int64_t n, int shift, int64_t nb,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[SPH_BLOCK / 64][256];
    int wv = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < 256 * (SPH_BLOCK / 64); k += SPH_BLOCK) (&h[0][0])[k] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * (int64_t)SPH_SORT_TILE;
    for (int r = 0; r < SPH_SORT_ITEMS; ++r) {
        int64_t i = base + r * SPH_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[wv][(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += SPH_BLOCK) {
        uint32_t t = 0;
        for (int k = 0; k < SPH_BLOCK / 64; ++k) t += h[k][d];
        hist[(int64_t)d * nb + blockIdx.x] = t;
    }
}

// Stable scatter of one tile: the tile's keys are ranked in index order
// (16 rounds of 256, equal digits of a wave ranked by ballots) into LDS,
// grouped by digit, then written out in that order, so that the keys of one
// digit leave the tile as one contiguous run instead of one store each.
__global__ __launch_bounds__(SPH_BLOCK) void k_sort_scatter(
    const uint32_t *__restrict__ key_in, const int32_t *__restrict__ val_in, int64_t n, int shift,
    int64_t nb, const uint32_t *__restrict__ offs, uint32_t *__restrict__ key_out,
    int32_t *__restrict__ val_out)
{
    __shared__ uint32_t lkey[SPH_SORT_TILE];
    __shared__ int32_t lval[SPH_SORT_TILE];
    __shared__ uint32_t lstart[256];   // first slot of each digit in the tile
    __shared__ uint32_t run[256];      // next slot of each digit
    __shared__ uint32_t wcount[SPH_BLOCK / 64][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x * (int64_t)SPH_SORT_TILE;
    const int tn = (int)min((int64_t)SPH_SORT_TILE, n - tile);   // keys in this tile
    // the tile's digit counts, then their exclusive prefix
    for (int d = threadIdx.x; d < 256; d += SPH_BLOCK) run[d] = 0;
    __syncthreads();
    for (int r = 0; r < SPH_SORT_ITEMS; ++r) {
        const int k = r * SPH_BLOCK + threadIdx.x;
        if (k < tn) atomicAdd(&run[(key_in[tile + k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // 256 counts, 4 per lane, exclusive scan across the wave
        uint32_t c[4], t = 0;
        for (int v = 0; v < 4; ++v) {
            c[v] = run[4 * threadIdx.x + v];
            t += c[v];
        }
        uint32_t incl = t;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
            if ((int)threadIdx.x >= o) incl += y;
        }
        uint32_t e = incl - t;
        for (int v = 0; v < 4; ++v) {
            lstart[4 * threadIdx.x + v] = e;
            run[4 * threadIdx.x + v] = e;
            e += c[v];
        }
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < SPH_SORT_ITEMS; ++r) {
        for (int k = threadIdx.x; k < 256 * (SPH_BLOCK / 64); k += SPH_BLOCK)
            (&wcount[0][0])[k] = 0;
        __syncthreads();
        const int k = r * SPH_BLOCK + threadIdx.x;
        const bool valid = k < tn;
        const uint32_t k_ = valid ? key_in[tile + k] : 0u;
        const int32_t v_ = valid ? val_in[tile + k] : 0;
        const uint32_t d = (k_ >> shift) & 255u;
        uint64_t same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(same & lt);
        if (valid && rank == 0) wcount[wv][d] = (uint32_t)__popcll(same);
        __syncthreads();
        // per digit: prefix over the waves, then advance the digit's slot
        for (int dd = threadIdx.x; dd < 256; dd += SPH_BLOCK) {
            uint32_t at = run[dd];
            for (int w = 0; w < SPH_BLOCK / 64; ++w) {
                const uint32_t t = wcount[w][dd];
                wcount[w][dd] = at;
                at += t;
            }
            run[dd] = at;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcount[wv][d] + rank;
            lkey[pos] = k_;
            lval[pos] = v_;
        }
        // every wave has read this round's wcount before the next clears it
        __syncthreads();
    }
    // out in slot order: slot s of digit d goes to offs[d] + (s - lstart[d])
    for (int s = threadIdx.x; s < tn; s += SPH_BLOCK) {
        const uint32_t k_ = lkey[s];
        const uint32_t d = (k_ >> shift) & 255u;
        const uint32_t pos = offs[(int64_t)d * nb + blockIdx.x] + ((uint32_t)s - lstart[d]);
        key_out[pos] = k_;
        val_out[pos] = lval[s];
    }
}

// sorts c->w.key_a / val_a (filled by launch_keys) into key_out / val_out
hipError_t launch_radix_sort(sph_ctx *c, int64_t n, uint32_t *key_out, int32_t *val_out)
{
    if (n == 0) return hipSuccess;
    int64_t nb = ceil_div(n, SPH_SORT_TILE);
    if (nb > c->w.nb_sort) return hipErrorInvalidValue;
    const uint32_t *kin = c->w.key_a;
    const int32_t *vin = c->w.val_a;
    // ping-pong: pass 0 a->b, 1 b->out, 2 out->b, 3 b->out
    uint32_t *kdst[4] = {c->w.key_b, key_out, c->w.key_b, key_out};
    int32_t *vdst[4] = {c->w.val_b, val_out, c->w.val_b, val_out};
    for (int pass = 0; pass < 4; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, kin, n,
                           shift, nb, c->w.hist);
        hipError_t e = launch_scan_u32(c, c->w.hist, c->w.hist, 256 * nb);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, kin,
                           vin, n, shift, nb, c->w.hist, kdst[pass], vdst[pass]);
        kin = kdst[pass];
        vin = vdst[pass];
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// permutation of every carried field from buffer cur into 1 - cur
// ---------------------------------------------------------------------------
#define SPH_PERM_MAX 16
struct PermArgs {
    int nf;   // double fields in use (15, or 16 with the Adams-Bashforth du_prev)
    const double *src[SPH_PERM_MAX];
    double *dst[SPH_PERM_MAX];
    const int32_t *isrc[2];
    int32_t *idst[2];
};

__global__ __launch_bounds__(SPH_BLOCK) void k_permute(PermArgs a, const int32_t *__restrict__ perm,
                                                       int64_t n)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t s = perm[k];
#pragma unroll
    for (int f = 0; f < SPH_PERM_MAX; ++f)
        if (f < a.nf) a.dst[f][k] = a.src[f][s];
    a.idst[0][k] = a.isrc[0][s];
    a.idst[1][k] = a.isrc[1][s];
}

hipError_t launch_permute(sph_ctx *c, sph_particles *s, const int32_t *perm)
{
    if (s->n == 0) return hipSuccess;
    int a = s->cur, b = 1 - s->cur;
    PermArgs pa;
    double **fields[15] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m, s->h,
                           s->u, s->ax, s->ay, s->az, s->du, s->rho, s->divv};
    for (int f = 0; f < 15; ++f) {
        pa.src[f] = fields[f][a];
        pa.dst[f] = fields[f][b];
    }
    pa.nf = 15;
    if (c->p.integrator == SPH_INTEGRATOR_AB2) {
        pa.src[15] = c->w.du_prev[a];
        pa.dst[15] = c->w.du_prev[b];
        pa.nf = 16;
    }
    pa.isrc[0] = s->nc[a]; pa.idst[0] = s->nc[b];
    pa.isrc[1] = s->id[a]; pa.idst[1] = s->id[b];
    hipLaunchKernelGGL(k_permute, dim3((unsigned)ceil_div(s->n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, pa, perm, s->n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cell-start table at level lmax: start[c] = first sorted index whose key is
// in cell c (or later), for c in [0, 8^lmax]; one thread per entry, by
// binary search over the sorted keys (the table stays cheap to build where
// most cells are empty).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_cell_table(const uint32_t *__restrict__ key,
                                                          int64_t n, int shift, int64_t ncell,
                                                          int32_t *__restrict__ start)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c > ncell) return;
    int64_t lo = 0, hi = n;   // first k in [lo, hi] with key[k] >> shift >= c
    if (c < ncell) {
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(key[mid] >> shift) < c) lo = mid + 1;
            else hi = mid;
        }
    } else {
        lo = n;
    }
    start[c] = (int32_t)lo;
}

hipError_t launch_cell_table(sph_ctx *c, const uint32_t *sorted_key, int64_t n)
{
    int l = c->p.max_level;
    int64_t ncell = (int64_t)1 << (3 * l);
    hipLaunchKernelGGL(k_cell_table, dim3((unsigned)ceil_div(ncell + 1, SPH_BLOCK)), dim3(SPH_BLOCK),
                       0, c->stream, sorted_key, n, 3 * (10 - l), ncell, c->w.cell_start);
    return hipGetLastError();
}
