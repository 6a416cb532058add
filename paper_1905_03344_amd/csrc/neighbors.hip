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
    int prefilter;   // SPH_PREFILTER_*
    int defer;       // first round: sub-groups of at most this many go to the tail
    double lo[3], L[3];
    double margin;
    Geo g;
};

__device__ __forceinline__ Search make_search(const int32_t *cs, int lmax, int div, int prefilter,
                                              int defer, const double *bbox, Geo g)
{
    Search S;
    S.cs = cs;
    S.lmax = lmax;
    S.div = div;
    S.prefilter = prefilter;
    S.defer = defer;
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
// the set into row i of idx.
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
                if (write && cnt < K) idx[(int64_t)i * K + cnt] = j;
                ++cnt;
            }
        }
    });
    return cnt;
}

// ---------------------------------------------------------------------------
// Smoothing-length iteration.
// Per particle the arithmetic is the iteration of the paper's reading:
//   N = count at h; keep the best (h, N) by |N - target| (ties: smaller h);
//   stop when |N - target| <= tol; below the band raise the lower bracket,
//   above it lower the upper bracket; bisect once both are set, else
//   h *= T[min(N, 1023)]; at most maxit counts.
// Structure: round 0 counts every particle once with wave-cooperative
// walks (below) and, in runs below SPH_BIG_N particles, keeps iterating on
// the shell of that count while the next h stays inside it.  Particles that
// need another full count go to one wave-cooperative worklist round (large
// runs: with the shell there), and what remains, with the particles of small
// (scattered) groups that round 0 leaves alone, to the tail: one wave per
// particle, full counts until the iteration ends.
// With h_try (learned mode) round 0 counts at h_try[i] (with the plain
// count's shell only where many tries miss, SPH_TRY_SHELL_MIN_N) and accepts
// it when in the band.  A miss starts the plain iteration from h[i]: on the
// try's shell when h[i] lies inside it, else in the worklist round (the tail
// when misses are few), whose first count of such a particle is the plain
// solve's round-0 count (with the shell and the iteration on it).
// Every count is exact, so a miss follows the plain solve's path and ends
// on its h; cells are walked in Morton order, so gather sets do not depend
// on which wave counts them.
// The gather set of the last counted h is written (row i of idx), ascending
// (a set completed from a shell is merged in place); particles whose kept h
// is not the last counted one are rewritten by k_refill.
//
// Counting is wave-cooperative: a wave owns 64 particles (consecutive in
// Morton order, or consecutive entries of a worklist), split into groups of
// nearby particles.  A large group builds the union of its search boxes,
// walks its cells in batches of 64 (one cell per lane, prefix sums of the
// cell sizes), streams the candidates in tiles of 64 through LDS and lets
// every member lane test every candidate of the tile against its own
// particle (broadcast LDS reads): control flow is uniform and candidate
// loads are coalesced.  A small group is counted one particle at a time
// with one candidate per lane (transposed mode).
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
#define WAVES_PER_BLOCK (SPH_BLOCK / 64)

struct WaveLds {
    Cand c[64];
    int start[64];
    int pre[64];
    int qs[128];   // queue of non-empty cells in Morton order: first particle
    int ql[128];   // and particle count
    uint32_t cf[64][8];   // Gram features of the tile's candidates (16 bf16 each)
    uint32_t mf[64][8];   // Gram features of the members, outer threshold
    uint32_t ma[64];      // the two features that differ for the inner threshold
};

// ---------------------------------------------------------------------------
// Gram prefilter of a union tile on the matrix cores.  With u = s (x - c)
// (c the box centre, s a power of two with s R_max in [1/2, 1)), the squared
// distance of member i and candidate j minus a threshold T_i is the dot
// product of two 16-vectors:
//   member    M = (-2a_i, -2a_i, -2b_i, 1, 1, hi(|u_i|^2 - T_i), lo(..), 0, 0, 0)
//   candidate C = ( a_j,   b_j,   a_j,  hi(|u_j|^2), lo(|u_j|^2), 1, 1, 0, 0, 0)
// where a + b is a two-term bfloat16 split of u (the dropped b_i b_j and the
// split remainders are below 2^-17 U^2) and the products are exact in the
// FP32 accumulator.  With U^2 >= |u|^2 over the whole cell box, every error
// term together stays below 2^-14 (U^2 + T_max) (2^-16 observed on random
// boxes), so with the band delta = 2^-11 (U^2 + T_max):
//   D < 0 for T = B + delta  keeps every candidate with r^2 < B  (a superset),
//   D < 0 for T = A - delta  holds only candidates with r^2 < A  (certainly inner),
// and the candidates between the two are decided by the exact FP64 r^2.
// One 16x16x16 MFMA covers 16 candidates x 16 members; a 64 x 64 tile takes
// 16 per threshold.
// ---------------------------------------------------------------------------
typedef short gs4_t __attribute__((ext_vector_type(4)));
typedef float gf4_t __attribute__((ext_vector_type(4)));

struct Gram {
    bool ok;
    double c[3];
    double s, s2, delta;
    int wrap[3];
    double L[3], halfL[3];
};

__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_float(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ void bf16_split(double v, uint32_t &hi, uint32_t &lo)
{
    hi = bf16_rne((float)v);
    lo = bf16_rne((float)(v - (double)bf16_float(hi)));
}

__device__ __forceinline__ double gram_rel(const Gram &G, int d, double x)
{
    double r = x - G.c[d];
    if (G.wrap[d]) {
        if (r > G.halfL[d]) r -= G.L[d];
        else if (r < -G.halfL[d]) r += G.L[d];
    }
    return r * G.s;
}

// candidate features into f[0..7] (pairs of bf16, element 2k in the low half)
__device__ __forceinline__ void gram_cand(const Gram &G, double x, double y, double z, uint32_t *f)
{
    const double u[3] = {gram_rel(G, 0, x), gram_rel(G, 1, y), gram_rel(G, 2, z)};
    uint32_t a[3], b[3], nh, nl;
    for (int d = 0; d < 3; ++d) bf16_split(u[d], a[d], b[d]);
    bf16_split(u[0] * u[0] + u[1] * u[1] + u[2] * u[2], nh, nl);
    const uint32_t one = 0x3F80u;
    f[0] = a[0] | a[1] << 16;
    f[1] = a[2] | b[0] << 16;
    f[2] = b[1] | b[2] << 16;
    f[3] = a[0] | a[1] << 16;
    f[4] = a[2] | nh << 16;
    f[5] = nl | one << 16;
    f[6] = one;
    f[7] = 0u;
}

// member features for thresholds TB (all eight words) and TA (words 5 and 6
// differ: ma = hi | lo << 16 of |u|^2 - TA)
__device__ __forceinline__ void gram_member(const Gram &G, double x, double y, double z, double TB,
                                            double TA, uint32_t *f, uint32_t &ma)
{
    const double u[3] = {gram_rel(G, 0, x), gram_rel(G, 1, y), gram_rel(G, 2, z)};
    uint32_t m2a[3], m2b[3];
    for (int d = 0; d < 3; ++d) {
        uint32_t a, b;
        bf16_split(u[d], a, b);
        m2a[d] = bf16_rne(-2.0f * bf16_float(a));   // exact
        m2b[d] = bf16_rne(-2.0f * bf16_float(b));
    }
    const double n = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    uint32_t bh, bl, ah, al;
    bf16_split(n - TB, bh, bl);
    bf16_split(n - TA, ah, al);
    const uint32_t one = 0x3F80u;
    f[0] = m2a[0] | m2a[1] << 16;
    f[1] = m2a[2] | m2a[0] << 16;
    f[2] = m2a[1] | m2a[2] << 16;
    f[3] = m2b[0] | m2b[1] << 16;
    f[4] = m2b[2] | one << 16;
    f[5] = one | bh << 16;
    f[6] = bl;
    f[7] = 0u;
    ma = ah | al << 16;
}

__device__ __forceinline__ gs4_t gram_op(uint32_t w0, uint32_t w1)
{
    gs4_t r;
    r[0] = (short)(w0 & 0xFFFFu);
    r[1] = (short)(w0 >> 16);
    r[2] = (short)(w1 & 0xFFFFu);
    r[3] = (short)(w1 >> 16);
    return r;
}

// All 64 lanes: this lane's masks over the tile's candidates (lane = member):
// bit t of hb when D_B(t) < 0, of ha when D_A(t) < 0.
// Lane (q, j) = (lane / 16, lane % 16) feeds row j of each row block rb with
// candidate 16 (j / 4) + 4 rb + j % 4, so that the D rows it holds (4q + v)
// are the candidates 16q + 4rb + v: its sign bits, collected rb- and v-major
// by alignbit, are bits 16q .. 16q + 15 of the mask of member cb*16 + j.  A
// 4 x 4 transpose over the lanes (q, j), q = 0..3, in two exchange steps
// then gives every lane the four words of its own member.
__device__ __forceinline__ void gram_tile(const WaveLds &L, int lane, uint64_t &hb, uint64_t &ha)
{
    const int q = lane >> 4, j = lane & 15;
    const int cbase = 16 * (j >> 2) + (j & 3);
    gs4_t A[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const uint2 w = *reinterpret_cast<const uint2 *>(&L.cf[cbase + 4 * rb][2 * q]);
        A[rb] = gram_op(w.x, w.y);
    }
    const gf4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
    uint32_t w[4];   // per column block: outer bits | inner bits << 16
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int m = cb * 16 + j;
        const uint2 mw = *reinterpret_cast<const uint2 *>(&L.mf[m][2 * q]);
        const uint32_t mav = L.ma[m];
        uint2 wa = mw;
        if (q == 2) wa.y = (mw.y & 0xFFFFu) | (mav << 16);        // element 11
        if (q == 3) wa.x = (mw.x & 0xFFFF0000u) | (mav >> 16);    // element 12
        const gs4_t MB = gram_op(mw.x, mw.y), MA = gram_op(wa.x, wa.y);
        uint32_t ob = 0, ib = 0;
#pragma unroll
        for (int rb = 3; rb >= 0; --rb) {
            const gf4_t db = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[rb], MB, zero, 0, 0, 0);
            const gf4_t da = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[rb], MA, zero, 0, 0, 0);
#pragma unroll
            for (int v = 3; v >= 0; --v) {
                ob = __builtin_amdgcn_alignbit(ob, __float_as_uint(db[v]), 31);
                ib = __builtin_amdgcn_alignbit(ib, __float_as_uint(da[v]), 31);
            }
        }
        w[cb] = (ob & 0xFFFFu) | (ib << 16);
    }
    // step 1, partner q ^ 1: keep the columns of this lane's parity
    const bool odd = (q & 1) != 0, upper = (q & 2) != 0;
    const uint32_t keep0 = odd ? w[1] : w[0], keep2 = odd ? w[3] : w[2];
    const uint32_t r0 = (uint32_t)__shfl_xor((int)(odd ? w[0] : w[1]), 16, 64);
    const uint32_t r2 = (uint32_t)__shfl_xor((int)(odd ? w[2] : w[3]), 16, 64);
    // step 2, partner q ^ 2: keep this lane's column
    const uint32_t u0 = (uint32_t)__shfl_xor((int)(upper ? keep0 : keep2), 32, 64);
    const uint32_t u1 = (uint32_t)__shfl_xor((int)(upper ? r0 : r2), 32, 64);
    // rows q, q^1, q^2, q^3 of column q, put in row order (index xor q)
    uint32_t e0 = upper ? keep2 : keep0, e1 = upper ? r2 : r0, e2 = u0, e3 = u1;
    if (odd) {
        const uint32_t t0 = e0, t2 = e2;
        e0 = e1; e1 = t0; e2 = e3; e3 = t2;
    }
    if (upper) {
        const uint32_t t0 = e0, t1 = e1;
        e0 = e2; e1 = e3; e2 = t0; e3 = t1;
    }
    const uint32_t blo = (e0 & 0xFFFFu) | (e1 << 16), bhi = (e2 & 0xFFFFu) | (e3 << 16);
    const uint32_t alo = (e0 >> 16) | (e1 & 0xFFFF0000u), ahi = (e2 >> 16) | (e3 & 0xFFFF0000u);
    hb = (uint64_t)blo | ((uint64_t)bhi << 32);
    ha = (uint64_t)alo | ((uint64_t)ahi << 32);
}

// ascending bitonic sort of one value per lane across the wave
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t v)
{
    const int lane = threadIdx.x & 63;
    for (int k = 2; k <= 64; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint32_t o = (uint32_t)__shfl_xor((int)v, j, 64);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            v = (lower == up) ? min(v, o) : max(v, o);
        }
    return v;
}

// hits of one LDS tile for this lane: bit t of *in set when candidate t has
// r^2 < A (inside the shell), bit t of *sh when A <= r^2 < B (in the shell).
// FULL tiles skip the bound test; PMW is the periodic mask the tile needs
// (0 when the sub-group's box cannot wrap).
template <int PMW, bool FULL>
__device__ __forceinline__ void tile_hits(const WaveLds &L, int m, double xi, double yi, double zi,
                                          double A2, double B2, const Geo &g, uint64_t *in,
                                          uint64_t *sh)
{
#pragma clang fp contract(off)
    uint64_t hin = 0, hsh = 0;
    const int nb8 = FULL ? 8 : ((m + 7) >> 3);
    for (int b = 0; b < nb8; ++b) {
        uint32_t i8 = 0, s8 = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = 8 * b + u;
            const Cand cd = L.c[t];
            double dx = mimg<PMW, 0>(xi, cd.x, g);
            double dy = mimg<PMW, 1>(yi, cd.y, g);
            double dz = mimg<PMW, 2>(zi, cd.z, g);
            double r2 = exact_r2(dx, dy, dz);
            bool a = r2 < A2, b2 = r2 < B2;
            if (!FULL) { a = a && (t < m); b2 = b2 && (t < m); }
            i8 |= a ? (1u << u) : 0u;
            s8 |= b2 ? (1u << u) : 0u;
        }
        hin |= (uint64_t)i8 << (8 * b);
        hsh |= (uint64_t)s8 << (8 * b);
    }
    *in = hin;
    *sh = hsh & ~hin;
}

// exact r^2 of lane position and tile candidate t (same arithmetic as above)
template <int PMW>
__device__ __forceinline__ double tile_r2(const WaveLds &L, int t, double xi, double yi, double zi,
                                          const Geo &g)
{
#pragma clang fp contract(off)
    const Cand cd = L.c[t];
    return exact_r2(mimg<PMW, 0>(xi, cd.x, g), mimg<PMW, 1>(yi, cd.y, g),
                    mimg<PMW, 2>(zi, cd.z, g));
}

// Shell around a counted h: members with A <= r^2 < B, A = (2h(1-d))^2,
// B = (2h(1+d))^2, d = 1/SPH_SHELL_D.  For any h' with A <= (2h')^2 <= B the count
// is exactly N_inner + #{shell: r^2 < (2h')^2}: both sides use the same
// rounded r^2 and the same rounded (2h')^2.
// the shell is |r - 2h| < 2h / SPH_SHELL_D.  Its width only trades shell
// records against new walks (results do not depend on it): measured 1/24
// best on the jittered lattice (of 1/16 .. 1/64; the lattice's count moves
// by whole shells), 1/48 .. 1/64 on the smooth clumpy mixture (2% there)
#ifndef SPH_SHELL_D
#define SPH_SHELL_D 24.0
#endif
// shell of the learned try when it records none: 0 (every miss restarts
// with a new walk).  Where tries are accepted almost always, a shell costs
// more than it saves: a narrow one (|r - 2h| < 2h/96) took the 64M patch
// from 143 to 163 ms per step, the 1M clumpy mixture from 4.75 to 4.88 ms.
// Where many tries miss (the lattice, whose count moves by whole shells of
// neighbours), the try records the plain count's shell (SPH_SHELL_D)
// instead, chosen per solve from the previous one's misses
// (sph_params.learned_try_shell): 1M patch with 55% misses 3.91 -> 3.63 ms
// per step.  Not below SPH_TRY_SHELL_MIN_N particles, where a walk's time is
// one wave's latency and the shell's stores lengthen it more than the tail
// gains (8k patch, 69% misses: 1.60 -> 1.67 ms).
#ifndef SPH_TRY_SHELL_D
#define SPH_TRY_SHELL_D 0.0
#endif
#ifndef SPH_TRY_SHELL_MIN_N
#define SPH_TRY_SHELL_MIN_N 131072
#endif
// shell of round 0 under the worklist strategy (0: none).  Recording one
// costs round 0 more than the worklist round saves: 64M patch 165.5 ms per
// step without, 173.8 with |r - 2h| < 2h/48, 175.5 with 2h/96
// Skipping the cells of a union box that lie beyond every member's outer
// radius from the members' bounding box (its corners and edges) was
// measured and not kept: 6% fewer candidates on the 64M patch (1,559 ->
// 1,463 per particle) but a slower walk (52.5 -> 54.3 ms: the per-cell
// test and its registers), 1M clumpy mixture 6.02 -> 5.83 ms per step.
//
// widest union box, in cells per dimension, at the level a walk uses: a box
// of span <= S cells touches at most S + 2 cells, and up to 13 cells lie in
// at most 4 aligned blocks of 4 (64 blocks, one sorted batch).  On the 64M
// patch a 64-member union spans more than 12 cells of the next finer level
// (0.78 spacings), so S = 12 with level-9 cells and a search divisor of 3 or
// 4 left the level, the candidates (~1,540 per particle) and the walk time
// as they were, while the larger cell table cost 2.5 ms per step.
#ifndef SPH_SPAN_CELLS
#define SPH_SPAN_CELLS 11.0
#endif
// Learned mode gives its misses (restarted from h_prev) a wave-cooperative
// worklist round whatever n, unless they are few: fewer than
// SPH_LEARNED_ROUND_MIN and under a tenth of the particles, when the
// per-particle tail serves them better (scattered misses make large union
// boxes).  Measured, ms per step (mixed + learned): 1M patch (55% misses)
// 8.64 with the tail alone, 3.93 with the round; 8k patch 3.31 -> 1.55;
// 1M clumpy mixture (0.6%) 4.73 with the tail, 5.63 with the round.
// Deferring small groups of a worklist round to the tail (as round 0 does)
// made the plain 64M step slower (163.7 -> 170.7 ms) and is not done.
#ifndef SPH_LEARNED_ROUND_MIN
#define SPH_LEARNED_ROUND_MIN 65536
#endif
#ifndef SPH_WL_SHELL_D
#define SPH_WL_SHELL_D 0.0
#endif
// A shell member is one 8-byte entry: its index and its r^2 rounded to FP32
// (one store per member).  Counts from the shell stay exact: the FP32 value
// decides a comparison with a threshold T when it lies outside a relative
// band of 2^-22 around T (its rounding error is at most 2^-24 relative),
// and inside the band the FP64 r^2 is formed again from the positions.
#ifndef SPH_SHELL_BATCH
#define SPH_SHELL_BATCH 2
#endif
static_assert(SPH_SHELL_SLOTS + SPH_SHELL_BATCH <= 64, "shell member masks are 64-bit");
struct Shell {
    int2 *e;        // SPH_SHELL_SLOTS * sstride: (j, float bits of r^2)
    int64_t sstride;
};
__device__ __forceinline__ int2 shell_entry(int32_t j, double r2)
{
    return make_int2(j, __float_as_int((float)r2));
}

// Sub-groups of at most this many particles are counted one particle at a
// time with the candidates spread over the lanes (transposed mode); larger
// ones stream their union box through LDS tiles that every member tests
// (4 with SPH_SPLIT_H 3: measured best of 4, 6, 8, 16 on the jittered
// lattice; 16 suits the clumpy mixture alone)
#ifndef SPH_SMALL_GROUP
#define SPH_SMALL_GROUP 4
#endif
// in the all-particle first round, sub-groups of at most this many particles
// are left to the per-particle tail (one wave per particle) instead; the
// default of sph_params.walk_defer_group (4: best on the jittered lattice,
// 16 on the clumpy mixture, whose sparse regions leave many small groups)
#ifndef SPH_DEFER_GROUP
#define SPH_DEFER_GROUP 4
#endif
// a group is split by Morton prefix while its positions spread over more than
// this many search diameters (3: measured best of 1.5, 2, 3, 5)
#ifndef SPH_SPLIT_SPREAD
#define SPH_SPLIT_SPREAD 3.0
#endif
// lanes whose search radius exceeds this multiple of the group's smallest
// form a later group (3: measured best of 1.5, 2, 3, 4, 6 with the matrix-core
// candidate test; the clumpy mixture gains 7%, the lattice is indifferent)
#ifndef SPH_SPLIT_H
#define SPH_SPLIT_H 3.0
#endif

// exact r^2 between a lane's particle and candidate coordinates (the same
// arithmetic in both modes; PMW = 0 when the box cannot wrap, where the
// minimum image is the plain difference)
template <int PMW>
__device__ __forceinline__ double pair_r2(double xi, double yi, double zi, double xj, double yj,
                                          double zj, const Geo &g)
{
#pragma clang fp contract(off)
    return exact_r2(mimg<PMW, 0>(xi, xj, g), mimg<PMW, 1>(yi, yj, g), mimg<PMW, 2>(zi, zj, g));
}

// One walk over the cells of the box covering the member lanes' search
// spheres (radius sqrt(B)), in ascending Morton code.  Union mode: every
// member lane tests every candidate (LDS tiles).  Transposed mode
// (tm >= 0, one member, lane tm): lane t tests candidate t of each chunk of
// 64 against the member, and the member's counters are kept wave-uniform.
// Candidates with r^2 < T (A <= T <= B, the counted radius squared) are
// written to the row in candidate order, those with A <= r^2 < B to the
// shell; N counts the row's members.
template <int PM, bool TRANSPOSED>
__device__ void walk_group(WaveLds &L, uint64_t members, int tm, int64_t i, double xi, double yi,
                           double zi, double A2, double B2, double T2, const double *__restrict__ x,
                           const double *__restrict__ y, const double *__restrict__ z,
                           int32_t *__restrict__ idx, int64_t stride, int K, const Shell &SH,
                           const Search &S, const Geo &g, int &N, int &nsh, int32_t *&wp,
                           int64_t &tested)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const bool me = (members >> lane) & 1ull;
    const double Rout = sqrt(B2) * (1.0 + 1e-12);

    // union box of the members, wide enough for the shell's outer radius
    double Rmax = wave_max_d(me ? Rout : 0.0);
    double blo[3], bhi[3];
    {
        const double p3[3] = {xi, yi, zi};
        for (int d = 0; d < 3; ++d) {
            blo[d] = wave_min_d(me ? p3[d] - Rout : INFINITY) - S.margin;
            bhi[d] = wave_max_d(me ? p3[d] + Rout : -INFINITY) + S.margin;
        }
    }
    double span = fmax(fmax(bhi[0] - blo[0], bhi[1] - blo[1]), bhi[2] - blo[2]);
    int l = S.lmax;
    while (l > 0) {
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            double cw = ldexp(S.L[d], -l);
            if (S.L[d] > 0.0 && (cw * S.div < Rmax + S.margin || cw * SPH_SPAN_CELLS < span))
                ok = false;
        }
        if (ok) break;
        --l;
    }
    const int nl = 1 << l;
    const int msk = nl - 1;
    int a[3], cnt[3];
    bool wraps = false;
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
            // without a wrapped cell and with the box (plus one cell of
            // slack) under half the period, every |x_j - x_i| < L/2: the
            // minimum image is the plain difference
            if (ia < 0 || ib >= nl || (double)(ib - ia + 2) * wd > g.halfL[d]) wraps = true;
        } else {
            ia = max(ia, 0);
            ib = min(ib, nl - 1);
        }
        a[d] = ia;
        cnt[d] = max(ib - ia + 1, 0);
    }
    const int sh = 3 * (S.lmax - l);

    // Gram prefilter of the union tiles (see gram_tile): relative coordinates
    // to the box centre stay minimum images while the cell box spans under
    // half of every periodic length it wraps in
    Gram G;
    G.ok = false;
    if (!TRANSPOSED) {
        double U2 = 0.0;
        bool ok = S.prefilter == SPH_PREFILTER_MATRIX && Rmax > 0.0 && Rmax < INFINITY;
        for (int d = 0; d < 3; ++d) {
            const double cwd = ldexp(S.L[d], -l);
            G.c[d] = 0.5 * (blo[d] + bhi[d]);
            G.wrap[d] = wraps && S.g.per[d];
            G.L[d] = g.L[d];
            G.halfL[d] = g.halfL[d];
            if (S.g.per[d] && (double)cnt[d] * cwd > 0.45 * g.L[d]) ok = false;
            const double e0 = fabs(S.lo[d] + (double)a[d] * cwd - G.c[d]);
            const double e1 = fabs(S.lo[d] + (double)(a[d] + cnt[d]) * cwd - G.c[d]);
            const double e = fmax(fmax(e0, e1), fabs(bhi[d] - G.c[d]));
            U2 += e * e;
        }
        if (ok) {
            G.s = ldexp(1.0, -(ilogb(Rmax) + 1));
            G.s2 = G.s * G.s;
            U2 *= G.s2;
            G.delta = ldexp(U2 + Rmax * Rmax * G.s2, -11);
            G.ok = U2 < 1e30;
        }
        if (G.ok) {
            uint32_t f[8], ma = 0;
            if (me) {
                gram_member(G, xi, yi, zi, B2 * G.s2 + G.delta, A2 * G.s2 - G.delta, f, ma);
            } else {
                for (int k = 0; k < 8; ++k) f[k] = 0u;
            }
            for (int k = 0; k < 8; ++k) L.mf[lane][k] = f[k];
            L.ma[lane] = ma;
        }
    }
    // Cells are visited in ascending Morton code, so every member meets its
    // candidates in ascending particle index whatever the group: the gather
    // set of a particle at a given h comes out in one order.  The box is
    // covered by aligned blocks of 4^3 cells (fewer at levels 0 and 1) whose
    // codes are sorted across the wave (at most 64: at most 12 cells, so 4
    // blocks, per dimension by the level choice); inside a block lane t
    // takes the cell of local code t.
    const int kb = l < 2 ? l : 2;
    const int NB = nl >> kb;   // blocks per dimension
    int sa[3], sb[3], nbd[3];
    for (int d = 0; d < 3; ++d) {
        sa[d] = a[d] & msk;
        if (cnt[d] + (1 << kb) - 1 >= nl) {
            sb[d] = 0;
            nbd[d] = NB;
        } else {
            const int e = (sa[d] + cnt[d] - 1) & msk;
            sb[d] = sa[d] >> kb;
            nbd[d] = (((e >> kb) - sb[d]) & (NB - 1)) + 1;
        }
    }
    const int nblk = (cnt[0] > 0 && cnt[1] > 0 && cnt[2] > 0) ? nbd[0] * nbd[1] * nbd[2] : 0;
    const int nloc = 1 << (3 * kb);
    const uint32_t lx = compact3((uint32_t)lane), ly = compact3((uint32_t)lane >> 1),
                   lz = compact3((uint32_t)lane >> 2);

    // transposed mode: the member's data and counters, wave-uniform
    const double xm = TRANSPOSED ? __shfl(xi, tm, 64) : 0.0;
    const double ym = TRANSPOSED ? __shfl(yi, tm, 64) : 0.0;
    const double zm = TRANSPOSED ? __shfl(zi, tm, 64) : 0.0;
    const double A2m = TRANSPOSED ? __shfl(A2, tm, 64) : 0.0;
    const double B2m = TRANSPOSED ? __shfl(B2, tm, 64) : 0.0;
    const double T2m = TRANSPOSED ? __shfl(T2, tm, 64) : 0.0;
    const int64_t im = TRANSPOSED ? (int64_t)__shfl((int)i, tm, 64) : 0;
    int Nm = 0, nshm = 0;
    const uint64_t below = (1ull << lane) - 1ull;

    int wtag = 0;   // window tags of this walk
    L.pre[lane] = -1;
    // one batch of up to 64 non-empty cells (this lane: s0, len)
    auto batch = [&](int s0, int len) {
        int incl = wave_incl_scan_i(len);
        int total = __shfl(incl, 63, 64);
        wave_lds_sync();
        const int pre_me = incl - len;   // this cell-lane's first candidate in the batch
        L.start[lane] = s0 - pre_me;     // candidate v of cell r is particle start[r] + v
        wave_lds_sync();
        if (TRANSPOSED ? lane == tm : me) tested += total;
        // Candidates of the window [w0, w0 + 64), one per lane (-1 past the
        // batch's end), windows taken in order.  rw is the cell holding
        // candidate w0; the cells starting inside the window are flagged at
        // their offsets with the window's tag (unique in this walk, the
        // flags were cleared at its start), so a lane's cell is rw plus the
        // starts at or before it (non-empty cells start at distinct
        // candidates).
        int rw = 0;
        auto window = [&](int w0) {
            const int k = pre_me - w0;
            const int tag = wtag++;
            wave_lds_sync();
            if (len > 0 && k > 0 && k < 64) L.pre[k] = tag;
            wave_lds_sync();
            const uint64_t starts = __ballot(L.pre[lane] == tag);
            const int v = w0 + lane;
            int j = -1;
            if (v < total) j = L.start[rw + __popcll(starts & ((2ull << lane) - 1ull))] + v;
            rw += __popcll(starts) + (__ballot(len > 0 && k == 64) != 0 ? 1 : 0);
            return j;
        };
        // the next tile's (union) or chunk's (transposed) candidate stays in
        // flight while the current one is tested
        int jn = window(0);
        double xn = 0.0, yn = 0.0, zn = 0.0;
        if (jn >= 0) { xn = x[jn]; yn = y[jn]; zn = z[jn]; }
        for (int base = 0; base < total; base += 64) {
            if (TRANSPOSED) {
                const int j = jn;
                const double xc = xn, yc = yn, zc = zn;
                jn = window(base + 64);
                if (jn >= 0) { xn = x[jn]; yn = y[jn]; zn = z[jn]; }
                bool hin = false, hsh = false;
                double r2 = 0.0;
                if (j >= 0) {
                    r2 = wraps ? pair_r2<PM>(xm, ym, zm, xc, yc, zc, g)
                               : pair_r2<0>(xm, ym, zm, xc, yc, zc, g);
                    hin = r2 < T2m && j != (int)im;
                    hsh = !(r2 < A2m) && r2 < B2m;
                }
                const uint64_t bin = __ballot(hin);
                const int pos = Nm + __popcll(bin & below);
                if (hin && pos < K) idx[(int64_t)im * K + pos] = j;
                Nm += __popcll(bin);
                const uint64_t bsh = __ballot(hsh);
                const int c = __popcll(bsh);
                if (c > 0 && nshm >= 0) {
                    if (nshm + c <= SPH_SHELL_SLOTS) {
                        const int ps = nshm + __popcll(bsh & below);
                        if (hsh) {
                            SH.e[(int64_t)ps * SH.sstride + im] = shell_entry(j, r2);
                        }
                        nshm += c;
                    } else {
                        nshm = -1;
                    }
                }
            } else {
                if (jn >= 0) {
                    Cand cd;
                    cd.x = xn;
                    cd.y = yn;
                    cd.z = zn;
                    cd.j = jn;
                    cd.pad = 0;
                    L.c[lane] = cd;
                    if (G.ok) {
                        uint32_t f[8];
                        gram_cand(G, xn, yn, zn, f);
                        for (int k = 0; k < 8; ++k) L.cf[lane][k] = f[k];
                    }
                }
                wave_lds_sync();
                jn = window(base + 64);
                if (jn >= 0) { xn = x[jn]; yn = y[jn]; zn = z[jn]; }
                const int m = min(64, total - base);
                uint64_t gb = 0, ga = 0;
                if (G.ok) gram_tile(L, lane, gb, ga);   // all lanes (matrix cores)
                if (me) {
                    uint64_t hin, hsh;
                    if (G.ok) {
                        // certainly inner from the prefilter; the band and the
                        // shell by the exact r^2, shell members recorded here
                        // (in candidate order)
                        const uint64_t valid = m == 64 ? ~0ull : ((1ull << m) - 1ull);
                        hin = ga & valid;
                        hsh = 0;
                        uint64_t chk = gb & ~ga & valid;
                        while (chk) {
                            const int t = __ffsll((unsigned long long)chk) - 1;
                            chk &= chk - 1;
                            const double r2 = wraps ? tile_r2<PM>(L, t, xi, yi, zi, g)
                                                    : tile_r2<0>(L, t, xi, yi, zi, g);
                            if (r2 < A2) {
                                hin |= 1ull << t;
                            } else if (r2 < B2) {
                                if (r2 < T2) hin |= 1ull << t;
                                if (nsh >= 0 && nsh < SPH_SHELL_SLOTS) {
                                    SH.e[(int64_t)nsh * SH.sstride + i] = shell_entry(L.c[t].j, r2);
                                    ++nsh;
                                } else {
                                    nsh = -1;
                                }
                            }
                        }
                    } else if (m == 64) {
                        if (wraps) tile_hits<PM, true>(L, m, xi, yi, zi, A2, B2, g, &hin, &hsh);
                        else tile_hits<0, true>(L, m, xi, yi, zi, A2, B2, g, &hin, &hsh);
                    } else {
                        if (wraps) tile_hits<PM, false>(L, m, xi, yi, zi, A2, B2, g, &hin, &hsh);
                        else tile_hits<0, false>(L, m, xi, yi, zi, A2, B2, g, &hin, &hsh);
                    }
                    // shell members with their exact r^2; those below T join
                    // the row
                    while (hsh) {
                        int t = __ffsll((unsigned long long)hsh) - 1;
                        hsh &= hsh - 1;
                        const double r2 = wraps ? tile_r2<PM>(L, t, xi, yi, zi, g)
                                                : tile_r2<0>(L, t, xi, yi, zi, g);
                        if (r2 < T2) hin |= 1ull << t;
                        if (nsh >= 0 && nsh < SPH_SHELL_SLOTS) {
                            SH.e[(int64_t)nsh * SH.sstride + i] = shell_entry(L.c[t].j, r2);
                            ++nsh;
                        } else {
                            nsh = -1;
                        }
                    }
                    // the row's members in candidate order, skipping self;
                    // each hit's index is read from LDS one hit ahead, so
                    // that the read is in flight while the previous hit is
                    // stored
                    if (hin) {
                        int32_t *wq = wp + N;            // next entry of the row
                        int32_t *const wend = wp + K;    // (counted on past it)
                        int jj = L.c[__ffsll((unsigned long long)hin) - 1].j;
                        hin &= hin - 1;
                        for (;;) {
                            // (past the last hit: a read of slot 63, unused)
                            const bool more = hin != 0;
                            const int jn = L.c[(__ffsll((unsigned long long)hin) - 1) & 63].j;
                            hin &= hin - 1;
                            if (jj != (int)i) {
                                if (wq < wend) *wq = jj;
                                ++wq;
                            }
                            if (!more) break;
                            jj = jn;
                        }
                        N = (int)(wq - wp);
                    }
                }
                wave_lds_sync();
            }
        }
    };

    int qn = 0;   // cells waiting in the queue
    // (more than 64 blocks cannot occur; they would still be covered, 64 at
    // a time)
    for (int cb = 0; cb < nblk; cb += 64) {
        const int nb = min(64, nblk - cb);
        uint32_t bcode = 0xFFFFFFFFu;
        if (lane < nb) {
            const int k = cb + lane;
            const int kx = k % nbd[0];
            const int ky = (k / nbd[0]) % nbd[1];
            const int kz = k / (nbd[0] * nbd[1]);
            bcode = morton((uint32_t)((sb[0] + kx) & (NB - 1)), (uint32_t)((sb[1] + ky) & (NB - 1)),
                           (uint32_t)((sb[2] + kz) & (NB - 1)));
        }
        bcode = wave_sort_u32(bcode);
        for (int b = 0; b < nb; ++b) {
            const uint32_t bc = (uint32_t)__shfl((int)bcode, b, 64);
            int s0 = 0, len = 0;
            if (lane < nloc) {
                const uint32_t f[3] = {(compact3(bc) << kb) | lx, (compact3(bc >> 1) << kb) | ly,
                                       (compact3(bc >> 2) << kb) | lz};
                bool in = true;
                for (int d = 0; d < 3; ++d)
                    in = in && (int)(((int)f[d] - sa[d]) & msk) < cnt[d];
                if (in) {
                    const uint32_t code = (bc << (3 * kb)) | (uint32_t)lane;
                    s0 = S.cs[(int64_t)code << sh];
                    len = S.cs[((int64_t)code + 1) << sh] - s0;
                }
            }
            const uint64_t ne = __ballot(len > 0);
            const int pos = qn + __popcll(ne & below);
            wave_lds_sync();
            if (len > 0) {
                L.qs[pos] = s0;
                L.ql[pos] = len;
            }
            qn += __popcll(ne);
            wave_lds_sync();
            if (qn >= 64) {
                const int q0 = L.qs[lane], q1 = L.ql[lane];
                const int rest = qn - 64;
                const int r0 = lane < rest ? L.qs[64 + lane] : 0;
                const int r1 = lane < rest ? L.ql[64 + lane] : 0;
                wave_lds_sync();
                if (lane < rest) {
                    L.qs[lane] = r0;
                    L.ql[lane] = r1;
                }
                qn = rest;
                batch(q0, q1);
            }
        }
    }
    if (qn > 0) {
        wave_lds_sync();
        const int q0 = lane < qn ? L.qs[lane] : 0;
        const int q1 = lane < qn ? L.ql[lane] : 0;
        batch(q0, q1);
    }
    if (TRANSPOSED && lane == tm) {
        N = Nm;
        nsh = nshm;
    }
}

// One wave-cooperative count for every lane with act set at its own hc:
// the gather set at hc (members with r^2 < T = (2 hc)^2) is written to row i
// of idx (at most K, ascending), shell members (A <= r^2 < B) to the shell
// arrays (at most SPH_SHELL_SLOTS; *nsh = -1 when more).  Returns the number
// of the row's members (self excluded); self is never a shell member.  With
// A = B = T there is no shell.  The output does not depend
// on which lanes are counted together.  Lanes are grouped by position and by
// hsplit (their h for that purpose); with DEFER, lanes that end up in
// a small group are not counted and get *deferred = true (their particles
// are better served one per wave).
template <int PM, bool DEFER>
__device__ int wave_count(WaveLds &L, bool act, int64_t i, double xi, double yi, double zi,
                          uint32_t ki, double hsplit, bool *deferred,
                          double A2, double B2, double T2, const double *__restrict__ x,
                          const double *__restrict__ y, const double *__restrict__ z,
                          int32_t *__restrict__ idx, int64_t stride, int K, const Shell &SH,
                          int *nsh_out, const Search &S, const Geo &g, int64_t &tested)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const double twoh = 2.0 * hsplit;
    *deferred = false;
    int N = 0, nsh = 0;
    int32_t *wp = idx + i * (int64_t)K;   // this particle's row of the gather sets
    uint64_t pending = __ballot(act);
    while (pending) {
        // sub-group: the pending lanes, split by search radius, then by
        // Morton prefix while their positions spread over more than
        // SPH_SPLIT_SPREAD search diameters (a group that straddles a large
        // Morton jump would otherwise scan the gap)
        uint64_t members = pending;
        for (int sp = 0; sp < 32; ++sp) {
            bool mem = (members >> lane) & 1ull;
            double Rm = wave_max_d(mem ? twoh : 0.0);
            double ext = 0.0;
            const double p3[3] = {xi, yi, zi};
            for (int d = 0; d < 3; ++d) {
                double a = wave_min_d(mem ? p3[d] : INFINITY);
                double b = wave_max_d(mem ? p3[d] : -INFINITY);
                ext = fmax(ext, b - a);
            }
            // lanes whose search radius exceeds SPH_SPLIT_H times the group's
            // smallest wait for a later group (one large-h particle would
            // size the box and its cells for every member)
            const double Rlo = wave_min_d(mem ? twoh : INFINITY);
            if (Rm > SPH_SPLIT_H * Rlo) {
                members &= __ballot(twoh <= SPH_SPLIT_H * Rlo);
                continue;
            }
            if (!(ext > SPH_SPLIT_SPREAD * Rm) || __popcll(members) <= SPH_SMALL_GROUP) break;
            uint32_t kmin = wave_min_u(mem ? ki : 0xFFFFFFFFu);
            uint32_t kmax = wave_max_u(mem ? ki : 0u);
            if (kmin == kmax) break;
            int hb = 31 - __clz(kmin ^ kmax);
            int leader = __ffsll((unsigned long long)members) - 1;
            uint32_t lk = (uint32_t)__shfl((int)ki, leader, 64);
            members &= __ballot(((ki ^ lk) >> hb) == 0u);
        }
        pending &= ~members;
        if (DEFER && __popcll(members) <= S.defer) {
            if ((members >> lane) & 1ull) *deferred = true;
        } else if (!DEFER && __popcll(members) <= SPH_SMALL_GROUP) {
            uint64_t rest = members;
            while (rest) {
                const int m = __ffsll((unsigned long long)rest) - 1;
                rest &= rest - 1;
                walk_group<PM, true>(L, 1ull << m, m, i, xi, yi, zi, A2, B2, T2, x, y, z, idx, stride,
                                     K, SH, S, g, N, nsh, wp, tested);
            }
        } else {
            walk_group<PM, false>(L, members, -1, i, xi, yi, zi, A2, B2, T2, x, y, z, idx, stride, K,
                                  SH, S, g, N, nsh, wp, tested);
        }
    }
    *nsh_out = nsh;
    return N;
}

// iteration state carried between rounds (structure of arrays)
struct HIter {
    double *next, *lo, *hi, *best_h, *last_h;
    int32_t *best_n, *itk, *bits;   // bits: 1 lower bracket, 2 upper bracket, 4 try pending,
                                    // bits 8..15: full walks taken (HS_WALK units)
};

struct HState {
    double next, lo, hi, best_h, last_h;
    int best_n, itk, bits;
};

__device__ __forceinline__ HState hs_load(const HIter &H, int64_t i)
{
    HState s;
    s.next = H.next[i]; s.lo = H.lo[i]; s.hi = H.hi[i];
    s.best_h = H.best_h[i]; s.last_h = H.last_h[i];
    s.best_n = H.best_n[i]; s.itk = H.itk[i]; s.bits = H.bits[i];
    return s;
}

__device__ __forceinline__ void hs_store(const HIter &H, int64_t i, const HState &s)
{
    H.next[i] = s.next; H.lo[i] = s.lo; H.hi[i] = s.hi;
    H.best_h[i] = s.best_h; H.last_h[i] = s.last_h;
    H.best_n[i] = s.best_n; H.itk[i] = s.itk; H.bits[i] = s.bits;
}

#define HS_WALK 256        // one full walk in the bits field
// Large runs (n >= SPH_BIG_N) count round 0 without a shell and give the
// particles that need another count one wave-cooperative worklist round,
// with the shell, before the per-particle tail: recording a shell for every
// particle costs more than the worklist round for the few percent that
// iterate (64M patch, plain: 170 against 194 ms per step).  Smaller runs
// record the shell in round 0 and send only the rest to the tail: their
// worklist would be too short to fill the GPU (1M patch 3.95 against 4.52
// ms, 1M clumpy mixture 6.29 against 7.21 ms).  sph_params.walk_strategy
// can force either.
#ifndef SPH_BIG_N
#define SPH_BIG_N 4000000
#endif

// one step of the iteration after a count N at hc.
// returns 0 = count again at s.next, 1 = converged, 2 = stopped unconverged
__device__ __forceinline__ int h_update(HState &s, double hc, int N, double h_prev, int target,
                                        int tol, int maxit, const double *__restrict__ hk,
                                        uint8_t &fl, int64_t &acc, int64_t &fallback)
{
#pragma clang fp contract(off)
    s.last_h = hc;
    int dev = N > target ? N - target : target - N;
    if (s.bits & 4) {   // the learned try
        s.bits &= ~4;
        if (dev <= tol) {
            s.best_h = hc;
            s.best_n = N;
            fl = SPH_FLAG_LEARNED;
            ++acc;
            return 1;
        }
        ++fallback;
        s.next = h_prev;
        return 0;
    }
    int bdev = s.best_n > target ? s.best_n - target : target - s.best_n;
    if (s.best_n < 0 || dev < bdev || (dev == bdev && hc < s.best_h)) {
        s.best_h = hc;
        s.best_n = N;
    }
    if (dev <= tol) return 1;
    if (N < target - tol) {
        if (!(s.bits & 1) || hc > s.lo) s.lo = hc;
        s.bits |= 1;
    } else {
        if (!(s.bits & 2) || hc < s.hi) s.hi = hc;
        s.bits |= 2;
    }
    ++s.itk;
    if (s.itk >= maxit) return 2;
    if ((s.bits & 3) == 3) s.next = 0.5 * (s.lo + s.hi);
    else s.next = hc * hk[N < 1023 ? N : 1023];
    return 0;
}

// final values of a finished particle
__device__ __forceinline__ void h_finish(const HState &s, int res, uint8_t fl, int64_t i,
                                         double *__restrict__ h, int32_t *__restrict__ nc,
                                         uint8_t *__restrict__ flags, uint8_t *__restrict__ refill,
                                         int K, int64_t &nonconv, int64_t &overflow)
{
    if (res != 1) { fl |= SPH_FLAG_NOCONV; ++nonconv; }
    h[i] = s.best_h;
    nc[i] = s.best_n;
    flags[i] = fl;
    bool again = s.best_h != s.last_h;
    refill[i] = again ? 1 : 0;
    if (!again && s.best_n > K) ++overflow;
}

struct HArgs {
    const double *x, *y, *z;
    const uint32_t *key;
    double *h;
    const double *h_try;
    int32_t *nc;
    uint8_t *flags;
    uint8_t *refill;
    int32_t *work;
    int32_t *idx;
    int64_t stride;
    int K;
    const int32_t *cs;
    const double *bbox;
    const double *hk;
    Geo g;
    int lmax, div, prefilter, defer, target, tol, maxit;
    int first_shell;   // round 0 records the shell of its count (plain counts)
    int rounds;        // wave-cooperative worklist rounds after round 0
    int try_shell;     // the learned try's shell: 0 none, 2 always, 1 when lstep[2] is set
    int64_t *lstep;    // accepted and missed tries of this solve; [2]: the next try's shell
    HIter H;
    Shell SH;
    int64_t *status;
};

// After a walk at hc that wrote the gather set at hc (nrow members, r^2 <
// T = (2 hc)^2) to row i and the nsh shell members (A <= r^2 < B; -1 when
// they overflowed) to the shell arrays: one iteration step at hc, then more
// while the next h stays inside the shell, all counted exactly from the
// shell.  Returns the h_update result; 0 leaves st.next for the next full
// count (hc itself after an overflow).  When the iteration ends on an h
// inside this shell other than hc, the writer adjusts the row to that h's
// gather set (shell members merged in or taken out, the row stays
// ascending); a kept h outside the shell sets st.last_h = -1, marking the
// row for rewriting.
__device__ int shell_iterate(const HArgs &A, int64_t i, HState &st, double hc, double hprev,
                             int nrow, int nsh, double A2, double B2, bool writer, uint8_t &fl,
                             int64_t &counts, int64_t &acc, int64_t &fallback)
{
#pragma clang fp contract(off)
    if (nsh < 0) {
        st.next = hc;   // shell overflow: the exact count needs a full walk
        return 0;
    }
    const int64_t ss = A.SH.sstride;
    const int2 *se = A.SH.e + i;   // shell member k at se[k * ss]
    const double t0 = 2.0 * hc;
    const double T2 = t0 * t0;
    // r^2 of shell member e below T (exact: see Shell)
    auto below = [&](int2 e, double T) {
        const double f = (double)__int_as_float(e.y);
        if (f < T * (1.0 - 0x1p-22)) return true;
        if (f > T * (1.0 + 0x1p-22)) return false;
        const int64_t j = e.x;
        double d[3] = {A.x[j] - A.x[i], A.y[j] - A.y[i], A.z[j] - A.z[i]};
        for (int a = 0; a < 3; ++a) {
            if (A.g.per[a]) {
                const double up = d[a] - A.g.L[a], dn = d[a] + A.g.L[a];
                d[a] = (d[a] > A.g.halfL[a]) ? up : ((d[a] < -A.g.halfL[a]) ? dn : d[a]);
            }
        }
        return exact_r2(d[0], d[1], d[2]) < T;
    };
    // bit k: shell member k has r^2 < T; members read SPH_SHELL_BATCH at a
    // time so that their loads are in flight together (padding reads as
    // r^2 = +inf)
    auto mask_below = [&](double T) {
        uint64_t m = 0;
        for (int k0 = 0; k0 < nsh; k0 += SPH_SHELL_BATCH) {
            int2 e[SPH_SHELL_BATCH];
#pragma unroll
            for (int u = 0; u < SPH_SHELL_BATCH; ++u)
                e[u] = k0 + u < nsh ? se[(int64_t)(k0 + u) * ss] : make_int2(0, 0x7f800000);
#pragma unroll
            for (int u = 0; u < SPH_SHELL_BATCH; ++u)
                m |= (uint64_t)(below(e[u], T) ? 1 : 0) << (k0 + u);
        }
        return m;
    };
    // members below T (in the row), read from the shell only when the
    // iteration goes on past hc
    uint64_t mT = 0;
    bool have_mT = false;
    auto shell_count = [&](double r2m) {
        if (!have_mT) {
            mT = mask_below(T2);
            have_mT = true;
        }
        return nrow - __popcll(mT) + __popcll(mask_below(r2m));
    };
    auto in_shell = [&](double r2m) { return r2m >= A2 && r2m <= B2; };
    ++counts;
    int res = h_update(st, hc, nrow, hprev, A.target, A.tol, A.maxit, A.hk, fl, acc, fallback);
    while (res == 0) {
        const double tn = 2.0 * st.next;
        const double r2n = tn * tn;
        if (!in_shell(r2n)) break;
        const double hn = st.next;
        ++counts;
        res = h_update(st, hn, shell_count(r2n), hprev, A.target, A.tol, A.maxit, A.hk, fl, acc,
                       fallback);
    }
    if (res != 0) {
        const double tk = 2.0 * st.best_h;
        const double r2k = tk * tk;
        if (in_shell(r2k) && (r2k == T2 ? st.best_n == nrow : st.best_n == shell_count(r2k))) {
            st.last_h = st.best_h;
            if (r2k != T2 && (nrow > A.K || st.best_n > A.K)) {
                // the row does not hold the gather set at hc whole: rewrite it
                if (st.best_n <= A.K) st.last_h = -1.0;
            } else if (writer && r2k != T2) {
                // the row reads four entries ahead of its cursor q (in
                // flight together); every write lands at or behind q
                int32_t *row = A.idx + i * (int64_t)A.K;
                const int dq = r2k > T2 ? -1 : 1;
                int q = r2k > T2 ? nrow - 1 : 0;
                auto rd = [&](int p) { return (p >= 0 && p < nrow) ? row[p] : 0; };
                int32_t w0 = rd(q), w1 = rd(q + dq), w2 = rd(q + 2 * dq), w3 = rd(q + 3 * dq);
                auto advance = [&]() {
                    q += dq;
                    w0 = w1;
                    w1 = w2;
                    w2 = w3;
                    w3 = rd(q + 3 * dq);
                };
                if (r2k > T2) {
                    // shell members with T <= r^2 < (2h)^2 join the row: merge
                    // from the back, in place (both runs ascending, disjoint);
                    // joins in descending k, i.e. descending index
                    uint64_t rest = mask_below(r2k) & ~mT;
                    int t = __popcll(rest);
                    int32_t sj = 0, sn = 0;
                    if (t > 0) {
                        const int k = 63 - __clzll(rest);
                        rest &= ~(1ull << k);
                        sj = se[(int64_t)k * ss].x;
                        if (rest) sn = se[(int64_t)(63 - __clzll(rest)) * ss].x;
                    }
                    while (t > 0) {
                        if (q >= 0 && w0 > sj) {
                            row[q + t] = w0;
                            advance();
                        } else {
                            row[q + t] = sj;
                            if (--t > 0) {
                                rest &= ~(1ull << (63 - __clzll(rest)));
                                sj = sn;
                                if (rest) sn = se[(int64_t)(63 - __clzll(rest)) * ss].x;
                            }
                        }
                    }
                } else {
                    // shell members with (2h)^2 <= r^2 < T leave the row
                    uint64_t rest = mT & ~mask_below(r2k);
                    int32_t sj = -1, sn = -1;
                    if (rest) {
                        const int k = __ffsll((unsigned long long)rest) - 1;
                        rest &= rest - 1;
                        sj = se[(int64_t)k * ss].x;
                        if (rest) sn = se[(int64_t)(__ffsll((unsigned long long)rest) - 1) * ss].x;
                    }
                    int o = 0;
                    while (q < nrow) {
                        const int32_t v = w0;
                        advance();
                        if (v == sj) {
                            sj = sn;
                            if (rest) {
                                rest &= rest - 1;
                                sn = rest ? se[(int64_t)(__ffsll((unsigned long long)rest) - 1) * ss].x
                                          : -1;
                            }
                            continue;
                        }
                        row[o++] = v;
                    }
                }
            }
        } else {
            st.last_h = -1.0;   // the kept h lies outside this shell: rewrite its set
        }
    }
    return res;
}

#ifndef SPH_ROUND_WAVES
#define SPH_ROUND_WAVES 4   // waves per SIMD the round kernel is compiled for (measured best)
#endif
// Round 0 (wl == nullptr: every particle, grouped by index) and later rounds
// (the worklist wl of wcount particles).  After its count a particle keeps
// iterating on its shell while the next h stays inside it; particles that
// need another full count save their state and raise work[i].
template <int PM, bool FIRST>
__global__ __launch_bounds__(SPH_BLOCK)
__attribute__((amdgpu_waves_per_eu(SPH_ROUND_WAVES, SPH_ROUND_WAVES))) void k_hsolve_round(HArgs A, int64_t n,
                                                            const int32_t *__restrict__ wl,
                                                            const int64_t *__restrict__ wcount)
{
#pragma clang fp contract(off)
    __shared__ WaveLds lds[WAVES_PER_BLOCK];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // a compacted worklist occupies the first blocks only: deal those to the
    // XCDs round-robin (plain block order) instead of in contiguous ranges
    const int64_t blk = wl ? (int64_t)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
    const int64_t grp = blk * WAVES_PER_BLOCK + w;
    const int64_t slot = grp * 64 + lane;
    const int64_t total = wl ? *wcount : n;
    // few learned misses: all of them to the tail
    if (wl && A.h_try && total < SPH_LEARNED_ROUND_MIN && total * 10 < n) return;
    const bool listed = slot < total;
    const int64_t i = listed ? (wl ? (int64_t)wl[slot] : slot) : 0;
    // each particle takes at most A.rounds + 1 full walks in these
    // rounds (a learned try that is left behind does not count); one that
    // has used them waits, still listed, for the per-particle tail
    const bool valid = listed && (!wl || (A.H.bits[i] >> 8) < A.rounds + 1);
    const Search S = make_search(A.cs, A.lmax, A.div, A.prefilter, A.defer, A.bbox, A.g);

    // only what the walk needs is live across it; the iteration state is
    // set up (round 0) or loaded (later rounds) afterwards
    double hc = 0.0, hsplit = 0.0;
    if (valid) {
        if (FIRST) {
            hsplit = A.h[i];
            hc = A.h_try ? A.h_try[i] : hsplit;
        } else {
            hc = A.H.next[i];
            hsplit = hc;
        }
    }
    int64_t tested = 0, counts = 0, acc = 0, fallback = 0, nonconv = 0, overflow = 0;
    // The learned try, accepted almost always, is counted without a shell
    // (SPH_TRY_SHELL_D): a miss restarts the plain iteration from h_prev,
    // with its shell, in the worklist round (or, when misses are few, the
    // tail: SPH_LEARNED_ROUND_MIN).  Plain
    // counts of small runs record the shell, on which most misses of h_prev
    // converge (SPH_BIG_N).
    const bool try_walk = FIRST && A.h_try != nullptr;
    const bool try_shell = try_walk && (A.try_shell == 2 || (A.try_shell == 1 && A.lstep[2] != 0));
    const double sd = try_walk ? (try_shell ? SPH_SHELL_D : SPH_TRY_SHELL_D)
                               : ((FIRST && !A.first_shell) ? SPH_WL_SHELL_D : SPH_SHELL_D);
    const double ta = sd > 0.0 ? 2.0 * hc * (1.0 - 1.0 / sd) : 2.0 * hc;
    const double tb = sd > 0.0 ? 2.0 * hc * (1.0 + 1.0 / sd) : 2.0 * hc;
    const double tt = 2.0 * hc;
    const double A2 = ta * ta, B2 = tb * tb, T2 = tt * tt;
    int nin = 0, nsh = 0;
    bool deferred = false;
    // a wave whose slots are all past the end has nothing to do.  Round 0
    // groups by h_prev (the same groups with or without a learned try) and
    // leaves particles of small groups to the per-particle tail.
    if (__ballot(valid)) {
        double xi = 0.0, yi = 0.0, zi = 0.0;
        uint32_t ki = 0;
        if (valid) {
            xi = A.x[i]; yi = A.y[i]; zi = A.z[i];
            ki = A.key[i];
        }
        nin = wave_count<PM, FIRST>(lds[w], valid, i, xi, yi, zi, ki, hsplit, &deferred, A2, B2,
                                    T2, A.x, A.y, A.z, A.idx, A.stride, A.K, A.SH, &nsh, S, A.g,
                                    tested);
    }
    double hprev = 0.0;
    HState st = {};
    if (valid) {
        hprev = A.h[i];
        if (!FIRST) {
            st = hs_load(A.H, i);
        } else {
            st.next = hc;
            st.lo = st.hi = 0.0;
            st.best_h = st.last_h = hprev;
            st.best_n = -1;
            st.itk = 0;
            st.bits = A.h_try ? 4 : 0;
        }
    }
    if (valid && deferred) {
        // no walk taken: untouched state, walk budget spent so that only
        // the tail takes it up (with full counts)
        st.bits |= (A.rounds + 1) * HS_WALK;
        hs_store(A.H, i, st);
        A.work[i] = 1;
    } else if (valid) {
        uint8_t fl = 0;
        int res;
        st.bits += HS_WALK;
        const double tp = 2.0 * hprev;
        const double tp2 = tp * tp;
        if (FIRST && A.h_try && (nsh < 0 || !(tp2 >= A2 && tp2 <= B2))) {
            // the try pass, for a particle whose plain start h_prev lies
            // outside the try's shell (or whose count is unknown because the
            // shell overflowed): accept the predicted h when in band,
            // otherwise the plain iteration starts from h_prev in the tail,
            // with the plain start's state (no walk taken yet)
            if (nsh >= 0) {
                res = shell_iterate(A, i, st, hc, hprev, nin, nsh, A2, B2, true, fl, counts, acc,
                                    fallback);
            } else {
                ++counts;
                ++fallback;
                res = 0;
            }
            if (res == 0) {
                st.next = hprev;
                st.lo = st.hi = 0.0;
                st.best_h = st.last_h = hprev;
                st.best_n = -1;
                st.itk = 0;
                st.bits = 0;
            }
        } else {
            res = shell_iterate(A, i, st, hc, hprev, nin, nsh, A2, B2, true, fl, counts, acc,
                                fallback);
        }
        if (res == 0) {
            hs_store(A.H, i, st);
            A.work[i] = 1;
        } else {
            h_finish(st, res, fl, i, A.h, A.nc, A.flags, A.refill, A.K, nonconv, overflow);
            A.work[i] = 0;
        }
    }
    block_add_i64(counts, A.status + ST_HCOUNTS);
    block_add_i64(tested, A.status + ST_CANDIDATES);
    if (!wl) block_add_i64(tested, A.status + ST_CANDIDATES_FIRST);
    block_add_i64(nonconv, A.status + ST_NONCONV);
    block_add_i64(overflow, A.status + ST_LIST_OVERFLOW);
    if (A.h_try) {
        block_add2_i64(acc, A.status + ST_LEARN_ACC, A.lstep);
        block_add2_i64(fallback, A.status + ST_LEARN_FALLBACK, A.lstep + 1);
    }
}

// worklist: wl[woff[i]] = i for flagged particles (index order kept)
__global__ __launch_bounds__(SPH_BLOCK) void k_compact(int64_t n, const int32_t *__restrict__ work,
                                                       const int64_t *__restrict__ woff,
                                                       int32_t *__restrict__ wl)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && work[i]) wl[woff[i]] = (int32_t)i;
}

// The particles still iterating after the wave rounds: one wave each,
// iterating to the end with full wave-cooperative counts (the whole gather
// set written at every count, no shell).
template <int PM>
// waves per SIMD the tail kernel is compiled for (4 against 2: 64M patch,
// learned form, 152 against 156 ms per step; the plain form is indifferent)
#ifndef SPH_TAIL_WAVES
#define SPH_TAIL_WAVES 4
#endif
__global__ __launch_bounds__(SPH_BLOCK)
__attribute__((amdgpu_waves_per_eu(SPH_TAIL_WAVES, SPH_TAIL_WAVES))) void k_hsolve_tail(HArgs A, const int32_t *__restrict__ wl,
                                                           const int64_t *__restrict__ wcount)
{
#pragma clang fp contract(off)
    __shared__ WaveLds lds[WAVES_PER_BLOCK];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * WAVES_PER_BLOCK + w;
    const int64_t nw = (int64_t)gridDim.x * WAVES_PER_BLOCK;
    const int64_t total = *wcount;
    const Search S = make_search(A.cs, A.lmax, A.div, A.prefilter, A.defer, A.bbox, A.g);
    int64_t counts = 0, tested = 0, nonconv = 0, overflow = 0, acc = 0, fallback = 0;
    for (int64_t t = gw; t < total; t += nw) {
        const int64_t i = wl[t];
        const double xi = A.x[i], yi = A.y[i], zi = A.z[i];
        const uint32_t ki = A.key[i];
        const double hprev = A.h[i];
        HState st = hs_load(A.H, i);
        uint8_t fl = 0;
        int res = 0;
        // a particle that has not been walked yet (a learned miss restarted
        // from h_prev) gets the plain solve's first walk: with a shell and
        // the iteration on it, so that it follows the plain path
        bool shell_walk = (st.bits >> 8) == 0;
        while (res == 0) {
            const double hc = st.next;
            int nsh = 0;
            bool dfr;
            if (shell_walk) {
                shell_walk = false;
                const double ta = 2.0 * hc * (1.0 - 1.0 / SPH_SHELL_D), tb = 2.0 * hc * (1.0 + 1.0 / SPH_SHELL_D);
                const double tt = 2.0 * hc;
                const double A2 = ta * ta, B2 = tb * tb, T2 = tt * tt;
                int nin = wave_count<PM, false>(lds[w], lane == 0, i, xi, yi, zi, ki, hc, &dfr, A2,
                                                B2, T2, A.x, A.y, A.z, A.idx, A.stride, A.K, A.SH,
                                                &nsh, S, A.g, tested);
                nin = __shfl(nin, 0, 64);
                nsh = __shfl(nsh, 0, 64);
                // the shell arrays were written by other lanes: make them visible
                __threadfence_block();
                res = shell_iterate(A, i, st, hc, hprev, nin, nsh, A2, B2, lane == 0, fl, counts,
                                    acc, fallback);
                continue;
            }
            const double t2 = 2.0 * hc;
            const double r2m = t2 * t2;
            int N = wave_count<PM, false>(lds[w], lane == 0, i, xi, yi, zi, ki, hc, &dfr, r2m, r2m,
                                   r2m, A.x, A.y, A.z, A.idx, A.stride, A.K, A.SH, &nsh, S, A.g,
                                   tested);
            N = __shfl(N, 0, 64);
            ++counts;
            res = h_update(st, hc, N, hprev, A.target, A.tol, A.maxit, A.hk, fl, acc, fallback);
        }
        if (lane == 0) h_finish(st, res, fl, i, A.h, A.nc, A.flags, A.refill, A.K, nonconv, overflow);
    }
    // state and counters are wave-uniform: lane 0 reports them
    const bool rep = lane == 0;
    block_add_i64(rep ? counts : 0, A.status + ST_HCOUNTS);
    block_add_i64(tested, A.status + ST_CANDIDATES);
    block_add_i64(rep ? nonconv : 0, A.status + ST_NONCONV);
    block_add_i64(rep ? overflow : 0, A.status + ST_LIST_OVERFLOW);
    if (A.h_try) {
        block_add2_i64(rep ? acc : 0, A.status + ST_LEARN_ACC, A.lstep);
        block_add2_i64(rep ? fallback : 0, A.status + ST_LEARN_FALLBACK, A.lstep + 1);
    }
}

// rewrite the gather set of particles whose kept h is not the last counted
// one (wave-cooperative, the whole set at the kept h)
template <int PM>
__global__ __launch_bounds__(SPH_BLOCK) void k_refill(HArgs A, int64_t n)
{
#pragma clang fp contract(off)
    __shared__ WaveLds lds[WAVES_PER_BLOCK];
    const int w = threadIdx.x >> 6;
    const int64_t i = global_index();
    int64_t overflow = 0, tested = 0;
    if (A.h_try && i == 0) {
        // the solve's tries are all counted (round 0, worklist round, tail):
        // the next try records a shell when more than a tenth missed
        const int64_t ac = A.lstep[0], mi = A.lstep[1];
        A.lstep[2] = mi * 10 > ac + mi ? 1 : 0;
        A.lstep[0] = 0;
        A.lstep[1] = 0;
    }
    const bool act = i < n && A.refill[i];
    if (__ballot(act)) {
        const Search S = make_search(A.cs, A.lmax, A.div, A.prefilter, A.defer, A.bbox, A.g);
        double xi = 0.0, yi = 0.0, zi = 0.0, hi = 0.0;
        uint32_t ki = 0;
        if (i < n) {
            xi = A.x[i]; yi = A.y[i]; zi = A.z[i];
            hi = A.h[i];
            ki = A.key[i];
        }
        const double t2 = 2.0 * hi;
        const double r2m = t2 * t2;
        int nsh = 0;
        bool dfr;
        int N = wave_count<PM, false>(lds[w], act, i, xi, yi, zi, ki, hi, &dfr, r2m, r2m, r2m, A.x,
                               A.y, A.z, A.idx, A.stride, A.K, A.SH, &nsh, S, A.g, tested);
        if (act && N > A.K) ++overflow;
    }
    block_add_i64(overflow, A.status + ST_LIST_OVERFLOW);
}

// phase 0: round 0 alone; phase 1: the worklist round, tail and refill
hipError_t launch_hsolve(sph_ctx *c, sph_particles *s, sph_nlist *nl, const double *h_try,
                         int phase)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    const sph_params &p = c->p;
    int cur = s->cur;
    unsigned nb = (unsigned)ceil_div(n, SPH_BLOCK);
    Geo g = make_geo(p);
    HArgs A;
    A.x = s->x[cur]; A.y = s->y[cur]; A.z = s->z[cur];
    A.key = s->key;
    A.h = s->h[cur];
    A.h_try = h_try;
    A.nc = s->nc[cur];
    A.flags = s->flags;
    A.refill = c->w.refill;
    A.work = c->w.work;
    A.idx = nl->idx;
    A.stride = nl->stride;
    A.K = p.list_stride;
    A.cs = c->w.cell_start;
    A.bbox = c->w.bbox;
    A.hk = c->w.hk;
    A.g = g;
    A.lmax = p.max_level;
    A.div = p.search_div;
    A.prefilter = p.walk_prefilter;
    A.defer = p.walk_defer_group > 0 ? p.walk_defer_group : SPH_DEFER_GROUP;
    const bool worklist = p.walk_strategy == SPH_WALK_WORKLIST ||
                          (p.walk_strategy == SPH_WALK_AUTO && n >= SPH_BIG_N);
    A.first_shell = worklist ? 0 : 1;
    A.rounds = (worklist || h_try) ? 1 : 0;
    A.try_shell = p.learned_try_shell == SPH_TRY_SHELL_ALWAYS ? 2
                : (p.learned_try_shell == SPH_TRY_SHELL_AUTO && !worklist &&
                   n >= SPH_TRY_SHELL_MIN_N) ? 1 : 0;
    A.lstep = c->w.learn_step;
    A.target = p.n_target;
    A.tol = p.n_tol;
    A.maxit = p.h_max_iter;
    A.H = {c->w.hs_next, c->w.hs_lo, c->w.hs_hi, c->w.hs_best_h, c->w.hs_last_h,
           c->w.hs_best_n, c->w.hs_itk, c->w.hs_bits};
    A.SH = {c->w.shell_e, c->w.shell_stride};
    A.status = c->w.status;
    const int pm = periodic_mask(g);
    if (phase == 0) {
        SPH_DISPATCH_PM(pm,
            hipLaunchKernelGGL((k_hsolve_round<PM, true>), dim3(nb), dim3(SPH_BLOCK), 0, c->stream, A,
                               n, (const int32_t *)nullptr, (const int64_t *)nullptr))
        return hipGetLastError();
    }
    const int rounds = A.rounds;
    for (int r = 0; r <= rounds; ++r) {
        hipError_t e = launch_scan_i32_to_i64(c, c->w.work, c->w.woff, n);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_compact, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, c->w.work,
                           c->w.woff, c->w.wl);
        if (r < rounds) {
            // the worklist size is only known on the device: launch for all
            // and let waves past its end return at once
            SPH_DISPATCH_PM(pm,
                hipLaunchKernelGGL((k_hsolve_round<PM, false>), dim3(nb), dim3(SPH_BLOCK), 0, c->stream,
                                   A, n, c->w.wl, c->w.woff + n))
        } else {
            SPH_DISPATCH_PM(pm,
                hipLaunchKernelGGL(k_hsolve_tail<PM>, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, A,
                                   c->w.wl, c->w.woff + n))
        }
    }
    SPH_DISPATCH_PM(pm,
        hipLaunchKernelGGL(k_refill<PM>, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, A, n))
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
            int j = idx[(int64_t)i * K + k];
            double dx = mimg<PM, 0>(xi, x[j], g);
            double dy = mimg<PM, 1>(yi, y[j], g);
            double dz = mimg<PM, 2>(zi, z[j], g);
            double r2 = exact_r2(dx, dy, dz);
            double twoh = 2.0 * h[j];
            if (!(r2 < twoh * twoh)) extra_append(j, (int)i, ecnt, eidx, slots, appended, dropped);
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

// ---------------------------------------------------------------------------
// The interaction sets as CSR, S_i = L_i U E_i with ascending rows, exported
// from the padded rows: row sizes, their exclusive scan, then every row
// merged by ranking.  L_i is ascending and E_i unordered; the two are
// disjoint, so an entry's place in S_i is the number of entries of both
// below it (a binary search in L_i, a count over the short E_i).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_csr_sizes(int64_t n, const int32_t *__restrict__ nc,
                                                         int K, const int32_t *__restrict__ ecnt,
                                                         int slots, int32_t *__restrict__ sz)
{
    const int64_t i = global_index();
    if (i < n) sz[i] = min(nc[i], K) + min(ecnt[i], slots);
}

__global__ __launch_bounds__(SPH_BLOCK) void k_csr_fill(
    int64_t n, const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K,
    const int32_t *__restrict__ ecnt, const int32_t *__restrict__ eidx, int slots,
    const int64_t *__restrict__ off, int32_t *__restrict__ out, int64_t cap,
    int64_t *__restrict__ status)
{
    const int64_t i = global_index();
    int64_t dropped = 0;
    if (i < n) {
        const int nl = min(nc[i], K), ne = min(ecnt[i], slots);
        const int32_t *L = idx + i * (int64_t)K;
        const int32_t *E = eidx + i * (int64_t)slots;
        const int64_t o = off[i];
        for (int k = 0; k < nl; ++k) {
            const int32_t v = L[k];
            int r = k;
            for (int e = 0; e < ne; ++e) r += E[e] < v ? 1 : 0;
            if (o + r < cap) out[o + r] = v;
            else ++dropped;
        }
        for (int e = 0; e < ne; ++e) {
            const int32_t v = E[e];
            int r = 0;
            for (int f = 0; f < ne; ++f) r += E[f] < v ? 1 : 0;
            int a = 0, b = nl;   // entries of L below v: the first index with L[a] > v
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (L[mid] < v) a = mid + 1;
                else b = mid;
            }
            r += a;
            if (o + r < cap) out[o + r] = v;
            else ++dropped;
        }
    }
    block_add_i64(dropped, status + ST_CSR_OVERFLOW);
}

hipError_t launch_interaction_csr(sph_ctx *c, const sph_particles *s, const sph_nlist *nl,
                                  int64_t *off, int32_t *out, int64_t cap)
{
    const int64_t n = s->n;
    const sph_params &p = c->p;
    const int cur = s->cur;
    const unsigned nb = (unsigned)ceil_div(n > 0 ? n : 1, SPH_BLOCK);
    if (n > 0)
        hipLaunchKernelGGL(k_csr_sizes, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->nc[cur],
                           p.list_stride, nl->ecnt, p.extra_slots, c->w.work);
    hipError_t e = launch_scan_i32_to_i64(c, c->w.work, off, n);
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(k_csr_fill, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, s->nc[cur],
                       nl->idx, p.list_stride, nl->ecnt, nl->eidx, p.extra_slots, off, out, cap,
                       c->w.status);
    return hipGetLastError();
}
