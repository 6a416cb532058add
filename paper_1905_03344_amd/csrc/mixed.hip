// Mixed-precision form of the density and force kernels: pair arithmetic in
// FP32 on cell-relative split coordinates, Neumaier-compensated FP32 sums,
// results stored in FP64.  Neighbour sets, counts and h come from the exact
// FP64 search; the one-sided complement test keeps its exact answer through
// an FP32 prefilter with an FP64 test for the ambiguous band.
#include "sph_internal.h"

// Per-particle FP32 fields, three float4 arrays (one 16-byte quad per
// particle each, so that a group of lanes reading consecutive particles
// touches consecutive memory; a pair costs three loads):
//   A = {delta_x, delta_y, delta_z, cell}   cell = gx | gy << 10 | gz << 20
//   B = {vx, vy, vz, m}
//   C = {h, c_sound, rho, P/rho^2}
// with x = lo + g * w + delta, w = L/1024 the key-cell width.  1/h of a
// neighbour is formed in the pair (hardware reciprocal, 1 ulp).
struct MixQ {
    float4 *A, *B, *C, *D;   // D: IAD (c_xx, c_xy, c_xz, c_yy); generalized volumes
                             // (X, X/m, 0, 0); else unused
};
__host__ __device__ static inline MixQ mix_quads(void *base, int64_t n_max)
{
    float4 *q = (float4 *)base;
    return MixQ{q, q + n_max, q + 2 * n_max, q + 3 * n_max};
}

// lanes per particle in the pair loops (8: measured best of 4, 8, 16, 32, 64),
// and their partial sums combined in a fixed butterfly order (Neumaier
// steps: the same value in every lane)
#ifndef SPH_MGROUP
#define SPH_MGROUP 8
#endif
// rounds per block of the mixed force kernel: a block takes
// SPH_MROUNDS_F * SPH_BLOCK / SPH_MGROUP consecutive particles (64M patch,
// ms per launch: 8 rounds 29.3, 4 rounds 29.6, 2 rounds 30.3; the FP64
// kernel, whose records are larger, prefers 2)
#ifndef SPH_MROUNDS_F
#define SPH_MROUNDS_F 8
#endif
#define SPH_MPTILE_F (SPH_MROUNDS_F * (SPH_BLOCK / SPH_MGROUP))
// pairs per lane per batch of the mixed density pass (64M patch, density
// stage: 3 pairs 30.3 ms, 4 pairs 29.1, 5 pairs 27.7 at 124 VGPRs; a lane
// takes the same pairs in the same order whatever the batch)
#ifndef SPH_MBATCH
#define SPH_MBATCH 5
#endif
#ifndef SPH_MFBATCH
#define SPH_MFBATCH 4
#endif
__device__ __forceinline__ float mgroup_max(float v)
{
    for (int o = SPH_MGROUP / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, SPH_MGROUP));
    return v;
}

struct MixGeo {
    float w[3];    // key-cell width per dimension
    int per[3];
};

// Neumaier (1974) compensated summation in FP32: the rounding error of each
// addition s + v is accumulated in c.  The error is formed by Knuth's
// branch-free TwoSum, exact whichever operand is larger (the same value as
// Neumaier's choice between (s - t) + v and (v - t) + s, in six operations
// instead of seven with the comparison and select)
struct NeuF {
    float s, c;
};
__device__ __forceinline__ void neu_add(NeuF &a, float v)
{
#pragma clang fp contract(off)
    const float t = a.s + v;
    const float vv = t - a.s;
    a.c += (a.s - (t - vv)) + (v - vv);
    a.s = t;
}
__device__ __forceinline__ double neu_val(const NeuF &a) { return (double)a.s + (double)a.c; }
__device__ __forceinline__ NeuF mgroup_neu(NeuF a)
{
    for (int o = SPH_MGROUP / 2; o > 0; o >>= 1) {
        const float os = __shfl_xor(a.s, o, SPH_MGROUP), oc = __shfl_xor(a.c, o, SPH_MGROUP);
        neu_add(a, os);
        a.c += oc;
    }
    return a;
}

__device__ __forceinline__ uint32_t cell_of(float4 a) { return __float_as_uint(a.w); }

// 1/sqrt(r^2) of a pair (r^2 > 0) by the hardware instruction (about 1 ulp),
// without the denormal rescaling of the library's rsqrtf: a nonzero FP32 r^2
// of split coordinates is at least (2^-24 w)^2 for the key-cell width w, a
// normal number for any box wider than about 2e-9 length units; below that
// the clamp keeps the result finite
__device__ __forceinline__ float rsq_pair(float r2)
{
    return __builtin_amdgcn_rsqf(fmaxf(r2, 1.17549435e-38f));
}

// offset x_j - x_i in dimension D from split coordinates (wrap on the
// integer cell difference in periodic dimensions)
template <int PM, int D>
__device__ __forceinline__ float split_diff(uint32_t gi, uint32_t gj, float di, float dj,
                                            const MixGeo &G)
{
    int ci = (int)((gi >> (10 * D)) & 1023u), cj = (int)((gj >> (10 * D)) & 1023u);
    int dg = cj - ci;
    if constexpr (((PM >> D) & 1) != 0) {
        dg = dg > 512 ? dg - 1024 : (dg < -512 ? dg + 1024 : dg);
    }
    return (float)dg * G.w[D] + (dj - di);
}

// kernel and derivative in FP32 (SPH_KERNEL_*; knorm = B_5 of the sinc kernel)
__device__ __forceinline__ float sinc_f(float x, float &deriv)
{
    // sin(x)/x and its derivative on 0 <= x <= pi: series in x^2 to x^18
    // (the next terms are below 2e-10 at x = pi)
    const float x2 = x * x;
    float d = -1.4797143443923793e-16f;
    d = d * x2 + 4.498331606952833e-14f;
    d = d * x2 + -1.0706029224547743e-11f;
    d = d * x2 + 1.9270852604185937e-09f;
    d = d * x2 + -2.505210838544172e-07f;
    d = d * x2 + 2.2045855379188714e-05f;
    d = d * x2 + -0.0011904761904761906f;
    d = d * x2 + 0.03333333333333333f;
    d = d * x2 + -0.3333333333333333f;
    deriv = d * x;
    float s = -8.22063524662433e-18f;
    s = s * x2 + 2.8114572543455206e-15f;
    s = s * x2 + -7.647163731819816e-13f;
    s = s * x2 + 1.6059043836821613e-10f;
    s = s * x2 + -2.505210838544172e-08f;
    s = s * x2 + 2.7557319223985893e-06f;
    s = s * x2 + -0.0001984126984126984f;
    s = s * x2 + 0.008333333333333333f;
    s = s * x2 + -0.16666666666666666f;
    s = s * x2 + 1.0f;
    return s;
}
template <int KER>
__device__ __forceinline__ float kern_w_f(float r, float inv_h, float knorm)
{
    const float q = r * inv_h;
    const float ih3 = inv_h * inv_h * inv_h;
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        if (!(q < 2.0f)) return 0.0f;
        const float t = 1.0f - 0.5f * q, t2 = t * t;
        return (float)(21.0 / (16.0 * SPH_PI)) * ih3 * (t2 * t2) * (2.0f * q + 1.0f);
    } else if constexpr (KER == SPH_KERNEL_SINC5) {
        if (!(q < 2.0f)) return 0.0f;
        float d;
        const float s = sinc_f((float)(0.5 * SPH_PI) * q, d), s2 = s * s;
        return knorm * ih3 * (s2 * s2 * s);
    } else {
        float w;
        if (q < 1.0f) w = 1.0f - 1.5f * q * q + 0.75f * q * q * q;
        else if (q < 2.0f) { float t = 2.0f - q; w = 0.25f * t * t * t; }
        else w = 0.0f;
        return (float)(1.0 / SPH_PI) * ih3 * w;
    }
}
template <int KER>
__device__ __forceinline__ float kern_dwdr_f(float r, float inv_h, float knorm)
{
    const float q = r * inv_h;
    const float ih2 = inv_h * inv_h;
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        if (!(q < 2.0f)) return 0.0f;
        const float t = 1.0f - 0.5f * q;
        return (float)(21.0 / (16.0 * SPH_PI)) * (ih2 * ih2) * (-5.0f * q) * (t * t * t);
    } else if constexpr (KER == SPH_KERNEL_SINC5) {
        if (!(q < 2.0f)) return 0.0f;
        float d;
        const float s = sinc_f((float)(0.5 * SPH_PI) * q, d), s2 = s * s;
        return knorm * (ih2 * ih2) * (5.0f * (s2 * s2) * d * (float)(0.5 * SPH_PI));
    } else {
        float w;
        if (q < 1.0f) w = q * (-3.0f + 2.25f * q);
        else if (q < 2.0f) { float t = 2.0f - q; w = -0.75f * t * t; }
        else w = 0.0f;
        return (float)(1.0 / SPH_PI) * (ih2 * ih2) * w;
    }
}

// ---------------------------------------------------------------------------
// pack: split coordinates, FP32 velocity (the predicted one), m, h, 1/h
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_pack_mixed(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ vz, const double *__restrict__ m, const double *__restrict__ h,
    const double *__restrict__ bbox, MixQ Q)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {x[i], y[i], z[i]};
    uint32_t cell = 0;
    float dl[3];
    for (int d = 0; d < 3; ++d) {
        double lo = bbox[d], L = bbox[3 + d] - lo;
        int g = cell10(p[d], lo, L);
        double w = L / 1024.0;
        dl[d] = (float)((p[d] - lo) - (double)g * w);
        cell |= (uint32_t)g << (10 * d);
    }
    Q.A[i] = make_float4(dl[0], dl[1], dl[2], __uint_as_float(cell));
    Q.B[i] = make_float4((float)vx[i], (float)vy[i], (float)vz[i], (float)m[i]);
    double hi = h[i];
    Q.C[i] = make_float4((float)hi, 0.0f, 0.0f, 0.0f);
}

// ---------------------------------------------------------------------------
// density and divergence in FP32; complement E via prefilter + exact test
// ---------------------------------------------------------------------------
__device__ __forceinline__ MixGeo mix_geo(const double *__restrict__ bbox, const Geo &g)
{
    MixGeo G;
    for (int d = 0; d < 3; ++d) {
        G.w[d] = (float)((bbox[3 + d] - bbox[d]) / 1024.0);
        G.per[d] = g.per[d];
    }
    return G;
}

// GH: also the grad-h factor Omega_i = 1 - (1/(3 rho_i)) sum_j m_j (3 W + r dW/dr).
// GV: generalized volume elements, Y_i = X_i W(0,h_i) + sum_{L_i} X_j W(r_ij,h_i)
// with X from the D quads (compensated FP32 sum, stored in FP64 in ysum) and
// rho_i = m_i Y_i / X_i in FP64 (X and m from the FP64 arrays)
template <int PM, bool EXTRA, int KER, bool GH, bool GV>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_D void k_density_mixed(
    int64_t n, MixQ Q, const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K,
    const double *__restrict__ bbox, Geo g, float knorm, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const double *__restrict__ h,
    double *__restrict__ rho, double *__restrict__ divv, double *__restrict__ omega,
    int32_t *__restrict__ ecnt,
    int32_t *__restrict__ eidx, int slots, int64_t *__restrict__ status,
    const double *__restrict__ X, const double *__restrict__ m, double *__restrict__ ysum)
{
    const int lane = threadIdx.x & (SPH_MGROUP - 1);
    const int grp = threadIdx.x / SPH_MGROUP;
    const int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SPH_BLOCK;
    int64_t appended = 0, dropped = 0;
    const MixGeo G = mix_geo(bbox, g);
    for (int rr = 0; rr < SPH_MGROUP; ++rr) {   // SPH_BLOCK / SPH_MGROUP groups, SPH_MGROUP rounds
        const int64_t i = base + (int64_t)rr * (SPH_BLOCK / SPH_MGROUP) + grp;
        NeuF s = {0.0f, 0.0f}, dv = {0.0f, 0.0f}, t = {0.0f, 0.0f};
        float4 ai = make_float4(0.f, 0.f, 0.f, 0.f), bi = ai;
        float inv_h = 0.0f;
        if (i < n) {
            ai = Q.A[i];
            bi = Q.B[i];
            inv_h = (float)(1.0 / h[i]);
            const uint32_t gi = cell_of(ai);
            const int cnt = min(nc[i], K);
            const int32_t *row = idx + i * (int64_t)K;
            // batches of SPH_MBATCH pairs per lane: indices, then the
            // gathers, then the arithmetic (slots past the end are skipped)
            for (int k0 = lane; k0 < cnt; k0 += SPH_MBATCH * SPH_MGROUP) {
                int jb[SPH_MBATCH];
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    const int k = k0 + q * SPH_MGROUP;
                    jb[q] = k < cnt ? row[k] : (int)i;
                }
                float4 ab[SPH_MBATCH], bb[SPH_MBATCH];
                float hb[SPH_MBATCH], xb[SPH_MBATCH];
                int ek[SPH_MBATCH];   // complement slot taken for pair q (-1: none)
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    ab[q] = Q.A[jb[q]];
                    bb[q] = Q.B[jb[q]];
                    if (EXTRA) hb[q] = Q.C[jb[q]].x;
                    xb[q] = GV ? Q.D[jb[q]].x : 0.0f;
                    ek[q] = -1;
                }
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    if (k0 + q * SPH_MGROUP >= cnt) break;
                    const int j = jb[q];
                    const float4 aj = ab[q], bj = bb[q];
                    const uint32_t gj = cell_of(aj);
                    float dx = split_diff<PM, 0>(gi, gj, ai.x, aj.x, G);
                    float dy = split_diff<PM, 1>(gi, gj, ai.y, aj.y, G);
                    float dz = split_diff<PM, 2>(gi, gj, ai.z, aj.z, G);
                    float r2 = dx * dx + dy * dy + dz * dz;
                    if (EXTRA) {
                        // is i outside j's gather sphere?  FP32 decides clear
                        // cases (|error| of r2 is below 1e-6 relative), FP64
                        // the band
                        const float hj = hb[q];
                        const float lim = 4.0f * hj * hj;
                        bool outside;
                        if (r2 > lim * (1.0f + 1e-5f)) {
                            outside = true;
                        } else if (r2 < lim * (1.0f - 1e-5f)) {
                            outside = false;
                        } else {
#pragma clang fp contract(off)
                            double ex = mimg<PM, 0>(x[i], x[j], g),
                                   ey = mimg<PM, 1>(y[i], y[j], g),
                                   ez = mimg<PM, 2>(z[i], z[j], g);
                            double e2 = exact_r2(ex, ey, ez);
                            double twoh = 2.0 * h[j];
                            outside = !(e2 < twoh * twoh);
                        }
                        if (outside) ek[q] = extra_take(j, ecnt);
                    }
                    const float rinv = r2 > 0.0f ? rsq_pair(r2) : 0.0f;
                    const float r = r2 * rinv;
                    const float mj = bj.w;
                    const float wk = kern_w_f<KER>(r, inv_h, knorm);
                    neu_add(s, (GV ? xb[q] : mj) * wk);
                    if (r > 0.0f) {
                        const float dw = kern_dwdr_f<KER>(r, inv_h, knorm);
                        float gw = dw * rinv;
                        float vdot = (bj.x - bi.x) * (-dx) + (bj.y - bi.y) * (-dy) +
                                     (bj.z - bi.z) * (-dz);
                        neu_add(dv, mj * vdot * gw);
                        if (GH) neu_add(t, mj * (3.0f * wk + r * dw));
                    } else if (GH) {
                        neu_add(t, mj * 3.0f * wk);
                    }
                }
                if (EXTRA) {
#pragma unroll
                    for (int q = 0; q < SPH_MBATCH; ++q)
                        if (ek[q] >= 0) extra_put(jb[q], ek[q], (int)i, eidx, slots, appended, dropped);
                }
            }
        }
        s = mgroup_neu(s);
        dv = mgroup_neu(dv);
        if (GH) t = mgroup_neu(t);
        if (i < n && lane == 0) {
            const float w0 = kern_w_f<KER>(0.0f, inv_h, knorm);
            NeuF tot = {(GV ? Q.D[i].x : bi.w) * w0, 0.0f};
            neu_add(tot, s.s);
            tot.c += s.c;
            double sd = neu_val(tot);
            if (GV) {
                ysum[i] = sd;
                sd = m[i] * sd / X[i];
            }
            rho[i] = sd;
            divv[i] = neu_val(dv) / sd;
            if (GH) omega[i] = 1.0 - (3.0 * (double)(bi.w * w0) + neu_val(t)) / (3.0 * sd);
        }
    }
    if (EXTRA) {
        block_add_i64(appended, status + ST_EXTRA_TOTAL);
        block_add_i64(dropped, status + ST_EXTRA_OVERFLOW);
    }
}

// EOS in FP64 (as the plain form) and the FP32 force fields of the record
// (generalized volumes, X non-NULL: the record carries q = (X/m) P / Y^2)
__global__ __launch_bounds__(SPH_BLOCK) void k_eos_mixed(int64_t n, const double *__restrict__ rho,
                                                         const double *__restrict__ u, double gamma,
                                                         const double *__restrict__ omega,
                                                         double *__restrict__ p,
                                                         double *__restrict__ c,
                                                         MixQ Q, int check,
                                                         int64_t *__restrict__ status,
                                                         const double *__restrict__ X,
                                                         const double *__restrict__ m,
                                                         const double *__restrict__ ysum)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t bad = 0;
    if (i < n) {
        double rh = rho[i];
        double pv = (gamma - 1.0) * rh * u[i];
        double cv = sqrt(gamma * (gamma - 1.0) * u[i]);
        p[i] = pv;
        c[i] = cv;
        Q.C[i].y = (float)cv;
        Q.C[i].z = (float)rh;
        if (X) {
            const double yv = ysum[i];
            Q.C[i].w = (float)(X[i] / m[i] * pv / (yv * yv));
        } else {
            Q.C[i].w = (float)(pv / (omega ? omega[i] * (rh * rh) : rh * rh));   // P / (Omega rho^2)
        }
        if (check && !(isfinite(pv) && isfinite(cv) && isfinite(rh))) bad = 1;
    }
    if (check) block_add_i64(bad, status + ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// momentum, energy, viscosity and Courant step in FP32
// ---------------------------------------------------------------------------
struct ForceAccF {
    NeuF ax, ay, az, du;
    float mumax;
};

// own fields of particle i (a, b, c) and the gathered fields of j; d, e:
// the IAD matrix when gradients are IAD
struct QuadF {
    float4 a, b, c, d;
    float2 e;
};

// GR: 0 averaged kernel gradient; 1 pressure terms with each particle's own
// kernel gradient (grad-h form); 2 pressure terms with each particle's own
// IAD gradient A = c d W, the viscosity with their mean; 3 generalized
// volume elements (c.w = q = r g, d.x = X, d.y = r = X/m), the viscosity with
// the averaged gradient
template <int PM, int KER, int GR>
__device__ __forceinline__ void force_pair_f(const QuadF &ri, float inv_hi, uint32_t gi,
                                             const QuadF &rj, const MixGeo &G, float knorm,
                                             float alpha, float beta, float eta2, ForceAccF &A)
{
    const uint32_t gj = cell_of(rj.a);
    float dx = split_diff<PM, 0>(gi, gj, ri.a.x, rj.a.x, G);
    float dy = split_diff<PM, 1>(gi, gj, ri.a.y, rj.a.y, G);
    float dz = split_diff<PM, 2>(gi, gj, ri.a.z, rj.a.z, G);
    float r2 = dx * dx + dy * dy + dz * dz;
    // a pair at r = 0 adds zero to every sum (1/r taken as 0 zeroes the
    // kernel gradients, the offset zeroes the IAD ones); no early exit, so
    // that the compiler issues all of a batch's gathers before its arithmetic
    float inv_r = r2 > 0.0f ? rsq_pair(r2) : 0.0f;
    float r = r2 * inv_r;
    float xij = -dx, yij = -dy, zij = -dz;
    float vxij = ri.b.x - rj.b.x, vyij = ri.b.y - rj.b.y, vzij = ri.b.z - rj.b.z;
    float w = vxij * xij + vyij * yij + vzij * zij;
    if (GR == 2) {
        float Pi = 0.0f;
        if (w < 0.0f) {
            float hb = 0.5f * (ri.c.x + rj.c.x);
            float cb = 0.5f * (ri.c.y + rj.c.y);
            float rb = 0.5f * (ri.c.z + rj.c.z);
            const float den = r2 + eta2 * hb * hb;
            const float rq = __builtin_amdgcn_rcpf(den * rb);
            const float mu = hb * w * (rb * rq);
            Pi = (-alpha * cb * mu + beta * mu * mu) * (den * rq);
            A.mumax = fmaxf(A.mumax, fabsf(mu));
        }
        const float wi = kern_w_f<KER>(r, inv_hi, knorm);
        const float wj = kern_w_f<KER>(r, __builtin_amdgcn_rcpf(rj.c.x), knorm);
        // A = c d W with d = x_j - x_i = (dx, dy, dz); c = (d.x d.y d.z d.w e.x e.y)
        const float aix = (ri.d.x * dx + ri.d.y * dy + ri.d.z * dz) * wi;
        const float aiy = (ri.d.y * dx + ri.d.w * dy + ri.e.x * dz) * wi;
        const float aiz = (ri.d.z * dx + ri.e.x * dy + ri.e.y * dz) * wi;
        const float ajx = (rj.d.x * dx + rj.d.y * dy + rj.d.z * dz) * wj;
        const float ajy = (rj.d.y * dx + rj.d.w * dy + rj.e.x * dz) * wj;
        const float ajz = (rj.d.z * dx + rj.e.x * dy + rj.e.y * dz) * wj;
        const float abx = 0.5f * (aix + ajx), aby = 0.5f * (aiy + ajy), abz = 0.5f * (aiz + ajz);
        const float mj = rj.b.w, pi_t = ri.c.w, pj_t = rj.c.w;
        neu_add(A.ax, -mj * ((pi_t * aix + pj_t * ajx) + Pi * abx));
        neu_add(A.ay, -mj * ((pi_t * aiy + pj_t * ajy) + Pi * aby));
        neu_add(A.az, -mj * ((pi_t * aiz + pj_t * ajz) + Pi * abz));
        neu_add(A.du, mj * (pi_t * (vxij * aix + vyij * aiy + vzij * aiz) +
                            0.5f * Pi * (vxij * abx + vyij * aby + vzij * abz)));
        return;
    }
    float gwi = kern_dwdr_f<KER>(r, inv_hi, knorm) * inv_r;
    float gwj = kern_dwdr_f<KER>(r, __builtin_amdgcn_rcpf(rj.c.x), knorm) * inv_r;
    float gbar = 0.5f * (gwi + gwj);
    float Pi = 0.0f;
    if (w < 0.0f) {
        float hb = 0.5f * (ri.c.x + rj.c.x);
        float cb = 0.5f * (ri.c.y + rj.c.y);
        float rb = 0.5f * (ri.c.z + rj.c.z);
        // mu = hb w / den and Pi = (..) / rb from one reciprocal of den rb
        const float den = r2 + eta2 * hb * hb;
        const float rq = __builtin_amdgcn_rcpf(den * rb);
        const float mu = hb * w * (rb * rq);
        Pi = (-alpha * cb * mu + beta * mu * mu) * (den * rq);
        A.mumax = fmaxf(A.mumax, fabsf(mu));
    }
    float mj = rj.b.w;
    if (GR == 3) {
        // m_j r_i r_j g_i = X_j q_i and m_j r_i r_j g_j = r_i m_j q_j
        const float ti = rj.d.x * ri.c.w * gwi;
        float f = (ti + ri.d.y * mj * rj.c.w * gwj) + mj * Pi * gbar;
        neu_add(A.ax, -f * xij);
        neu_add(A.ay, -f * yij);
        neu_add(A.az, -f * zij);
        neu_add(A.du, (ti + 0.5f * mj * Pi * gbar) * w);
        return;
    }
    if (GR == 1) {
        float f = mj * ((ri.c.w * gwi + rj.c.w * gwj) + Pi * gbar);
        neu_add(A.ax, -f * xij);
        neu_add(A.ay, -f * yij);
        neu_add(A.az, -f * zij);
        neu_add(A.du, mj * (ri.c.w * gwi + 0.5f * Pi * gbar) * w);
        return;
    }
    float sfac = (ri.c.w + rj.c.w) + Pi;
    float f = mj * sfac * gbar;
    neu_add(A.ax, -f * xij);
    neu_add(A.ay, -f * yij);
    neu_add(A.az, -f * zij);
    neu_add(A.du, mj * (ri.c.w + 0.5f * Pi) * gbar * w);
}

// S_i = L_i (row order) then E_i (ascending), SPH_MGROUP lanes per particle;
// ELDS: E rows ranked in LDS here (capacity <= SPH_ELDS), else sorted already
template <int PM, bool ELDS, int KER, int GR>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_F void k_forces_mixed(
    int64_t n, MixQ Q, const float2 *__restrict__ qe, const int32_t *__restrict__ nc, const int32_t *__restrict__ idx, int K,
    const int32_t *__restrict__ ecnt, const int32_t *__restrict__ eidx, int slots,
    const double *__restrict__ bbox, Geo g, float knorm, float alpha, float beta, float eta2,
    double alpha_d,
    double beta_d, double cfl, const double *__restrict__ h, const double *__restrict__ c,
    double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az,
    double *__restrict__ du, double *__restrict__ dt_part)
{
    const int lane = threadIdx.x & (SPH_MGROUP - 1);
    const int grp = threadIdx.x / SPH_MGROUP;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = blk * SPH_MPTILE_F;
    double dti = INFINITY;
    const MixGeo G = mix_geo(bbox, g);
    __shared__ int32_t e_raw[ELDS ? SPH_BLOCK / SPH_MGROUP : 1][ELDS ? SPH_ELDS : 1];
    __shared__ int32_t e_srt[ELDS ? SPH_BLOCK / SPH_MGROUP : 1][ELDS ? SPH_ELDS : 1];
    for (int rr = 0; rr < SPH_MROUNDS_F; ++rr) {   // SPH_BLOCK / SPH_MGROUP groups per round
        const int64_t i = base + (int64_t)rr * (SPH_BLOCK / SPH_MGROUP) + grp;
        ForceAccF A = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, 0.f};
        if (i < n) {
            QuadF ri;
            ri.a = Q.A[i]; ri.b = Q.B[i]; ri.c = Q.C[i];
            if (GR == 2) { ri.d = Q.D[i]; ri.e = qe[i]; }
            if (GR == 3) ri.d = Q.D[i];
            const float inv_hi = (float)(1.0 / h[i]);
            const uint32_t gi = cell_of(ri.a);
            const int cnt = min(nc[i], K);
            const int ne = min(ecnt[i], slots);
            const int tot = cnt + ne;
            const int32_t *lrow = idx + i * (int64_t)K;
            const int32_t *erow = eidx + i * (int64_t)slots;
            if (ELDS && ne > 0) erow_sort_lds<SPH_MGROUP>(erow, ne, lane, e_raw[grp], e_srt[grp]);
            const int32_t *es = ELDS ? e_srt[grp] : erow;
            for (int k0 = lane; k0 < tot; k0 += SPH_MFBATCH * SPH_MGROUP) {
                int jb[SPH_MFBATCH];
#pragma unroll
                for (int q = 0; q < SPH_MFBATCH; ++q) {
                    const int k = k0 + q * SPH_MGROUP;
                    jb[q] = k < cnt ? lrow[k] : (k < tot ? es[k - cnt] : (int)i);
                }
                QuadF rb[SPH_MFBATCH];
#pragma unroll
                for (int q = 0; q < SPH_MFBATCH; ++q) {
                    rb[q].a = Q.A[jb[q]]; rb[q].b = Q.B[jb[q]]; rb[q].c = Q.C[jb[q]];
                    if (GR == 2) { rb[q].d = Q.D[jb[q]]; rb[q].e = qe[jb[q]]; }
                    if (GR == 3) rb[q].d = Q.D[jb[q]];
                }
#pragma unroll
                for (int q = 0; q < SPH_MFBATCH; ++q) {
                    if (k0 + q * SPH_MGROUP >= tot) break;
                    force_pair_f<PM, KER, GR>(ri, inv_hi, gi, rb[q], G, knorm, alpha, beta, eta2, A);
                }
            }
        }
        A.ax = mgroup_neu(A.ax);
        A.ay = mgroup_neu(A.ay);
        A.az = mgroup_neu(A.az);
        A.du = mgroup_neu(A.du);
        A.mumax = mgroup_max(A.mumax);
        if (i < n && lane == 0) {
            ax[i] = neu_val(A.ax);
            ay[i] = neu_val(A.ay);
            az[i] = neu_val(A.az);
            du[i] = neu_val(A.du);
            const double ci = c[i];
            dti = fmin(dti, cfl * h[i] / (ci + 1.2 * (alpha_d * ci + beta_d * (double)A.mumax)));
        }
    }
    __shared__ double sh[SPH_BLOCK];
    sh[threadIdx.x] = dti;
    __syncthreads();
    for (int s = SPH_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dt_part[blk] = sh[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// the record area holds n_max particles (at least one) of each quad array
static MixQ ctx_quads(sph_ctx *c)
{
    return mix_quads(c->w.mixrec, c->p.n_max > 0 ? c->p.n_max : 1);
}

hipError_t launch_pack_mixed(sph_ctx *c, sph_particles *s)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    hipLaunchKernelGGL(k_pack_mixed, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, s->x[k], s->y[k], s->z[k], s->pvx, s->pvy, s->pvz, s->m[k],
                       s->h[k], c->w.bbox, ctx_quads(c));
    return hipGetLastError();
}

// generalized volume elements: X_i = (m_i / rho_i)^p from the density held
// (FP64), with X and X/m in FP32 in the D quad for the pair loops
__global__ __launch_bounds__(SPH_BLOCK) void k_gve_weights_mixed(int64_t n,
                                                                 const double *__restrict__ m,
                                                                 const double *__restrict__ rho,
                                                                 double p, double *__restrict__ X,
                                                                 MixQ Q)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xv = pow(m[i] / rho[i], p);
    X[i] = xv;
    Q.D[i] = make_float4((float)xv, (float)(xv / m[i]), 0.0f, 0.0f);
}

hipError_t launch_density_mixed(sph_ctx *c, sph_particles *s, const sph_nlist *nl,
                                bool build_extra)
{
    int64_t n = s->n;
    if (build_extra) {
        hipError_t e = launch_zero_i32(c, nl->ecnt, n);
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    hipError_t e = launch_pack_mixed(c, s);
    if (e != hipSuccess) return e;
    int cur = s->cur;
    Geo g = make_geo(c->p);
    unsigned nb = (unsigned)ceil_div(n, SPH_BLOCK);
    const MixQ Q = ctx_quads(c);
#define SPH_DENSITY_ARGS                                                                      \
    dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, Q, s->nc[cur], nl->idx, c->p.list_stride,      \
        c->w.bbox, g, (float)c->knorm, s->x[cur], s->y[cur], s->z[cur], s->h[cur], s->rho[cur], \
        s->divv[cur], c->w.omega, nl->ecnt, nl->eidx, c->p.extra_slots, c->w.status,           \
        c->w.gve_x, s->m[cur], c->w.gve_y
#define SPH_DENSITY(EX, GHV, GVV)                                                             \
    SPH_DISPATCH_KER(c->p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                           \
        hipLaunchKernelGGL((k_density_mixed<PM, EX, KER, GHV, GVV>), SPH_DENSITY_ARGS)))
    if (c->p.volumes == SPH_VOLUMES_GENERALIZED) {
        // weights from the previous evaluation's density (the standard one
        // first when an evaluation starts a run), in FP64 and in the D quads
        bool extra = build_extra;
        if (c->gve_fresh) {
            if (extra) { SPH_DENSITY(true, false, false) }
            else { SPH_DENSITY(false, false, false) }
            extra = false;
        }
        hipLaunchKernelGGL(k_gve_weights_mixed, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n,
                           s->m[cur], s->rho[cur], c->p.gve_exponent, c->w.gve_x, Q);
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

hipError_t launch_eos_mixed(sph_ctx *c, sph_particles *s)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_eos_mixed, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, s->rho[s->cur], s->pu, c->p.gamma,
                       c->p.grad_h ? c->w.omega : nullptr, s->p, s->c, ctx_quads(c),
                       c->p.check_finite, c->w.status, c->w.gve_x, s->m[s->cur], c->w.gve_y);
    return hipGetLastError();
}

// IAD moment matrix in FP32 with compensated sums (SPH_MGROUP lanes per
// particle over its gather set), inverted in FP64 by adjugate over
// determinant, stored as floats: (xx, xy, xz, yy) in the D quad, (yz, zz) in qe
template <int PM, int KER>
__global__ __launch_bounds__(SPH_BLOCK) SPH_PAIR_WAVES_D void k_iad_mixed(
    int64_t n, MixQ Q, float2 *__restrict__ qe, const int32_t *__restrict__ nc,
    const int32_t *__restrict__ idx, int K, const double *__restrict__ bbox, Geo g, float knorm,
    const double *__restrict__ h, int64_t *__restrict__ status)
{
    const int lane = threadIdx.x & (SPH_MGROUP - 1);
    const int grp = threadIdx.x / SPH_MGROUP;
    const int64_t base = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SPH_BLOCK;
    const MixGeo G = mix_geo(bbox, g);
    int64_t bad = 0;
    for (int rr = 0; rr < SPH_MGROUP; ++rr) {
        const int64_t i = base + (int64_t)rr * (SPH_BLOCK / SPH_MGROUP) + grp;
        NeuF t[6] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        if (i < n) {
            const float4 ai = Q.A[i];
            const float inv_h = (float)(1.0 / h[i]);
            const uint32_t gi = cell_of(ai);
            const int cnt = min(nc[i], K);
            const int32_t *row = idx + i * (int64_t)K;
            for (int k0 = lane; k0 < cnt; k0 += SPH_MBATCH * SPH_MGROUP) {
                int jb[SPH_MBATCH];
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    const int k = k0 + q * SPH_MGROUP;
                    jb[q] = k < cnt ? row[k] : (int)i;
                }
                float4 ab[SPH_MBATCH];
                float mb[SPH_MBATCH], rb[SPH_MBATCH];
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    ab[q] = Q.A[jb[q]];
                    mb[q] = Q.B[jb[q]].w;
                    rb[q] = Q.C[jb[q]].z;
                }
#pragma unroll
                for (int q = 0; q < SPH_MBATCH; ++q) {
                    if (k0 + q * SPH_MGROUP >= cnt) break;
                    const uint32_t gj = cell_of(ab[q]);
                    const float dx = split_diff<PM, 0>(gi, gj, ai.x, ab[q].x, G);
                    const float dy = split_diff<PM, 1>(gi, gj, ai.y, ab[q].y, G);
                    const float dz = split_diff<PM, 2>(gi, gj, ai.z, ab[q].z, G);
                    const float r = sqrtf(dx * dx + dy * dy + dz * dz);
                    const float vw = mb[q] / rb[q] * kern_w_f<KER>(r, inv_h, knorm);
                    neu_add(t[0], vw * dx * dx); neu_add(t[1], vw * dx * dy);
                    neu_add(t[2], vw * dx * dz); neu_add(t[3], vw * dy * dy);
                    neu_add(t[4], vw * dy * dz); neu_add(t[5], vw * dz * dz);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) t[k] = mgroup_neu(t[k]);
        if (i < n && lane == 0) {
            const double txx = neu_val(t[0]), txy = neu_val(t[1]), txz = neu_val(t[2]);
            const double tyy = neu_val(t[3]), tyz = neu_val(t[4]), tzz = neu_val(t[5]);
            const double axx = tyy * tzz - tyz * tyz;
            const double axy = txz * tyz - txy * tzz;
            const double axz = txy * tyz - txz * tyy;
            const double det = txx * axx + txy * axy + txz * axz;
            if (!(det > 0.0) || !isfinite(det)) ++bad;
            const double id = 1.0 / det;
            const double ayy = txx * tzz - txz * txz;
            const double ayz = txy * txz - txx * tyz;
            const double azz = txx * tyy - txy * txy;
            Q.D[i] = make_float4((float)(axx * id), (float)(axy * id), (float)(axz * id),
                                 (float)(ayy * id));
            qe[i] = make_float2((float)(ayz * id), (float)(azz * id));
        }
    }
    block_add_i64(bad, status + ST_IAD_SINGULAR);
}

static hipError_t launch_iad_mixed(sph_ctx *c, sph_particles *s, const sph_nlist *nl)
{
    const int64_t n = s->n;
    if (n == 0) return hipSuccess;
    Geo g = make_geo(c->p);
    SPH_DISPATCH_KER(c->p.kernel, SPH_DISPATCH_PM(periodic_mask(g),
        hipLaunchKernelGGL((k_iad_mixed<PM, KER>), dim3((unsigned)ceil_div(n, SPH_BLOCK)),
                           dim3(SPH_BLOCK), 0, c->stream, n, ctx_quads(c), (float2 *)c->w.iad,
                           s->nc[s->cur], nl->idx, c->p.list_stride, c->w.bbox, g,
                           (float)c->knorm, s->h[s->cur], c->w.status)))
    return hipGetLastError();
}

hipError_t launch_forces_mixed(sph_ctx *c, sph_particles *s, const sph_nlist *nl)
{
    int64_t n = s->n;
    int cur = s->cur;
    const sph_params &p = c->p;
    int64_t nb = ceil_div(n > 0 ? n : 1, SPH_MPTILE_F);
    c->dt_parts = nb;
    Geo g = make_geo(p);
#define SPH_FORCE_ARGS                                                                        \
    dim3((unsigned)nb), dim3(SPH_BLOCK), 0, c->stream, n, ctx_quads(c), (const float2 *)c->w.iad, \
        s->nc[cur], nl->idx,                                                                   \
        p.list_stride, nl->ecnt, nl->eidx, p.extra_slots, c->w.bbox, g, (float)c->knorm,       \
        (float)p.av_alpha, (float)p.av_beta, (float)p.av_eta2, p.av_alpha, p.av_beta, p.cfl,   \
        s->h[cur], s->c, s->ax[cur], s->ay[cur], s->az[cur], s->du[cur], c->w.red_part
    if (p.extra_slots > SPH_ELDS) {
        hipError_t e = launch_sort_extra(c, nl, n);
        if (e != hipSuccess) return e;
    }
    const bool elds = p.extra_slots <= SPH_ELDS;
#define SPH_FORCE_GR(GRV)                                                                     \
    if (elds) {                                                                               \
        SPH_DISPATCH_KER(p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                          \
            hipLaunchKernelGGL((k_forces_mixed<PM, true, KER, GRV>), SPH_FORCE_ARGS)))        \
    } else {                                                                                  \
        SPH_DISPATCH_KER(p.kernel, SPH_DISPATCH_PM(periodic_mask(g),                          \
            hipLaunchKernelGGL((k_forces_mixed<PM, false, KER, GRV>), SPH_FORCE_ARGS)))       \
    }
    if (p.gradients == SPH_GRADIENTS_IAD) {
        hipError_t e = launch_iad_mixed(c, s, nl);
        if (e != hipSuccess) return e;
        SPH_FORCE_GR(2)
    } else if (p.grad_h) {
        SPH_FORCE_GR(1)
    } else if (p.volumes == SPH_VOLUMES_GENERALIZED) {
        SPH_FORCE_GR(3)
    } else {
        SPH_FORCE_GR(0)
    }
#undef SPH_FORCE_GR
#undef SPH_FORCE_ARGS
    return hipGetLastError();
}
