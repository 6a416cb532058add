// Internal declarations of libsph: context, workspace layout, device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

#define SPH_BLOCK 256
// waves per SIMD the pair kernels are compiled for (empty: the compiler's
// choice)
#ifdef SPH_DENSITY_WAVES
#define SPH_PAIR_WAVES_D __attribute__((amdgpu_waves_per_eu(SPH_DENSITY_WAVES, SPH_DENSITY_WAVES)))
#else
#define SPH_PAIR_WAVES_D
#endif
#ifdef SPH_FORCE_WAVES
#define SPH_PAIR_WAVES_F __attribute__((amdgpu_waves_per_eu(SPH_FORCE_WAVES, SPH_FORCE_WAVES)))
#else
#define SPH_PAIR_WAVES_F
#endif
// shell records of the h iteration: slots per particle
#ifndef SPH_SHELL_SLOTS
#define SPH_SHELL_SLOTS 48
#endif
#ifndef SPH_SORT_ITEMS
#define SPH_SORT_ITEMS 16                      // keys per thread per sort tile
#endif
#define SPH_SORT_TILE (SPH_BLOCK * SPH_SORT_ITEMS)
#define SPH_SCAN_ITEMS 8
#define SPH_SCAN_TILE (SPH_BLOCK * SPH_SCAN_ITEMS)

// learned smoothing length: gradient partial rows (one per training wave)
#define SPH_MLP_TRAIN_WAVES 256
#define SPH_MLP_ROW 4680   // SPH_MLP_NPARAM gradients, the loss, padding

// device status words (int64) in the workspace
enum {
    ST_NONCONV = 0,
    ST_LIST_OVERFLOW = 1,
    ST_EXTRA_OVERFLOW = 2,
    ST_NONFINITE = 3,
    ST_HCOUNTS = 4,
    ST_LEARN_ACC = 5,
    ST_LEARN_FALLBACK = 6,
    ST_CANDIDATES = 7,
    ST_EXTRA_TOTAL = 8,
    ST_CANDIDATES_FIRST = 9,   // candidates tested by round 0 of the h iteration
    ST_IAD_SINGULAR = 10,      // IAD moment matrices that could not be inverted
    ST_CSR_OVERFLOW = 11,      // interaction-set CSR entries beyond the caller's capacity
    ST_COUNT = 16
};

// Geometry of the periodic box, by value into kernels.
struct Geo {
    int per[3];
    double L[3];      // box_hi - box_lo of periodic dimensions (0 otherwise)
    double halfL[3];  // 0.5 * L
};

// FP64 neighbour records read by the pair kernels, two fields per 16-byte
// load (a gather's cost follows the cache lines it touches, and lines of
// 16-byte pairs hold runs of neighbours almost as well as lines of single
// fields): xy = (x, y), zh = (z, h), vxy / vzm = (v*x, v*y) / (v*z, m)
// from the pack before density, rp = (rho, P / rho^2) from the EOS.
struct Pk64 {
    double2 *xy, *zh, *vxy, *vzm, *rp;
};

// Workspace carve-up.
struct Workspace {
    double *bbox;          // 6: lo[3], hi[3]
    double *bbox_part;     // nb_red * 6
    uint32_t *key_a;       // n_max  (unsorted keys / sort ping)
    uint32_t *key_b;       // n_max
    int32_t *val_a;        // n_max
    int32_t *val_b;        // n_max
    uint32_t *hist;        // 256 * nb_sort
    uint64_t *scan_part;   // scan partials
    int32_t *cell_start;   // 8^max_level + 1
    double *hk;            // 1024 Hernquist-Katz factors
    int64_t *status;       // ST_COUNT
    int64_t *learn_step;   // 4: tries and misses of the current learned h solve, and
                           // whether the next one's try records a shell (1) or not (0)
    double *dt_cur;        // 1: dt used by the current step
    double *red_part;      // reduction partials: nb_red * 8, or one per force block
    uint8_t *refill;       // n_max
    int32_t *work;         // n_max: particles needing the per-particle iteration
    int64_t *woff;         // n_max + 1: their worklist positions
    int32_t *wl;           // n_max: the worklist
    double *hs_next, *hs_lo, *hs_hi, *hs_best_h, *hs_last_h;  // h iteration state, n_max each
    int32_t *hs_best_n, *hs_itk, *hs_bits;
    int2 *shell_e;         // SPH_SHELL_SLOTS per particle, slot-major with shell_stride:
                           // (j, FP32 bits of r^2)
    int64_t shell_stride;
    void *mixrec;          // n_max records of 64 bytes (mixed form)
    // learned smoothing length
    float *mlp_master;     // SPH_MLP_NPARAM FP32 parameters
    float *mlp_m, *mlp_v;  // Adam moments
    float *mlp_grad;       // gradient + loss (SPH_MLP_NPARAM + 1)
    uint16_t *mlp_wb;      // bf16 copies of the parameters
    double *mlp_norm;      // feature mean[6], std[6]
    float *mlp_part;       // per-wave gradient partial rows
    double *h_try;         // n_max predicted smoothing lengths (learned mode)
    void *pk64;            // n_max * 80 bytes: FP64 neighbour records (Pk64, FP64 form)
    double *du_prev[2];    // AB2: du of the previous evaluation, ping-pong like the state
    double *dt_prev;       // AB2: the previous step's dt
    double *omega;         // grad-h: Omega of the last density (n_max, FP64 form)
    double2 *iad;          // IAD: c_i as 3 arrays of n_max double2 (xx,xy) (xz,yy) (yz,zz)
    double *gve_x;         // generalized volumes: weights X (n_max)
    double *gve_y;         // and the sums Y = sum_j X_j W(h_i) of the last density (n_max)
    int64_t nb_red;
    int64_t nb_sort;
    int64_t scan_part_len;
};

struct StageTimer;  // per-stage HIP-event intervals (api.cpp)

struct sph_ctx {
    sph_params p;
    hipStream_t stream;
    void *ws_base;
    size_t ws_bytes;
    Workspace w;
    int bound;
    int timing;
    StageTimer *timer;
    int mlp_ready;         // weights set since the last bind
    int mlp_t;             // Adam step counter of sph_mlp_train
    float *harvest_feat;   // step sink of (features, target) rows, or NULL
    float *harvest_target;
    int harvest_mode;      // SPH_TARGET_*
    double knorm;          // B_5 of the sinc kernel (sph_create)
    int ab2_hist;          // AB2: a step since the last bind / evaluation
    int gve_fresh;         // generalized volumes: no previous density (sph_evaluate)
    int64_t dt_parts;      // dt partials the last force launch wrote to red_part
    char err[512];
};

size_t sph_layout(const sph_params *p, void *base, Workspace *w);

// ---------------------------------------------------------------------------
// launchers (each returns hipError_t of the launch)
// ---------------------------------------------------------------------------
hipError_t launch_bbox(sph_ctx *c, const double *x, const double *y, const double *z, int64_t n);
hipError_t launch_keys(sph_ctx *c, const double *x, const double *y, const double *z, int64_t n);
hipError_t launch_radix_sort(sph_ctx *c, int64_t n, uint32_t *key_out, int32_t *val_out);
hipError_t launch_permute(sph_ctx *c, sph_particles *s, const int32_t *perm);
hipError_t launch_cell_table(sph_ctx *c, const uint32_t *sorted_key, int64_t n);
hipError_t launch_scan_i32_to_i64(sph_ctx *c, const int32_t *in, int64_t *out, int64_t n);
hipError_t launch_scan_u32(sph_ctx *c, const uint32_t *in, uint32_t *out, int64_t n);

hipError_t launch_hsolve(sph_ctx *c, sph_particles *s, sph_nlist *nl, const double *h_try,
                         int phase);
hipError_t launch_extra(sph_ctx *c, sph_particles *s, sph_nlist *nl);
hipError_t launch_sort_extra(sph_ctx *c, const sph_nlist *nl, int64_t n);
hipError_t launch_density(sph_ctx *c, sph_particles *s, const sph_nlist *nl, bool build_extra);
hipError_t launch_zero_i32(sph_ctx *c, int32_t *a, int64_t n);
hipError_t launch_eos(sph_ctx *c, sph_particles *s);
hipError_t launch_forces(sph_ctx *c, sph_particles *s, const sph_nlist *nl, double *d_dt);
hipError_t launch_dt_min(sph_ctx *c, int64_t n, double *d_dt);
hipError_t launch_pack_mixed(sph_ctx *c, sph_particles *s);
hipError_t launch_density_mixed(sph_ctx *c, sph_particles *s, const sph_nlist *nl,
                                bool build_extra);
hipError_t launch_eos_mixed(sph_ctx *c, sph_particles *s);
hipError_t launch_forces_mixed(sph_ctx *c, sph_particles *s, const sph_nlist *nl);
hipError_t launch_mlp_predict(sph_ctx *c, sph_particles *s, double *h_try);
hipError_t launch_mlp_features(sph_ctx *c, const sph_particles *s, const double *d_dt,
                               float *feat);
hipError_t launch_mlp_targets(sph_ctx *c, const sph_particles *s, const float *feat,
                              float *target, int centre);
hipError_t launch_mlp_forward(sph_ctx *c, const float *feat, int64_t n, float *y, uint16_t *h1,
                              uint16_t *h2);
hipError_t launch_mlp_grad(sph_ctx *c, const float *feat, const float *target,
                           const int32_t *rows, int64_t row0, int64_t n, float *grad,
                           float *loss_out);
hipError_t launch_mlp_adam(sph_ctx *c, const float *grad, double lr, double b1, double b2,
                           double eps, int t);
hipError_t launch_mlp_refresh(sph_ctx *c);
hipError_t launch_mlp_fit_norm(sph_ctx *c, const float *feat, int64_t n);
hipError_t launch_kick_drift(sph_ctx *c, sph_particles *s);
hipError_t launch_predict(sph_ctx *c, sph_particles *s);
hipError_t launch_kick(sph_ctx *c, sph_particles *s);
hipError_t launch_set_dt(sph_ctx *c, double dt, const double *d_dt);
hipError_t launch_copy_pred(sph_ctx *c, sph_particles *s);
hipError_t launch_conservation(sph_ctx *c, const sph_particles *s, double *out7);
hipError_t launch_interaction_csr(sph_ctx *c, const sph_particles *s, const sph_nlist *nl,
                                  int64_t *off, int32_t *out, int64_t cap);

static inline Geo make_geo(const sph_params &p)
{
    Geo g;
    for (int d = 0; d < 3; ++d) {
        g.per[d] = p.periodic[d] ? 1 : 0;
        g.L[d] = g.per[d] ? (p.box_hi[d] - p.box_lo[d]) : 0.0;
        g.halfL[d] = 0.5 * g.L[d];
    }
    return g;
}

__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#ifdef __HIPCC__

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical blocks so that spatially adjacent (Morton-adjacent)
// particles share one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t nx = 8;
    if (nb < 2 * nx) return b;
    int64_t per = nb / nx;          // full rounds
    int64_t full = per * nx;
    if (b >= full) return b;        // tail blocks keep their index
    return (b % nx) * per + b / nx;
}

__device__ __forceinline__ int64_t global_index()
{
    return xcd_block(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
}

// minimum-image difference component: t = b - a, wrapped once
__device__ __forceinline__ double min_image(double a, double b, int per, double L, double halfL)
{
#pragma clang fp contract(off)
    double t = b - a;
    if (per) {
        double up = t - L, dn = t + L;
        t = (t > halfL) ? up : ((t < -halfL) ? dn : t);
    }
    return t;
}

// minimum image with the periodic dimensions known at compile time (bit d
// of PM set = dimension d periodic); same arithmetic as min_image
template <int PM, int D>
__device__ __forceinline__ double mimg(double a, double b, const Geo &g)
{
#pragma clang fp contract(off)
    double t = b - a;
    if constexpr (((PM >> D) & 1) != 0) {
        double up = t - g.L[D], dn = t + g.L[D];
        t = (t > g.halfL[D]) ? up : ((t < -g.halfL[D]) ? dn : t);
    }
    return t;
}

static inline int periodic_mask(const Geo &g) { return g.per[0] | (g.per[1] << 1) | (g.per[2] << 2); }

// launches KERNEL<PM, ...> for the runtime periodic mask pm
#define SPH_DISPATCH_PM(pm, LAUNCH)                  \
    switch (pm) {                                    \
    case 0: { constexpr int PM = 0; LAUNCH; } break; \
    case 1: { constexpr int PM = 1; LAUNCH; } break; \
    case 2: { constexpr int PM = 2; LAUNCH; } break; \
    case 3: { constexpr int PM = 3; LAUNCH; } break; \
    case 4: { constexpr int PM = 4; LAUNCH; } break; \
    case 5: { constexpr int PM = 5; LAUNCH; } break; \
    case 6: { constexpr int PM = 6; LAUNCH; } break; \
    default: { constexpr int PM = 7; LAUNCH; } break; \
    }

// orders this wave's LDS writes before its later LDS reads (LDS is in order
// within a wave; this keeps the compiler from moving accesses across)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Force kernels visit E_i in ascending index order (so that sums do not
// depend on the order atomics filled the row).  Rows of up to SPH_ELDS
// entries are ranked in LDS by the particle's lane group inside the force
// kernel; with more slots the rows are sorted in memory beforehand.
#ifndef SPH_ELDS
#define SPH_ELDS 128
#endif
template <int G>
__device__ __forceinline__ void erow_sort_lds(const int32_t *__restrict__ erow, int ne, int lane,
                                              int32_t *raw, int32_t *srt)
{
    wave_lds_sync();   // the group's reads of the previous row are behind us
    for (int e = lane; e < ne; e += G) raw[e] = erow[e];
    wave_lds_sync();
    for (int e = lane; e < ne; e += G) {
        const int v = raw[e];
        int rank = 0;
        for (int f = 0; f < ne; ++f) {
            const int u = raw[f];
            rank += (u < v) | ((u == v) & (f < e));
        }
        srt[rank] = v;
    }
    wave_lds_sync();
}

// Complement rows: i goes into E_j when j is in L_i but i is not in L_j,
// i.e. r_ij^2 >= (2 h_j)^2 (the same exact test j's own gather used).
// Slots come from an integer atomic (row j at eidx + j * slots); rows past
// `slots` are counted.
__device__ __forceinline__ void extra_append(int j, int i, int32_t *__restrict__ ecnt,
                                             int32_t *__restrict__ eidx, int slots,
                                             int64_t &appended, int64_t &dropped)
{
    int k = atomicAdd(&ecnt[j], 1);
    if (k < slots) eidx[(int64_t)j * slots + k] = i;
    else if (k == slots) ++dropped;   // count each overflowing row once
    ++appended;
}

// The same append in two parts for a batch of pairs: the slot is taken by an
// atomic (extra_take) and the entry stored (extra_put) after the batch's
// arithmetic, so that the atomic's round trip overlaps it
__device__ __forceinline__ int extra_take(int j, int32_t *__restrict__ ecnt)
{
    return atomicAdd(&ecnt[j], 1);
}
__device__ __forceinline__ void extra_put(int j, int k, int i, int32_t *__restrict__ eidx,
                                          int slots, int64_t &appended, int64_t &dropped)
{
    if (k < slots) eidx[(int64_t)j * slots + k] = i;
    else if (k == slots) ++dropped;
    ++appended;
}

// r^2 = (dx*dx + dy*dy) + dz*dz, each operation rounded on its own
__device__ __forceinline__ double exact_r2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    double ab = a + b;
    return ab + c;
}

// Reciprocal and inverse square root for the pair sums (x positive and
// normal): the hardware estimate refined by two Newton-Raphson steps,
// y <- y + y (1 - x y) and y <- y + (y / 2)(1 - x y^2).  Each step squares
// the relative error, so the result is within a couple of ulps of the
// correctly rounded value -- far inside the pair sums' rounding -- for a
// third of the instructions of an IEEE division or square root.  The
// neighbour search never uses these: its decisions take exact r^2.
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// integer cell index in [0, 1023] of v within [lo, lo + L]
__device__ __forceinline__ int cell10(double v, double lo, double L)
{
#pragma clang fp contract(off)
    double w = L / 1024.0;
    if (!(w > 0.0)) return 0;
    double t = (v - lo) / w;
    if (!(t >= 0.0)) return 0;
    if (!(t < 1024.0)) return 1023;
    return (int)t;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t morton(uint32_t gx, uint32_t gy, uint32_t gz)
{
    return spread3(gx) | (spread3(gy) << 1) | (spread3(gz) << 2);
}

// inverse of spread3: bits 0, 3, 6, ... of v packed into bits 0, 1, 2, ...
__device__ __forceinline__ uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0x030000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

#define SPH_PI 3.14159265358979323846

// sinc(x) = sin(x)/x and its derivative on 0 <= x <= pi as series in x^2,
// sum_k (-1)^k x^2k / (2k+1)! and sum_k>=1 (-1)^k 2k x^(2k-1) / (2k+1)!,
// terms to k = 13 and 14 (the next term is below 1e-17 at x = pi): no
// division or trigonometric call in the pair loops
__device__ __forceinline__ double sinc_d(double x)
{
    const double x2 = x * x;
    double s = -9.183689863795546e-29;
    s = s * x2 + 6.446950284384474e-26;
    s = s * x2 + -3.868170170630684e-23;
    s = s * x2 + 1.9572941063391263e-20;
    s = s * x2 + -8.22063524662433e-18;
    s = s * x2 + 2.8114572543455206e-15;
    s = s * x2 + -7.647163731819816e-13;
    s = s * x2 + 1.6059043836821613e-10;
    s = s * x2 + -2.505210838544172e-08;
    s = s * x2 + 2.7557319223985893e-06;
    s = s * x2 + -0.0001984126984126984;
    s = s * x2 + 0.008333333333333333;
    s = s * x2 + -0.16666666666666666;
    s = s * x2 + 1.0;
    return s;
}
__device__ __forceinline__ double sinc_deriv_d(double x)
{
    const double x2 = x * x;
    double d = 3.166789608205361e-30;
    d = d * x2 + -2.387759364586842e-27;
    d = d * x2 + 1.5472680682522736e-24;
    d = d * x2 + -8.509974375387505e-22;
    d = d * x2 + 3.9145882126782523e-19;
    d = d * x2 + -1.4797143443923793e-16;
    d = d * x2 + 4.498331606952833e-14;
    d = d * x2 + -1.0706029224547743e-11;
    d = d * x2 + 1.9270852604185937e-09;
    d = d * x2 + -2.505210838544172e-07;
    d = d * x2 + 2.2045855379188714e-05;
    d = d * x2 + -0.0011904761904761906;
    d = d * x2 + 0.03333333333333333;
    d = d * x2 + -0.3333333333333333;
    return d * x;
}

// Kernel W(r, h) and dW/dr from r and 1/h (fields; rounding order free);
// knorm is B_5 of the sinc kernel (unused by the others)
template <int KER>
__device__ __forceinline__ double kern_w(double r, double inv_h, double knorm)
{
    const double q = r * inv_h;
    const double ih3 = inv_h * inv_h * inv_h;
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        if (!(q < 2.0)) return 0.0;
        const double t = 1.0 - 0.5 * q, t2 = t * t;
        return (21.0 / (16.0 * SPH_PI)) * ih3 * (t2 * t2) * (2.0 * q + 1.0);
    } else if constexpr (KER == SPH_KERNEL_SINC5) {
        if (!(q < 2.0)) return 0.0;
        const double s = sinc_d(0.5 * SPH_PI * q), s2 = s * s;
        return knorm * ih3 * (s2 * s2 * s);
    } else {
        double w;
        if (q < 1.0) w = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
        else if (q < 2.0) { double t = 2.0 - q; w = 0.25 * t * t * t; }
        else w = 0.0;
        return (1.0 / SPH_PI) * ih3 * w;
    }
}

template <int KER>
__device__ __forceinline__ double kern_dwdr(double r, double inv_h, double knorm)
{
    const double q = r * inv_h;
    const double ih2 = inv_h * inv_h;
    if constexpr (KER == SPH_KERNEL_WENDLAND) {
        if (!(q < 2.0)) return 0.0;
        const double t = 1.0 - 0.5 * q;
        return (21.0 / (16.0 * SPH_PI)) * (ih2 * ih2) * (-5.0 * q) * (t * t * t);
    } else if constexpr (KER == SPH_KERNEL_SINC5) {
        if (!(q < 2.0)) return 0.0;
        const double x = 0.5 * SPH_PI * q;
        const double s = sinc_d(x), s2 = s * s;
        return knorm * (ih2 * ih2) * (5.0 * (s2 * s2) * sinc_deriv_d(x) * (0.5 * SPH_PI));
    } else {
        double w;
        if (q < 1.0) w = q * (-3.0 + 2.25 * q);
        else if (q < 2.0) { double t = 2.0 - q; w = -0.75 * t * t; }
        else w = 0.0;
        return (1.0 / SPH_PI) * (ih2 * ih2) * w;
    }
}

#define SPH_DISPATCH_KER(k, LAUNCH)                                              \
    switch (k) {                                                                 \
    case SPH_KERNEL_WENDLAND: { constexpr int KER = SPH_KERNEL_WENDLAND; LAUNCH; } break; \
    case SPH_KERNEL_SINC5: { constexpr int KER = SPH_KERNEL_SINC5; LAUNCH; } break;       \
    default: { constexpr int KER = SPH_KERNEL_M4; LAUNCH; } break;                        \
    }

// wave and block reductions
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// one atomic per block for an int64 counter (deterministic total)
__device__ __forceinline__ void block_add_i64(int64_t v, int64_t *addr)
{
    __shared__ int64_t part[SPH_BLOCK / 64];
    v = wave_sum_i64(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
        if (t) atomicAdd((unsigned long long *)addr, (unsigned long long)t);
    }
    __syncthreads();  // the shared slots are reused by the next call
}

// one block total added to two counters (one atomic each)
__device__ __forceinline__ void block_add2_i64(int64_t v, int64_t *a, int64_t *b)
{
    __shared__ int64_t part[SPH_BLOCK / 64];
    v = wave_sum_i64(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
        if (t) {
            atomicAdd((unsigned long long *)a, (unsigned long long)t);
            atomicAdd((unsigned long long *)b, (unsigned long long)t);
        }
    }
    __syncthreads();
}

#endif  // __HIPCC__
