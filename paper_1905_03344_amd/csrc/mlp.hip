// Learned smoothing length: a 6-64-64-1 tanh MLP on bf16 MFMA.
//
// Features of particle i (from the state before the h iteration):
//   f1 = log h, f2 = N/100 - 1, f3 = log(rho h^3 / m), f4 = dt (div v),
//   f5 = dt |v| / h, f6 = dt c / h,  c = sqrt(gamma (gamma - 1) u),
// standardised z = (f - mean) / std in FP64 and rounded to bfloat16 (round
// to nearest even, from the double).  Weights are bf16, biases FP32, sums FP32
// (MFMA), tanh FP32; each hidden activation is rounded to bf16 before the
// next layer.  Output y = log(h_new / h); the predicted h is
// h exp(clamp(y, -1/2, 1/2)).
//
// MFMA v_mfma_f32_16x16x16_bf16, one wave, lane l (v = 0..3):
//   A[i][k]: lane holds A[l%16][4(l/16)+v]
//   B[k][j]: lane holds B[4(l/16)+v][l%16]
//   D[i][j]: lane holds D[4(l/16)+v][l%16]
// Units are rows (M), particles columns (N): a layer's D tiles, activated
// and rounded, are the next layer's B operands as they stand.
#include "sph_internal.h"

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 b2_t __attribute__((ext_vector_type(2)));

#define MLP_WAVES_PER_BLOCK (SPH_BLOCK / 64)

#define MLP_W1 0
#define MLP_B1 384
#define MLP_W2 448
#define MLP_B2 4544
#define MLP_W3 4608
#define MLP_B3 4672

__device__ __forceinline__ f4_t mfma(s4_t a, s4_t b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// bfloat16 bits of a float, round to nearest even
__device__ __forceinline__ uint16_t bf16_bits_f(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)(b >> 16);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
// bfloat16 bits of a double rounded directly (8 significant bits, ties even)
__device__ __forceinline__ uint16_t bf16_bits_d(double v)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    if ((b & 0x7ff0000000000000ull) != 0x7ff0000000000000ull) {
        b += 0x00000FFFFFFFFFFFull + ((b >> 45) & 1ull);
        b &= ~0x00001FFFFFFFFFFFull;
    }
    float f = (float)__longlong_as_double((long long)b);   // exact
    return (uint16_t)(__float_as_uint(f) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// four FP32 values rounded to bfloat16 (nearest, ties even) as an MFMA operand:
// gfx950 converts two per instruction (v_cvt_pk_bf16_f32), the same rounding
// as bf16_bits_f for finite values
__device__ __forceinline__ s4_t bf16x4(float a, float b, float c, float d)
{
    const b2_t lo = __builtin_convertvector((f2_t){a, b}, b2_t);
    const b2_t hi = __builtin_convertvector((f2_t){c, d}, b2_t);
    const uint2 u = make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
    return __builtin_bit_cast(s4_t, u);
}

struct MlpDev {
    const float *master;        // 4673 FP32 parameters
    const uint16_t *wb;         // bf16 weights: W1 (64x6), W2 (64x64), W3 (64), as in master
    const double *norm;         // mean[6], std[6]
};

// weight operands of one wave (registers)
struct MlpRegs {
    s4_t w1[4];        // A of layer 1, unit tile t: W1[16t + l%16][4(l/16)+v]
    s4_t w2[4][4];     // A of layer 2, [mt][kt]: W2[16mt + l%16][16kt + 4(l/16)+v]
    s4_t w3[4];        // A of layer 3 (row 0 = W3): [kt]
    float b1[4][4];    // bias of unit 16t + 4(l/16) + v
    float b2[4][4];
    float b3;
};

__device__ __forceinline__ void mlp_load_regs(const MlpDev &M, MlpRegs &R)
{
    const int l = threadIdx.x & 63;
    const int r = l & 15, g = l >> 4;
    for (int t = 0; t < 4; ++t) {
        for (int v = 0; v < 4; ++v) {
            int f = 4 * g + v;
            R.w1[t][v] = f < 6 ? (short)M.wb[MLP_W1 + (16 * t + r) * 6 + f] : (short)0;
            R.b1[t][v] = M.master[MLP_B1 + 16 * t + 4 * g + v];
            R.b2[t][v] = M.master[MLP_B2 + 16 * t + 4 * g + v];
            R.w3[t][v] = r == 0 ? (short)M.wb[MLP_W3 + 16 * t + 4 * g + v] : (short)0;
        }
        for (int kt = 0; kt < 4; ++kt)
            for (int v = 0; v < 4; ++v)
                R.w2[t][kt][v] = (short)M.wb[MLP_W2 + (16 * t + r) * 64 + 16 * kt + 4 * g + v];
    }
    R.b3 = M.master[MLP_B3];
}

// tanh in FP32, written from the function itself: for |x| < 0.625 the odd
// polynomial x (1 + s P(s)), s = x^2, P of degree 4 fitted to (tanh(x)/x - 1)/s
// on that interval (relative error below 2e-7 in FP32 arithmetic); above it
// 1 - 2 / (1 + e^{2|x|}) with the hardware exp2 and reciprocal (absolute error
// below 2e-7 where tanh > 0.55), sign restored; e^{2|x|} = inf gives 1.
// Activations are rounded to bfloat16 (relative half-ulp 2^-9) afterwards.
__device__ __forceinline__ float tanh_f(float x)
{
    const float ax = fabsf(x);
    const float s = x * x;
    float p = -0.005710217636078596f;
    p = p * s + 0.02064412832260132f;
    p = p * s - 0.05374139919877052f;
    p = p * s + 0.13331463932991028f;
    p = p * s - 0.3333328366279602f;
    const float small = x + x * (s * p);
    const float e = __builtin_amdgcn_exp2f(ax * 2.8853900817779268f);   // e^{2|x|}
    const float big = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
    return ax < 0.625f ? small : copysignf(big, x);
}

// forward of one tile of 16 particles; x = this lane's B operand of layer 1
// (features 4(l/16)+v of particle l%16, bf16 bits, zero beyond 6).
// Returns y of particle l%16 in every lane; a1/a2 (FP32 activations) and
// h1/h2 (their bf16 operands) are kept for the backward pass.
__device__ __forceinline__ float mlp_tile_forward(const MlpRegs &R, s4_t x, float a1[4][4],
                                                  s4_t h1[4], float a2[4][4], s4_t h2[4])
{
    const int l = threadIdx.x & 63;
    for (int t = 0; t < 4; ++t) {
        f4_t d = {0.f, 0.f, 0.f, 0.f};
        d = mfma(R.w1[t], x, d);
        for (int v = 0; v < 4; ++v) a1[t][v] = tanh_f(d[v] + R.b1[t][v]);
        h1[t] = bf16x4(a1[t][0], a1[t][1], a1[t][2], a1[t][3]);
    }
    for (int mt = 0; mt < 4; ++mt) {
        f4_t d = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < 4; ++kt) d = mfma(R.w2[mt][kt], h1[kt], d);
        for (int v = 0; v < 4; ++v) a2[mt][v] = tanh_f(d[v] + R.b2[mt][v]);
        h2[mt] = bf16x4(a2[mt][0], a2[mt][1], a2[mt][2], a2[mt][3]);
    }
    f4_t d = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < 4; ++kt) d = mfma(R.w3[kt], h2[kt], d);
    // row 0 of D lives in lanes 0..15, component 0
    float y = __shfl(d[0], l & 15, 64) + R.b3;
    return y;
}

// standardised features of particle p as this lane's layer-1 operand
__device__ __forceinline__ s4_t feature_operand(const double *f6, const double *norm, bool valid)
{
    const int g = (threadIdx.x & 63) >> 4;
    s4_t x;
    for (int v = 0; v < 4; ++v) {
        int f = 4 * g + v;
        double z = 0.0;
        if (valid && f < 6) z = (f6[f] - norm[f]) / norm[6 + f];
        x[v] = f < 6 ? (short)bf16_bits_d(z) : (short)0;
    }
    return x;
}

// raw features in FP64 from the state
__device__ __forceinline__ void raw_features(int64_t i, const double *__restrict__ h,
                                             const int32_t *__restrict__ nc,
                                             const double *__restrict__ rho,
                                             const double *__restrict__ divv,
                                             const double *__restrict__ m,
                                             const double *__restrict__ vx,
                                             const double *__restrict__ vy,
                                             const double *__restrict__ vz,
                                             const double *__restrict__ u, double gamma, double dt,
                                             double f[6])
{
    double hi = h[i];
    double vv = sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    double c = sqrt(gamma * (gamma - 1.0) * u[i]);
    f[0] = log(hi);
    f[1] = (double)nc[i] / 100.0 - 1.0;
    f[2] = log(rho[i] * hi * hi * hi / m[i]);
    f[3] = dt * divv[i];
    f[4] = dt * vv / hi;
    f[5] = dt * c / hi;
}

// ---------------------------------------------------------------------------
// step use: features -> MLP -> predicted h.  A wave takes 64 particles at a
// time: each lane forms one particle's standardised bf16 features (FP64
// logs, roots and divisions once per particle) into LDS, then the four
// tiles of 16 particles go through the network.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_predict(
    int64_t n, MlpDev M, const double *__restrict__ h, const int32_t *__restrict__ nc,
    const double *__restrict__ rho, const double *__restrict__ divv, const double *__restrict__ m,
    const double *__restrict__ vx, const double *__restrict__ vy, const double *__restrict__ vz,
    const double *__restrict__ u, double gamma, const double *__restrict__ dtp,
    double *__restrict__ h_try, float *__restrict__ y_out)
{
    __shared__ uint16_t xs[MLP_WAVES_PER_BLOCK][64][8];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    MlpRegs R;
    mlp_load_regs(M, R);
    const double dt = *dtp;
    const int64_t nchunks = (n + 63) / 64;
    for (int64_t ch = wave; ch < nchunks; ch += nwaves) {
        const int64_t p = ch * 64 + l;
        const bool valid = p < n;
        double f[6] = {0, 0, 0, 0, 0, 0};
        if (valid) {
            raw_features(p, h, nc, rho, divv, m, vx, vy, vz, u, gamma, dt, f);
            for (int k = 0; k < 6; ++k) f[k] = (double)(float)f[k];
        }
        for (int k = 0; k < 6; ++k)
            xs[w][l][k] = valid ? bf16_bits_d((f[k] - M.norm[k]) / M.norm[6 + k]) : (uint16_t)0;
        xs[w][l][6] = 0;
        xs[w][l][7] = 0;
        wave_lds_sync();
        for (int t = 0; t < 4; ++t) {
            const int q = 16 * t + (l & 15);
            s4_t x;
            for (int v = 0; v < 4; ++v) x[v] = (short)xs[w][q][(4 * g + v) & 7];
            if (g >= 2) x = s4_t{0, 0, 0, 0};
            float a1[4][4], a2[4][4];
            s4_t h1[4], h2[4];
            const float y = mlp_tile_forward(R, x, a1, h1, a2, h2);
            const int64_t pt = ch * 64 + q;
            if (l < 16 && pt < n) {
                const double yc = fmin(fmax((double)y, -0.5), 0.5);
                h_try[pt] = h[pt] * exp(yc);
                if (y_out) y_out[pt] = y;
            }
        }
        wave_lds_sync();
    }
}

// raw features for harvesting (FP32, 8 per particle, last two zero)
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_features(
    int64_t n, const double *__restrict__ h, const int32_t *__restrict__ nc,
    const double *__restrict__ rho, const double *__restrict__ divv, const double *__restrict__ m,
    const double *__restrict__ vx, const double *__restrict__ vy, const double *__restrict__ vz,
    const double *__restrict__ u, double gamma, const double *__restrict__ dtp,
    float *__restrict__ feat)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double f[6];
    raw_features(i, h, nc, rho, divv, m, vx, vy, vz, u, gamma, *dtp, f);
    for (int k = 0; k < 6; ++k) feat[i * 8 + k] = (float)f[k];
    feat[i * 8 + 6] = 0.0f;
    feat[i * 8 + 7] = 0.0f;
}

// training targets: y = log(h_now / h_then), h_then = exp(feature 1); with
// centre, h_now is replaced by h_c = h_now (n_target / N_now)^(1/3), the
// band centre estimated from the solved h and its count (counts scale with
// h^3 where the particle distribution is smooth on the scale of h)
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_targets(int64_t n, const double *__restrict__ h,
                                                           const int32_t *__restrict__ nc,
                                                           int n_target, int centre,
                                                           const float *__restrict__ feat,
                                                           float *__restrict__ target)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y = log(h[i]) - (double)feat[i * 8];
    if (centre && nc[i] > 0) y += log((double)n_target / (double)nc[i]) / 3.0;
    target[i] = (float)y;
}

// forward on raw FP32 feature rows (8 per particle)
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_forward(int64_t n, MlpDev M,
                                                           const float *__restrict__ feat,
                                                           float *__restrict__ y_out,
                                                           uint16_t *__restrict__ h1_out,
                                                           uint16_t *__restrict__ h2_out)
{
    const int l = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    MlpRegs R;
    mlp_load_regs(M, R);
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t p = t * 16 + (l & 15);
        const bool valid = p < n;
        double f[6] = {0, 0, 0, 0, 0, 0};
        if (valid)
            for (int k = 0; k < 6; ++k) f[k] = (double)feat[p * 8 + k];
        s4_t x = feature_operand(f, M.norm, valid);
        float a1[4][4], a2[4][4];
        s4_t h1[4], h2[4];
        float y = mlp_tile_forward(R, x, a1, h1, a2, h2);
        if (valid) {
            if (l < 16) y_out[p] = y;
            const int g = l >> 4;
            for (int tt = 0; tt < 4; ++tt)
                for (int v = 0; v < 4; ++v) {
                    int unit = 16 * tt + 4 * g + v;
                    if (h1_out) h1_out[p * 64 + unit] = (uint16_t)h1[tt][v];
                    if (h2_out) h2_out[p * 64 + unit] = (uint16_t)h2[tt][v];
                }
        }
    }
}

// ---------------------------------------------------------------------------
// training: forward + backward of the mean squared error over a batch.
// Each wave owns a fixed set of tiles and writes one partial gradient row;
// rows are reduced in index order afterwards (deterministic).
// ---------------------------------------------------------------------------
#define MLP_TRAIN_WAVES SPH_MLP_TRAIN_WAVES
#define MLP_NP SPH_MLP_NPARAM
#define MLP_ROW SPH_MLP_ROW

// FP32 value split into two bf16 operands: v ~ hi + lo
__device__ __forceinline__ void split_bf16(float v, short &hi, short &lo)
{
    uint16_t h = bf16_bits_f(v);
    hi = (short)h;
    lo = (short)bf16_bits_f(v - bf16_val(h));
}

struct TrainLds {
    float d2[64][17];   // [unit][particle]
    float h1[64][17];
    float d1[64][17];
    float xs[16][17];   // [particle][feature]
};

// batch element p is row rows[row0 + p] (rows NULL: row0 + p)
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_train(int64_t n, MlpDev M,
                                                         const float *__restrict__ feat,
                                                         const float *__restrict__ target,
                                                         const int32_t *__restrict__ rows,
                                                         int64_t row0, float *__restrict__ part)
{
    __shared__ TrainLds lds[MLP_WAVES_PER_BLOCK];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int r = l & 15, g = l >> 4;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    TrainLds &L = lds[w];
    MlpRegs R;
    mlp_load_regs(M, R);
    // A operand of d1 = W2^T d2: [kt][ot] holds W2[16ot + 4(l/16)+v][16kt + l%16]
    s4_t w2t[4][4];
    for (int kt = 0; kt < 4; ++kt)
        for (int ot = 0; ot < 4; ++ot)
            for (int v = 0; v < 4; ++v)
                w2t[kt][ot][v] = (short)M.wb[MLP_W2 + (16 * ot + 4 * g + v) * 64 + 16 * kt + r];
    float w3v[4][4];   // W3 (bf16 value) of unit 16t + 4(l/16) + v
    for (int t = 0; t < 4; ++t)
        for (int v = 0; v < 4; ++v) w3v[t][v] = bf16_val(M.wb[MLP_W3 + 16 * t + 4 * g + v]);

    f4_t gw2[4][4];    // D tiles of dL/dW2: [ot][kt]
    f4_t gw1[4];       // D tiles of dL/dW1: [kt] (features in columns)
    for (int a = 0; a < 4; ++a) {
        gw1[a] = (f4_t){0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 4; ++b) gw2[a][b] = (f4_t){0.f, 0.f, 0.f, 0.f};
    }
    float gw3[4][4], gb2[4][4], gb1[4][4];
    for (int a = 0; a < 4; ++a)
        for (int v = 0; v < 4; ++v) gw3[a][v] = gb2[a][v] = gb1[a][v] = 0.f;
    float gb3 = 0.f, loss = 0.f;
    const float scale = 2.0f / (float)n;

    const int64_t ntiles = (n + 15) / 16;
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t p = t * 16 + r;
        const bool valid = p < n;
        const int64_t row = valid ? (rows ? (int64_t)rows[row0 + p] : row0 + p) : 0;
        double f[6] = {0, 0, 0, 0, 0, 0};
        if (valid)
            for (int k = 0; k < 6; ++k) f[k] = (double)feat[row * 8 + k];
        s4_t x = feature_operand(f, M.norm, valid);
        float a1[4][4], a2[4][4];
        s4_t h1[4], h2[4];
        float y = mlp_tile_forward(R, x, a1, h1, a2, h2);
        float dy = 0.f;
        if (valid) {
            float e = y - target[row];
            dy = scale * e;
            if (g == 0) loss += e * e;
        }
        if (g == 0) gb3 += dy;
        // layer 3 and the error at layer 2: d2 = dy W3 (1 - a2^2)
        float d2[4][4];
        for (int mt = 0; mt < 4; ++mt)
            for (int v = 0; v < 4; ++v) {
                gw3[mt][v] += dy * bf16_val((uint16_t)h2[mt][v]);
                float dd = dy * w3v[mt][v] * (1.f - a2[mt][v] * a2[mt][v]);
                d2[mt][v] = dd;
                gb2[mt][v] += dd;
            }
        // d1 = (W2^T d2) (1 - a1^2): B operand = d2 in D layout, split hi/lo
        s4_t d2hi[4], d2lo[4];
        for (int ot = 0; ot < 4; ++ot)
            for (int v = 0; v < 4; ++v) {
                short hi, lo;
                split_bf16(d2[ot][v], hi, lo);
                d2hi[ot][v] = hi;
                d2lo[ot][v] = lo;
            }
        float d1[4][4];
        for (int kt = 0; kt < 4; ++kt) {
            f4_t acc = {0.f, 0.f, 0.f, 0.f};
            for (int ot = 0; ot < 4; ++ot) {
                acc = mfma(w2t[kt][ot], d2hi[ot], acc);
                acc = mfma(w2t[kt][ot], d2lo[ot], acc);
            }
            for (int v = 0; v < 4; ++v) {
                float dd = acc[v] * (1.f - a1[kt][v] * a1[kt][v]);
                d1[kt][v] = dd;
                gb1[kt][v] += dd;
            }
        }
        // transposes through LDS for the weight gradients (contraction over
        // the 16 particles of the tile)
        __builtin_amdgcn_wave_barrier();
        for (int tt = 0; tt < 4; ++tt)
            for (int v = 0; v < 4; ++v) {
                int unit = 16 * tt + 4 * g + v;
                L.d2[unit][r] = d2[tt][v];
                L.h1[unit][r] = bf16_val((uint16_t)h1[tt][v]);
                L.d1[unit][r] = d1[tt][v];
            }
        for (int v = 0; v < 4; ++v) {
            int fidx = 4 * g + v;
            L.xs[r][fidx] = bf16_val((uint16_t)x[v]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // dW2[o][k] += sum_p d2[o][p] h1[k][p]: A = d2 [o x p], B = h1^T [p x k]
        s4_t bh[4];
        for (int kt = 0; kt < 4; ++kt)
            for (int v = 0; v < 4; ++v) bh[kt][v] = (short)bf16_bits_f(L.h1[16 * kt + r][4 * g + v]);
        for (int ot = 0; ot < 4; ++ot) {
            s4_t ahi, alo;
            for (int v = 0; v < 4; ++v) {
                short hi, lo;
                split_bf16(L.d2[16 * ot + r][4 * g + v], hi, lo);
                ahi[v] = hi;
                alo[v] = lo;
            }
            for (int kt = 0; kt < 4; ++kt) {
                gw2[ot][kt] = mfma(ahi, bh[kt], gw2[ot][kt]);
                gw2[ot][kt] = mfma(alo, bh[kt], gw2[ot][kt]);
            }
        }
        // dW1[k][f] += sum_p d1[k][p] x[p][f]: A = d1 [k x p], B = x [p x f]
        s4_t bx;
        for (int v = 0; v < 4; ++v) bx[v] = (short)bf16_bits_f(L.xs[4 * g + v][r]);
        for (int kt = 0; kt < 4; ++kt) {
            s4_t ahi, alo;
            for (int v = 0; v < 4; ++v) {
                short hi, lo;
                split_bf16(L.d1[16 * kt + r][4 * g + v], hi, lo);
                ahi[v] = hi;
                alo[v] = lo;
            }
            gw1[kt] = mfma(ahi, bx, gw1[kt]);
            gw1[kt] = mfma(alo, bx, gw1[kt]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // per-unit sums over the 16 particle lanes of each group
    for (int a = 0; a < 4; ++a)
        for (int v = 0; v < 4; ++v) {
            float s3 = gw3[a][v], s2 = gb2[a][v], s1 = gb1[a][v];
            for (int o = 1; o < 16; o <<= 1) {
                s3 += __shfl_xor(s3, o, 64);
                s2 += __shfl_xor(s2, o, 64);
                s1 += __shfl_xor(s1, o, 64);
            }
            gw3[a][v] = s3;
            gb2[a][v] = s2;
            gb1[a][v] = s1;
        }
    for (int o = 1; o < 64; o <<= 1) {
        gb3 += __shfl_xor(gb3, o, 64);
        loss += __shfl_xor(loss, o, 64);
    }
    float *row = part + wave * MLP_ROW;
    // D layout of gradient tiles: lane holds [4(l/16)+v][l%16]
    for (int ot = 0; ot < 4; ++ot)
        for (int kt = 0; kt < 4; ++kt)
            for (int v = 0; v < 4; ++v)
                row[MLP_W2 + (16 * ot + 4 * g + v) * 64 + 16 * kt + r] = gw2[ot][kt][v];
    for (int kt = 0; kt < 4; ++kt)
        for (int v = 0; v < 4; ++v)
            if (r < 6) row[MLP_W1 + (16 * kt + 4 * g + v) * 6 + r] = gw1[kt][v];
    if (r == 0)
        for (int a = 0; a < 4; ++a)
            for (int v = 0; v < 4; ++v) {
                int unit = 16 * a + 4 * g + v;
                row[MLP_W3 + unit] = gw3[a][v];
                row[MLP_B2 + unit] = gb2[a][v];
                row[MLP_B1 + unit] = gb1[a][v];
            }
    if (l == 0) {
        row[MLP_B3] = gb3;
        row[MLP_NP] = loss / (float)n;
    }
}

// fixed-order sum of the partial rows: grad[k] = sum_w part[w][k].  A block
// takes 32 columns; its 8 slices of 32 threads sum the rows w = q, q + 8, ...
// of their slice q in order, and the 8 slice sums are added as a fixed tree.
#define MLP_RED_COLS 32
#define MLP_RED_SLICES (SPH_BLOCK / MLP_RED_COLS)
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_reduce(const float *__restrict__ part, int nrows,
                                                          float *__restrict__ grad,
                                                          float *__restrict__ loss_out)
{
    __shared__ float sh[MLP_RED_SLICES][MLP_RED_COLS];
    const int c = threadIdx.x % MLP_RED_COLS, q = threadIdx.x / MLP_RED_COLS;
    const int k = blockIdx.x * MLP_RED_COLS + c;
    float s = 0.f;
    if (k <= MLP_NP)
        for (int w = q; w < nrows; w += MLP_RED_SLICES) s += part[(int64_t)w * MLP_ROW + k];
    sh[q][c] = s;
    __syncthreads();
    for (int h = MLP_RED_SLICES / 2; h > 0; h >>= 1) {
        if (q < h) sh[q][c] += sh[q + h][c];
        __syncthreads();
    }
    if (q == 0 && k <= MLP_NP) {
        grad[k] = sh[0][c];   // grad[MLP_NP] = loss
        if (k == MLP_NP && loss_out) *loss_out = sh[0][c];
    }
}

// Feature standardisation: FP64 mean and population standard deviation of
// each of the 6 features over n rows, in a fixed reduction order (block b
// takes a fixed contiguous chunk; partials summed in block order).
#define MLP_NORM_BLOCKS 256

__global__ __launch_bounds__(SPH_BLOCK) void k_norm_partial(const float *__restrict__ feat, int64_t n,
                                                            const double *__restrict__ mean,
                                                            double *__restrict__ part)
{
    __shared__ double sh[6][SPH_BLOCK];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t a = blockIdx.x * chunk;
    const int64_t b = a + chunk < n ? a + chunk : n;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
        for (int k = 0; k < 6; ++k) {
            double v = (double)feat[i * 8 + k];
            if (mean) {
                v -= mean[k];
                v *= v;
            }
            acc[k] += v;
        }
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = SPH_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// phase 0: norm[k] = mean; phase 1: norm[6 + k] = std (1 where it is 0)
__global__ void k_norm_final(const double *__restrict__ part, int nb, int64_t n,
                             double *__restrict__ norm, int phase)
{
    int k = threadIdx.x;
    if (k >= 6) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b * 6 + k];
    s /= (double)n;
    if (phase == 0) {
        norm[k] = s;
    } else {
        double sd = sqrt(s);
        norm[6 + k] = sd > 0.0 ? sd : 1.0;
    }
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, then the bf16 copies
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_adam(float *__restrict__ master,
                                                        float *__restrict__ mom,
                                                        float *__restrict__ vel,
                                                        const float *__restrict__ grad,
                                                        uint16_t *__restrict__ wb, float lr,
                                                        float b1, float b2, float eps, float c1,
                                                        float c2)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NP) return;
    float gk = grad[k];
    float m = b1 * mom[k] + (1.0f - b1) * gk;
    float v = b2 * vel[k] + (1.0f - b2) * gk * gk;
    mom[k] = m;
    vel[k] = v;
    float p = master[k] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    master[k] = p;
    wb[k] = bf16_bits_f(p);
}

// bf16 copies of the master parameters
__global__ __launch_bounds__(SPH_BLOCK) void k_mlp_refresh(const float *__restrict__ master,
                                                           uint16_t *__restrict__ wb)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < MLP_NP) wb[k] = bf16_bits_f(master[k]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static MlpDev mlp_dev(sph_ctx *c)
{
    MlpDev M;
    M.master = c->w.mlp_master;
    M.wb = c->w.mlp_wb;
    M.norm = c->w.mlp_norm;
    return M;
}

static unsigned mlp_blocks(int64_t n)
{
    int64_t tiles = (n + 15) / 16;
    int64_t waves = tiles < 8192 ? tiles : 8192;
    return (unsigned)ceil_div(waves, MLP_WAVES_PER_BLOCK);
}

// k_mlp_predict: one wave per 64 particles, at most 8192 waves
static unsigned mlp_predict_blocks(int64_t n)
{
    int64_t chunks = (n + 63) / 64;
    int64_t waves = chunks < 8192 ? chunks : 8192;
    return (unsigned)ceil_div(waves, MLP_WAVES_PER_BLOCK);
}

hipError_t launch_mlp_predict(sph_ctx *c, sph_particles *s, double *h_try)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    hipLaunchKernelGGL(k_mlp_predict, dim3(mlp_predict_blocks(n)), dim3(SPH_BLOCK), 0, c->stream, n,
                       mlp_dev(c), s->h[k], s->nc[k], s->rho[k], s->divv[k], s->m[k], s->pvx,
                       s->pvy, s->pvz, s->pu, c->p.gamma, c->w.dt_cur, h_try, (float *)nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_features(sph_ctx *c, const sph_particles *s, const double *d_dt,
                               float *feat)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    int k = s->cur;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, s->h[k], s->nc[k], s->rho[k], s->divv[k], s->m[k], s->pvx,
                       s->pvy, s->pvz, s->pu, c->p.gamma, d_dt, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_targets(sph_ctx *c, const sph_particles *s, const float *feat,
                              float *target, int centre)
{
    int64_t n = s->n;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)ceil_div(n, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, n, s->h[s->cur], s->nc[s->cur], c->p.n_target, centre, feat,
                       target);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(sph_ctx *c, const float *feat, int64_t n, float *y, uint16_t *h1,
                              uint16_t *h2)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_blocks(n)), dim3(SPH_BLOCK), 0, c->stream, n,
                       mlp_dev(c), feat, y, h1, h2);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(sph_ctx *c, const float *feat, const float *target,
                           const int32_t *rows, int64_t row0, int64_t n, float *grad,
                           float *loss_out)
{
    if (n <= 0) return hipErrorInvalidValue;
    unsigned nb = MLP_TRAIN_WAVES / MLP_WAVES_PER_BLOCK;
    hipLaunchKernelGGL(k_mlp_train, dim3(nb), dim3(SPH_BLOCK), 0, c->stream, n, mlp_dev(c), feat,
                       target, rows, row0, c->w.mlp_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(MLP_NP + 1, MLP_RED_COLS)),
                       dim3(SPH_BLOCK), 0, c->stream, c->w.mlp_part, MLP_TRAIN_WAVES, grad,
                       loss_out);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(sph_ctx *c, const float *grad, double lr, double b1, double b2,
                           double eps, int t)
{
    float c1 = (float)(1.0 - pow(b1, (double)t));
    float c2 = (float)(1.0 - pow(b2, (double)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)ceil_div(MLP_NP, SPH_BLOCK)), dim3(SPH_BLOCK), 0,
                       c->stream, c->w.mlp_master, c->w.mlp_m, c->w.mlp_v, grad, c->w.mlp_wb,
                       (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_refresh(sph_ctx *c)
{
    hipLaunchKernelGGL(k_mlp_refresh, dim3((unsigned)ceil_div(MLP_NP, SPH_BLOCK)), dim3(SPH_BLOCK),
                       0, c->stream, c->w.mlp_master, c->w.mlp_wb);
    return hipGetLastError();
}

hipError_t launch_mlp_fit_norm(sph_ctx *c, const float *feat, int64_t n)
{
    if (n <= 0) return hipErrorInvalidValue;
    double *part = c->w.red_part;   // MLP_NORM_BLOCKS * 6 doubles
    hipLaunchKernelGGL(k_norm_partial, dim3(MLP_NORM_BLOCKS), dim3(SPH_BLOCK), 0, c->stream, feat,
                       n, (const double *)nullptr, part);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, c->stream, part, MLP_NORM_BLOCKS, n,
                       c->w.mlp_norm, 0);
    hipLaunchKernelGGL(k_norm_partial, dim3(MLP_NORM_BLOCKS), dim3(SPH_BLOCK), 0, c->stream, feat,
                       n, (const double *)c->w.mlp_norm, part);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, c->stream, part, MLP_NORM_BLOCKS, n,
                       c->w.mlp_norm, 1);
    return hipGetLastError();
}
