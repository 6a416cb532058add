/*
 * sph.h -- C ABI of libsph, one SPH time step on an AMD MI355X (gfx950).
 *
 * The per-timestep particle loop of the SPH mini-app described in
 * "SPH-EXA: Enhancing the Scalability of SPH codes Via an Exascale-Ready SPH
 * Mini-App" (Guerrera et al., arXiv:1905.03344): neighbour discovery (here a
 * Morton cell list in place of the tree walk of Table 1), smoothing-length
 * update, density sum with standard volume elements (Table 1), equation of
 * state, momentum equation after Rosswog (2009) with Monaghan (1983)
 * artificial viscosity, energy equation, Courant time step and the position
 * and energy update (section "Co-Design of the Mini-App").  The kernel is
 * the M4 cubic spline with support 0 <= r/h <= 2 (the support convention of
 * the Sinc and Wendland kernel equations).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer owned by the caller; the
 *     library never allocates device memory.  Scratch memory is one
 *     caller-allocated workspace of sph_workspace_size() bytes, bound with
 *     sph_bind() together with the HIP stream every call launches on (the
 *     one exception, sph_conservation_noalloc, uses a 64 KiB array the
 *     library's code object holds per GPU).
 *   - Calls are asynchronous on the bound stream and return an int status.
 *     Argument errors are reported at once; conditions found by kernels
 *     (list overflow, non-convergence, non-finite values) are reported by
 *     the next sph_sync().  Nothing throws across the ABI.
 *   - One context per stream; calls on one context must not overlap.
 *   - Particles are structure-of-arrays.  Carried fields come in ping-pong
 *     pairs [2]; member `cur` selects the current buffer.  sph_build_cells()
 *     reorders every carried field from buffer cur into 1-cur and flips cur.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SPH_OK 0
#define SPH_EINVAL (-1)      /* invalid argument */
#define SPH_ENOMEM (-2)      /* workspace too small or not bound */
#define SPH_ECAPACITY (-3)   /* a neighbour list exceeded its capacity (see sph_stats) */
#define SPH_EHIP (-4)        /* HIP runtime error; text in sph_last_error() */
#define SPH_ENONFINITE (-5)  /* non-finite field value (only with check_finite) */
#define SPH_WNOCONV 1        /* warning: some smoothing lengths did not converge */

/* Smoothing kernels of the density and force sums (support 2h, 0 <= v <= 2):
 *   M4        cubic spline, 1/(pi h^3) {1 - 1.5v^2 + 0.75v^3; 0.25(2-v)^3}
 *   WENDLAND  Wendland C2 of the paper's kernel section,
 *             21/(16 pi h^3) (1 - v/2)^4 (2v + 1)
 *   SINC5     the section's sinc family with exponent 5,
 *             B_5/h^3 sinc^5(pi v/2), sinc(x) = sin(x)/x, B_5 normalising
 *             the kernel to one (computed by the library at sph_create)
 * The neighbour search and h iteration do not depend on the kernel. */
#define SPH_KERNEL_M4 0
#define SPH_KERNEL_WENDLAND 1
#define SPH_KERNEL_SINC5 2
#define SPH_FP64 0
#define SPH_MIXED 1
#define SPH_H_PLAIN 0
#define SPH_H_LEARNED 1

/* particle flag bits */
#define SPH_FLAG_NOCONV 1u   /* h iteration ended outside the target band */
#define SPH_FLAG_LEARNED 2u  /* learned h was accepted (no iteration needed) */

typedef struct sph_ctx sph_ctx;

/* Candidate test of the group walk in the neighbour search.  NONE: every
 * candidate of a union tile gets the FP64 r^2 test.  MATRIX: a 64 x 64
 * tile's r^2 - threshold values are first formed as Gram products on the
 * matrix cores (bfloat16 hi/lo splits, FP32 sums) with a band of
 * 2^-11 (U^2 + T) around each threshold; only candidates inside the band
 * or the shell get the FP64 test.  Both give the same sets, counts, order
 * and h bit for bit. */
#define SPH_PREFILTER_NONE 0
#define SPH_PREFILTER_MATRIX 1

/* How the h iteration continues after its first count (speed only: h, counts,
 * sets and rows are the same).  SHELL_FIRST: the first count records the shell
 * |r - 2h| < 2h/24, on which most particles that miss the band converge
 * without another walk; the rest are counted one particle per wave.
 * WORKLIST: the first count records no shell; the particles that miss get one
 * more wave-cooperative count (with the shell) before the per-particle tail.
 * AUTO: WORKLIST from 4,000,000 particles on, else SHELL_FIRST. */
#define SPH_WALK_AUTO 0
#define SPH_WALK_SHELL_FIRST 1
#define SPH_WALK_WORKLIST 2

/* Shell of the learned try (SPH_H_LEARNED; speed only: h, counts, sets, rows
 * and the accepted/fallback split are the same).  NEVER: the try counts at the
 * predicted h without a shell and every miss restarts the plain iteration from
 * h_prev with a new walk.  ALWAYS: the try records the plain first count's
 * shell |r - 2h| < 2h/24 around the predicted h, so that a miss whose h_prev
 * lies inside it iterates on the shell without a walk.  AUTO: the shell when
 * the walk strategy is SHELL_FIRST, n >= 131,072 and more than a tenth of the
 * previous learned h solve's tries missed the band (none on the first). */
#define SPH_TRY_SHELL_AUTO 0
#define SPH_TRY_SHELL_NEVER 1
#define SPH_TRY_SHELL_ALWAYS 2

/* Time integrators of sph_step.  KDK: kick-drift-kick leapfrog (positions,
 * velocities and energy).  AB2: the same positions and velocities, the
 * energy by second-order Adams-Bashforth with a variable step (the paper's
 * energy update, the co-design section names it without a formula):
 *   u^{n+1} = u^n + dt_n [(1 + r/2) du^n - (r/2) du^{n-1}],  r = dt_n/dt_{n-1},
 * computed at the step's start and used as the energy of the force
 * evaluation; the first step after sph_bind or sph_evaluate is the Euler
 * step u + dt du.  du^{n-1} and dt_{n-1} live in the workspace. */
#define SPH_INTEGRATOR_KDK 0
#define SPH_INTEGRATOR_AB2 1

/* Gradient estimator of the momentum and energy sums (A9).  KERNEL: kernel
 * derivatives (the mini-app's, Table 1).  IAD: the integral approach to
 * derivatives that Table 1 lists for SPHYNX and, in development, for the
 * mini-app (Garcia-Senz, Cabezon & Escartin 2012): per particle the moment
 * matrix over its gather set,
 *   tau_i = sum_{j in L_i} (m_j/rho_j) d_ij d_ij^T W(r_ij,h_i),  d_ij = x_j - x_i,
 * its inverse c_i, and grad_i W(r,h_i) replaced by A_i = c_i d_ij W(r_ij,h_i),
 * grad_i W(r,h_j) by A_j = c_j d_ij W(r_ij,h_j).  In the mixed form tau is a
 * compensated FP32 sum, inverted in FP64 and used in FP32. */
#define SPH_GRADIENTS_KERNEL 0
#define SPH_GRADIENTS_IAD 1

/* Volume elements of the density sum (A7).  STANDARD: V_i = m_i / rho_i,
 * rho_i = sum_j m_j W(r_ij, h_i) (the mini-app's, Table 1).  GENERALIZED:
 * the generalized volume elements Table 1 lists for SPHYNX and, in
 * development, for the mini-app (Hopkins 2013; Cabezon, Garcia-Senz &
 * Figueira 2017): weights X_i = (m_i / rho_i)^p from the density of the
 * previous evaluation (p = gve_exponent; sph_evaluate takes the standard
 * density at its h first), Y_i = sum_j X_j W(r_ij, h_i) over L_i and i
 * itself, V_i = X_i / Y_i and rho_i = m_i Y_i / X_i.  The momentum and energy
 * equations are those of the Lagrangian with these volumes (X and h held
 * fixed), with r = X/m and g = P/Y^2:
 *   a_i  = -sum_j m_j [r_i r_j (g_i grad_i W(h_i) + g_j grad_i W(h_j)) + Pi_ij grad W_bar]
 *   du_i =  sum_j m_j [r_i r_j g_i v_ij . grad_i W(h_i) + (Pi_ij/2) v_ij . grad W_bar]
 * (pairwise antisymmetric: momentum and energy are conserved).  Not combined
 * with grad_h or IAD gradients. */
#define SPH_VOLUMES_STANDARD 0
#define SPH_VOLUMES_GENERALIZED 1

typedef struct sph_params {
    int64_t n_max;          /* largest particle count the workspace is sized for */
    int32_t list_stride;    /* K: capacity of each gather set L_i (default 128) */
    int32_t integrator;     /* SPH_INTEGRATOR_KDK (default) or SPH_INTEGRATOR_AB2 */
    int32_t extra_slots;    /* capacity of each complement row E_i (default 48) */
    int32_t walk_prefilter; /* SPH_PREFILTER_MATRIX (default) or SPH_PREFILTER_NONE */
    int32_t periodic[3];    /* 1 = periodic dimension (minimum image, wrap) */
    int32_t kernel;         /* SPH_KERNEL_M4 (default), _WENDLAND or _SINC5 */
    double box_lo[3];       /* box of the periodic dimensions */
    double box_hi[3];
    int32_t n_target;       /* target neighbour count (100) */
    int32_t n_tol;          /* accepted deviation (5) */
    int32_t h_max_iter;     /* iteration cap of the h solve (32) */
    int32_t precision;      /* SPH_FP64 or SPH_MIXED */
    double gamma;           /* adiabatic index (5/3) */
    double av_alpha;        /* artificial viscosity alpha (1) */
    double av_beta;         /* artificial viscosity beta (2) */
    double av_eta2;         /* viscosity softening eta^2 (0.01) */
    double cfl;             /* Courant factor (0.3) */
    int32_t h_mode;         /* SPH_H_PLAIN or SPH_H_LEARNED */
    int32_t check_finite;   /* 1 = count non-finite fields (slower) */
    int32_t max_level;      /* finest Morton level of the cell table, 1..8 */
    int32_t search_div;     /* search cells are at least 2h/search_div wide (1..4, default 2) */
    int32_t grad_h;         /* 1 = grad-h correction terms in A9 (default 0) */
    int32_t gradients;      /* SPH_GRADIENTS_KERNEL (default) or SPH_GRADIENTS_IAD */
    int32_t walk_defer_group; /* first h-iteration round: particles in walk sub-groups of at
                               * most this many (0 = default 4; 1..64) are counted one per
                               * wave afterwards; larger suits strongly clustered inputs.
                               * Speed only: sets, rows, h, counts and fields do not
                               * depend on it. */
    int32_t volumes;        /* SPH_VOLUMES_STANDARD (default) or SPH_VOLUMES_GENERALIZED */
    int32_t walk_strategy;  /* SPH_WALK_AUTO (default), _SHELL_FIRST or _WORKLIST (speed only)*/
    double gve_exponent;    /* p of the generalized weights X = (m/rho)^p, in [0, 1] (0.7) */
    int32_t learned_try_shell; /* SPH_TRY_SHELL_AUTO (default), _NEVER or _ALWAYS */
    int32_t pad1;
} sph_params;

typedef struct sph_particles {
    int64_t n;              /* particle count, <= n_max */
    int32_t cur;            /* current buffer of each pair, 0 or 1 */
    int32_t pad0;
    /* carried fields, ping-pong pairs, each of length n */
    double *x[2], *y[2], *z[2];      /* position */
    double *vx[2], *vy[2], *vz[2];   /* velocity (half-step value inside a step) */
    double *m[2];                    /* mass */
    double *h[2];                    /* smoothing length */
    double *u[2];                    /* specific internal energy */
    double *ax[2], *ay[2], *az[2];   /* acceleration of the last evaluation */
    double *du[2];                   /* du/dt of the last evaluation */
    double *rho[2];                  /* density of the last evaluation */
    double *divv[2];                 /* velocity divergence of the last evaluation */
    int32_t *nc[2];                  /* |L_i|, gather neighbour count */
    int32_t *id[2];                  /* persistent particle id */
    /* single buffers, length n, in the current order */
    double *pvx, *pvy, *pvz, *pu;    /* velocity and energy used by the force evaluation */
    double *p, *c;                   /* pressure, sound speed */
    uint8_t *flags;                  /* SPH_FLAG_* bits */
    uint32_t *key;                   /* sorted 30-bit cell keys (from sph_build_cells) */
    int32_t *perm;                   /* perm[k] = position before the sort of sorted particle k */
} sph_particles;

/* Neighbour lists.  The interaction set of particle i is
 *   S_i = L_i U E_i,   L_i = { j != i : r_ij^2 < (2 h_i)^2 }  (gather set),
 *                      E_i = { j : i in L_j, j not in L_i }    (complement),
 * so that j in S_i <=> i in S_j.  Both parts are stored particle-major: row
 * i of L is idx[i * list_stride + k], k < nc[i] (nc in sph_particles), and
 * row i of E is eidx[i * extra_slots + k], k < ecnt[i].  L_i comes in
 * ascending index order however it was counted (the same row, bit for bit,
 * whatever the walk grouping).  E_i is in no particular order (the force
 * kernel visits each E_i in ascending index order, so results do not depend
 * on it).  All indices refer to the current (sorted) particle order.
 * sph_interaction_csr exports S_i as compressed rows. */
typedef struct sph_nlist {
    int32_t *idx;           /* stride * list_stride entries */
    int64_t stride;         /* rows allocated, >= n (a multiple of 64) */
    int32_t *ecnt;          /* n: |E_i| (entries beyond extra_slots are dropped and counted) */
    int32_t *eidx;          /* stride * extra_slots entries */
} sph_nlist;

typedef struct sph_stats {
    int64_t nonconverged;    /* particles whose h iteration ended outside the band */
    int64_t list_overflow;   /* particles whose |L_i| exceeded list_stride */
    int64_t extra_total;     /* |E| summed over particles */
    int64_t extra_overflow;  /* particles whose E row exceeded extra_slots */
    int64_t nonfinite;       /* non-finite values found (check_finite) */
    int64_t h_counts;        /* neighbour counts taken by the h iteration (all particles) */
    int64_t learned_accepted;/* learned mode: particles whose predicted h was accepted */
    int64_t learned_fallback;/* learned mode: particles that fell back to the iteration */
    int64_t candidates;      /* candidate pairs tested by the h iteration */
    double dt;               /* Courant time step of the last evaluation */
    int64_t candidates_first;/* of those, tested by its first (all-particle) counting pass */
    int64_t iad_singular;    /* IAD: particles whose moment matrix was not invertible */
    int64_t csr_overflow;    /* sph_interaction_csr: entries beyond the caller's capacity */
} sph_stats;

/* Fill *p with the defaults above (n_max and capacities set to 0). */
void sph_default_params(sph_params *p);

/* Validate *p and create a context holding host metadata only.
 * Returns SPH_EINVAL for an invalid parameter (message via *out == NULL:
 * use sph_params_error()). */
int sph_create(const sph_params *p, sph_ctx **out);
void sph_destroy(sph_ctx *ctx);
const char *sph_params_error(void);

/* Bytes of device workspace needed for *p (sort buffers, cell table, scan
 * scratch, reduction partials, status words, MLP buffers). */
int sph_workspace_size(const sph_params *p, size_t *bytes);

/* Bind a caller-owned device workspace and a HIP stream (hipStream_t cast
 * to void*; NULL = the null stream).  Uploads the Hernquist-Katz factor
 * table.  May be called again to rebind. */
int sph_bind(sph_ctx *ctx, void *workspace, size_t bytes, void *stream);

/* A1-A4: bounding box (exact min/max; periodic dimensions use the box),
 * 30-bit Morton cell keys (10 bits per dimension of the cell index in the
 * box), stable LSD radix sort of the keys (ties keep the input order),
 * permutation of every carried field into buffer 1-cur (cur flips), and the
 * cell-start table at level max_level.  Writes s->key and s->perm. */
int sph_build_cells(sph_ctx *ctx, sph_particles *s);

/* A5-A6: smoothing-length iteration per particle from h[cur] (Hernquist &
 * Katz factor until bracketed, then bisection, until |N_i - n_target| <=
 * n_tol, at most h_max_iter counts; otherwise the best h is kept and
 * SPH_FLAG_NOCONV set), with the gather set L_i written in the same pass;
 * then the complement E.  Updates h[cur], nc[cur], flags. */
int sph_find_neighbors(sph_ctx *ctx, sph_particles *s, sph_nlist *nl);

/* A7: rho_i = m_i W(0,h_i) + sum_{j in L_i} m_j W(r_ij,h_i) and
 * divv_i = (1/rho_i) sum_{j in L_i} m_j (v_j - v_i) . grad_i W(r_ij,h_i),
 * with v the predicted velocity (pvx, pvy, pvz).  Writes rho[cur], divv[cur]. */
int sph_density(sph_ctx *ctx, sph_particles *s, const sph_nlist *nl);

/* The interaction sets S_i = L_i U E_i as compressed rows, for callers that
 * take neighbour lists in that form (the per-step neighbour discovery of the
 * mini-app's loop, section "Co-Design of the Mini-App"): d_off[n + 1]
 * (int64, device) receives the row offsets, d_off[n] = sum |S_i|, and
 * d_idx[d_off[i] ..] (int32, device) row i in ascending index order (the
 * current, sorted particle order).  Call after sph_find_neighbors (or a
 * step), before the next sph_build_cells.  Entries at positions >= capacity
 * are not written; they are counted in sph_stats.csr_overflow and make the
 * next sph_sync return SPH_ECAPACITY (d_off is always complete, so a caller
 * can size d_idx from d_off[n] and call again).  Uses the workspace's
 * per-particle scratch; the padded rows of sph_nlist stay as they are. */
int sph_interaction_csr(sph_ctx *ctx, const sph_particles *s, const sph_nlist *nl,
                        int64_t *d_off, int32_t *d_idx, int64_t capacity);

/* With grad_h set, sph_density also forms the grad-h factor of each
 * particle, for h taken as proportional to rho^(-1/3) (Springel & Hernquist
 * 2002: a refinement of the kernel-derivative gradients that Table 1 lists
 * for the mini-app, which the paper does not use itself):
 *   Omega_i = 1 - (1/(3 rho_i)) sum_j m_j (3 W(r_ij,h_i) + r_ij dW/dr(r_ij,h_i)),
 * the sum over L_i and i itself (equal to 1 + h_i/(3 rho_i) sum_j m_j dW/dh).
 * It stays in the workspace; sph_get_omega copies it out. */

/* A8: ideal gas, P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u), u = pu. */
int sph_eos(sph_ctx *ctx, sph_particles *s);

/* A9: over S_i, with grad W_bar = (grad_i W(r,h_i) + grad_i W(r,h_j))/2,
 *   a_i  = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) grad W_bar
 *   du_i =  sum_j m_j (P_i/rho_i^2 + Pi_ij/2) v_ij . grad W_bar
 * Monaghan viscosity Pi_ij for approaching pairs, and the Courant step
 * dt = cfl min_i h_i / (c_i + 1.2 (alpha c_i + beta max_j |mu_ij|)) written
 * to the device scalar *d_dt.  Writes ax, ay, az, du of buffer cur. */
int sph_momentum_energy(sph_ctx *ctx, sph_particles *s, const sph_nlist *nl, double *d_dt);

/* With grad_h set, A9 takes each pressure term with its own particle's
 * gradient and grad-h factor, the viscosity with the averaged gradient:
 *   a_i  = -sum_j m_j [P_i/(Omega_i rho_i^2) grad_i W(r,h_i)
 *                      + P_j/(Omega_j rho_j^2) grad_i W(r,h_j) + Pi_ij grad W_bar]
 *   du_i =  sum_j m_j [P_i/(Omega_i rho_i^2) v_ij . grad_i W(r,h_i)
 *                      + (Pi_ij/2) v_ij . grad W_bar]
 * (pairwise antisymmetric as before, so momentum and energy are conserved). */

/* With gradients = SPH_GRADIENTS_IAD, sph_momentum_energy first forms c_i
 * for every particle (rho from the last sph_eos), then sums
 *   a_i  = -sum_{j in S_i} m_j [f_i A_i + f_j A_j + Pi_ij (A_i + A_j)/2]
 *   du_i =  sum_{j in S_i} m_j [f_i v_ij . A_i + (Pi_ij/2) v_ij . (A_i + A_j)/2]
 * with f = P/rho^2 (P/(Omega rho^2) with grad_h).  A moment matrix whose
 * determinant is not positive and finite counts in sph_stats.iad_singular
 * and makes sph_sync return SPH_ENONFINITE. */

/* Copies Omega of the last sph_density (buffer cur order, n values) to
 * d_omega (device).  Error if the context was created without grad_h. */
int sph_get_omega(sph_ctx *ctx, const sph_particles *s, double *d_omega);

/* A1-A9 at the stored state (pv = v, pu = u): the force evaluation that
 * starts a run.  *d_dt receives the Courant step. */
int sph_evaluate(sph_ctx *ctx, sph_particles *s, sph_nlist *nl, double *d_dt);

/* One kick-drift-kick leapfrog step (A10 around A1-A9):
 *   v += dt/2 a, u += dt/2 du, x += dt v (periodic wrap); sort;
 *   pv = v + dt/2 a, pu = u + dt/2 du; A5-A9 at (x, pv, pu);
 *   v += dt/2 a_new, u += dt/2 du_new.
 * dt > 0 is used as given; dt <= 0 uses the device scalar *d_dt (the
 * Courant step of the previous evaluation).  *d_dt receives the new step. */
int sph_step(sph_ctx *ctx, sph_particles *s, sph_nlist *nl, double dt, double *d_dt);

/* Conservation sums in FP64 with a fixed reduction order:
 * d_out7 = [P_x, P_y, P_z, L_x, L_y, L_z, E], P = sum m v,
 * L = sum m x cross v, E = sum m (v.v/2 + u), over buffer cur. */
int sph_conservation(sph_ctx *ctx, const sph_particles *s, double *d_out7);

/* For callers that cannot allocate device memory or bind a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the conservation sums of sph_conservation without a context.
 * The same kernels, block count and reduction order, hence the same bits;
 * the block partials go to a 64 KiB array the library holds per GPU
 * (1024 blocks x 8 doubles, the most the launch uses for any n, so no n is
 * too large), looked up on the first call on each device.  Launches on
 * `stream` (hipStream_t cast to void*; NULL = the null stream), which must
 * belong to the current device.  Allocates nothing and does not wait.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  s needs x, y, z, vx, vy, vz, m, u of buffer s->cur; d_out7 is a
 * device array of 7 doubles.  Returns SPH_EINVAL for a NULL or inconsistent
 * argument, SPH_EHIP for a runtime error. */
int sph_conservation_noalloc(const sph_particles *s, double *d_out7, void *stream);

/* Wait for the bound stream; fill *st (may be NULL) from the device status
 * words and reset them.  Returns SPH_ECAPACITY on list overflow,
 * SPH_ENONFINITE when non-finite values were counted, SPH_WNOCONV when
 * some h did not converge, SPH_EHIP on a runtime error, else SPH_OK. */
int sph_sync(sph_ctx *ctx, sph_stats *st);

/* Last error message of this context (static storage inside ctx). */
const char *sph_last_error(const sph_ctx *ctx);

/* Copy an internal table into caller device memory dst (for tests):
 * which = 0: cell-start table (int32, 8^max_level + 1 entries),
 *         1: bounding box (6 doubles: lo[3], hi[3]).
 * *needed receives the size in bytes; dst may be NULL to query it. */
int sph_copy_internal(sph_ctx *ctx, int which, void *dst, size_t bytes, size_t *needed);

/* Stage timing with HIP events recorded on the bound stream around each
 * stage of every subsequent call (overhead: two event records per stage).
 * Stages: SPH_STAGE_CELLS (A1-A4), _HSOLVE (A5 and the gather sets),
 * _EXTRA (complement E), _DENSITY (A7), _EOS (A8), _FORCES (A9 + dt),
 * _INTEGRATE (A10 kicks, drift, prediction), _MLP (learned h prediction),
 * _HWALK (the first wave-cooperative counting pass of the h iteration, also
 * counted in _HSOLVE). */
#define SPH_STAGE_CELLS 0
#define SPH_STAGE_HSOLVE 1
#define SPH_STAGE_EXTRA 2
#define SPH_STAGE_DENSITY 3
#define SPH_STAGE_EOS 4
#define SPH_STAGE_FORCES 5
#define SPH_STAGE_INTEGRATE 6
#define SPH_STAGE_MLP 7          /* learned mode: feature build + MLP inference */
#define SPH_STAGE_HWALK 8        /* inside _HSOLVE: the first counting pass alone */
#define SPH_NSTAGES 9

/* enable = 1 clears the accumulators and starts recording; 0 stops. */
int sph_timing(sph_ctx *ctx, int enable);

/* Waits for the bound stream, then writes the summed elapsed milliseconds
 * (ms[k]) and the number of timed intervals (count[k]) of each stage k <
 * nstages since timing was enabled.  Either pointer may be NULL. */
int sph_timing_read(sph_ctx *ctx, double *ms, int64_t *count, int nstages);

/* ------------------------------------------------------------------------
 * Learned smoothing length (production form: h_mode = SPH_H_LEARNED).
 *
 * The paper's h update is an iteration towards a target neighbour count
 * (section "Co-Design of the Mini-App", the smoothing-length step of the
 * per-timestep loop); this form predicts its outcome.  A 6-64-64-1 MLP with
 * tanh hidden layers maps the standardised features of particle i,
 *   f1 = log h_i, f2 = N_i/100 - 1, f3 = log(rho_i h_i^3 / m_i),
 *   f4 = dt (div v)_i, f5 = dt |v_i| / h_i, f6 = dt c_i / h_i,
 * taken from the previous evaluation (h, N, rho, div v) and the predicted
 * state of this step (v = pv, c = sqrt(gamma (gamma-1) pu), dt of the step),
 * to y ~ log(h_new / h_i) (training targets below).  In sph_step (and sph_find_neighbors) the first
 * count of particle i is taken at h_i exp(clamp(y, -1/2, 1/2)); within
 * n_tol of n_target it is accepted (SPH_FLAG_LEARNED), otherwise the plain
 * iteration runs from h_i exactly as in SPH_H_PLAIN.  sph_evaluate always
 * uses the plain iteration (no previous evaluation to take features from).
 *
 * Numerics: features in FP64, rounded to FP32, standardised in FP64
 * z = (f - mean)/std and rounded to bfloat16 (round to nearest even).
 * Weights bfloat16, biases FP32, products summed in FP32 (MFMA), tanh in
 * FP32, hidden activations rounded to bfloat16 before the next layer.
 *
 * Parameters: SPH_MLP_NPARAM floats, [out][in] row-major,
 *   W1[64][6] at 0, b1[64] at 384, W2[64][64] at 448, b2[64] at 4544,
 *   W3[64] at 4608, b3 at 4672.
 * They live in the bound workspace (FP32 master, bf16 copy, Adam moments,
 * the 12 standardisation constants); binding again clears them.
 * Feature rows are SPH_MLP_NFEAT floats: f1..f6 and two zeros.
 * ------------------------------------------------------------------------ */
#define SPH_MLP_NPARAM 4673
#define SPH_MLP_NFEAT 8

/* Upload FP32 parameters (host array of SPH_MLP_NPARAM) and the
 * standardisation constants (host array mean[6], std[6], std > 0; NULL keeps
 * the current ones, zeros and ones after a bind).  Clears the Adam moments
 * and step counter.  Synchronous.  SPH_EINVAL for NULL params or std <= 0. */
int sph_mlp_set_weights(sph_ctx *ctx, const float *params, const double *norm12);

/* Download the FP32 parameters and the standardisation constants to host
 * arrays (either may be NULL).  Synchronous.  SPH_EINVAL before any
 * sph_mlp_set_weights since the bind. */
int sph_mlp_get_weights(sph_ctx *ctx, float *params, double *norm12);

/* Set the standardisation constants from n >= 1 device feature rows: FP64
 * mean and population standard deviation of each feature (1 where it is 0),
 * summed in a fixed order. */
int sph_mlp_fit_norm(sph_ctx *ctx, const float *d_feat, int64_t n);

/* Feature rows [n][SPH_MLP_NFEAT] of the current buffer of *s into d_feat,
 * with dt read from the device scalar *d_dt and v, u from pv, pu. */
int sph_get_features(sph_ctx *ctx, const sph_particles *s, const double *d_dt, float *d_feat);

/* Training sink: while set (both non-NULL), every sph_step writes, in the
 * particle order of that step, the feature rows of its start into
 * d_feat[n][SPH_MLP_NFEAT] and the targets into d_target[n] (n = particles
 * of the step; device arrays of at least n_max rows).  Target modes:
 *   SPH_TARGET_SOLVED:  log(h_new) - f1, the h the iteration settled on;
 *   SPH_TARGET_CENTRED: log(h_c) - f1, h_c = h_new (n_target / N_new)^(1/3),
 *     the solved h moved to the band centre by the h^3 scaling of the count.
 * Any h in the band solves the problem; the centred target leaves the widest
 * margin where the count grows smoothly with h (irregular particle
 * distributions), the solved one suits near-lattice distributions, whose
 * count grows in whole neighbour shells.  NULL, NULL turns the sink off. */
#define SPH_TARGET_SOLVED 0
#define SPH_TARGET_CENTRED 1
int sph_set_harvest(sph_ctx *ctx, float *d_feat, float *d_target, int32_t target_mode);

/* Inference on n device feature rows: y[n] (device), and, when non-NULL,
 * the bfloat16 bit patterns of the two hidden layers' rounded activations
 * d_h1[n][64], d_h2[n][64] (for checking). */
int sph_mlp_forward(sph_ctx *ctx, const float *d_feat, int64_t n, float *d_y, uint16_t *d_h1,
                    uint16_t *d_h2);

/* Mean squared error L = (1/n) sum_p (y_p - t_p)^2 over batch rows
 * p = d_rows[row0 + k], k < n (d_rows NULL: p = row0 + k), and its gradient
 * with respect to every parameter (chain rule; the bfloat16 roundings taken
 * as identity).  d_grad (device, SPH_MLP_NPARAM + 1 floats) receives the
 * gradient in parameter order and L last.  Per-wave partials are reduced in
 * a fixed order, so the result is reproducible. */
int sph_mlp_backward(sph_ctx *ctx, const float *d_feat, const float *d_target,
                     const int32_t *d_rows, int64_t row0, int64_t n, float *d_grad);

/* One Adam step (Kingma & Ba 2015), step number t >= 1, on the FP32 master
 * parameters with gradient d_grad (device); the bfloat16 copy is refreshed
 * with round to nearest even. */
int sph_mlp_adam_step(sph_ctx *ctx, const float *d_grad, double lr, double beta1, double beta2,
                      double eps, int32_t t);

/* Epoch loop on the device: for each of `epochs` passes over the n rows in
 * the order d_order (device, n indices; NULL = 0..n-1), batches of `batch`
 * consecutive entries (the last may be short): sph_mlp_backward, then Adam
 * (beta 0.9, 0.999, eps 1e-8) with the context's step counter.  d_loss
 * (device, epochs * ceil(n/batch) floats, or NULL) receives each batch's
 * loss. */
int sph_mlp_train(sph_ctx *ctx, const float *d_feat, const float *d_target,
                  const int32_t *d_order, int64_t n, int32_t batch, int32_t epochs, double lr,
                  float *d_loss);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
