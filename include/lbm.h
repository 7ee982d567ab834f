/*
 * lbm.h - C ABI of the vectorial lattice Boltzmann engine (single GPU, gfx950).
 *
 * The engine advances the vectorial D2Q5 (2D) / D3Q7 (3D) lattice Boltzmann
 * scheme for the incompressible Navier-Stokes system (paper, Section 2): one
 * 5- (7-) velocity distribution set for each conserved component
 * (rho, q_x, q_y[, q_z]); each set is relaxed toward its equilibrium with its
 * own relaxation parameter omega (equation (LBM_scheme)) and then transported
 * by one cell along its velocity on a periodic Cartesian grid.  Parameters
 * follow the paper's statement of the problem: cell-centred grid with spacing
 * dx (Section 2), time step dt with mu = dx^2/dt fixed (parabolic scaling,
 * eq. (parabolicScaling)), viscosity nu = 2 mu alpha_q (1/omega_q - 1/2)
 * (end of Section 3), pressure law P(rho) = rho^gamma (Section 2).
 *
 * Conventions
 *   - All entry points return an lbm_status; nothing else crosses the ABI.
 *   - Grids are indexed [z][y][x] with x fastest; "cells" = nx * ny * nz.
 *   - Host arrays are plain FP64, owned by the caller, copied during the call
 *     and never retained.
 *   - Device memory is never allocated by the library: the caller passes a
 *     device workspace of at least lbm_workspace_bytes() bytes which must
 *     outlive the context; the context holds only host-side state.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*, NULL = the null stream).  lbm_step is asynchronous; calls that
 *     return host data synchronise that stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = 1,      /* null pointer, bad size, dx or dt <= 0, gamma != 1, bad storage */
  LBM_EUNSTABLE = 2,   /* omega outside (0,2) or alpha outside [0, 1/(2 dim)] (Lemma 1) */
  LBM_ENOMEM = 3,      /* workspace smaller than lbm_workspace_bytes() */
  LBM_EDEVICE = 4,     /* a HIP runtime call or kernel launch failed */
  LBM_ENONFINITE = 5,  /* diagnostics found cells holding non-finite populations */
  LBM_ESTATE = 6       /* state blob of the wrong size or layout */
} lbm_status;

/* Storage of the distributions in HBM.  Arithmetic is FP32 in every mode
 * except LBM_F64, which loads, updates and stores FP64.
 * Every mode except LBM_F32_RAW stores g = f - fbar, the deviation from the
 * reference equilibrium fbar = f^eq(rho_ref, q = 0); the collision works on g
 * directly (the equilibria are affine in W_rho for P(rho) = rho), so the large
 * constant parts of the populations (rho_ref weights, +-rho_ref/(2 mu)) never
 * enter a rounding.
 *   LBM_F32           g in FP32 (15 planes 2D / 28 planes 3D)
 *   LBM_F16_DEV       g in FP16 (round to nearest even)
 *   LBM_BF16_DEV      g in BF16 (round to nearest even)
 *   LBM_F16_DEV_R32   moving populations as FP16 g, the rest population of
 *                     each set as FP32 g
 *   LBM_BF16_DEV_R32  as above with BF16 moving populations
 *   LBM_F32_RAW       the populations f themselves in FP32
 *   LBM_F16_NEQ       equilibrium-split storage: per cell the moments W in
 *                     FP32 (W_rho as a deviation from rho_ref) in place of the
 *                     rest planes, and per set and moving velocity the
 *                     non-equilibrium part n = f* - f^eq(W) in FP16, times a
 *                     power-of-two scale per set fixed by lbm_init from the
 *                     parameters (sized for lattice Mach numbers up to about
 *                     0.1; saved with the state); the rest entry's
 *                     part is minus the sum of the moving ones.  Same bytes as
 *                     LBM_F16_DEV_R32 with about FP32 accuracy, since FP16 only
 *                     rounds the small non-equilibrium parts
 *   LBM_F32_MOMENTS   the relaxation scheme omega_rho = omega_q = 1 only
 *                     (LBM_EINVAL otherwise): every post-relaxation population
 *                     is then the equilibrium of its cell's moments, so the
 *                     state is the moments W alone (D+1 FP32 planes, W_rho as a
 *                     deviation) and a step is the stencil W(t+1, x) =
 *                     sum_l f^eq_l(W(t, x - c_l)); 24 B per update in 2D, no
 *                     channel boundaries, not in lbm_batch
 *   LBM_F64           g in FP64 with FP64 arithmetic: the reference mode for
 *                     long fine-grid runs, where FP32 rounding accumulates over
 *                     many steps; one step per launch (lbm_set_fusion(2)
 *                     fails) and not available in lbm_batch              */
typedef enum lbm_storage {
  LBM_F32 = 0,
  LBM_F16_DEV = 1,
  LBM_BF16_DEV = 2,
  LBM_F16_DEV_R32 = 3,
  LBM_BF16_DEV_R32 = 4,
  LBM_F32_RAW = 5,
  LBM_F64 = 6,
  LBM_F16_NEQ = 7,
  LBM_F32_MOMENTS = 8
} lbm_storage;

/* Flag bits reported in lbm_diag.flags and by lbm_check_params(). */
#define LBM_WARN_LOWFREQ 0x1u /* mu^2 (alpha_rho + alpha_q) < 1: low-frequency acoustic
                                 modes may grow (Section 4.2, relaxation-scheme lemma) */

typedef struct lbm_params {
  int32_t dim;        /* 2 or 3 */
  int32_t storage;    /* lbm_storage */
  int64_t n[3];       /* cells along x, y, z; n[2] must be 1 when dim == 2 */
  double dx;          /* space step (> 0); cell centres at (i + 1/2) dx */
  double dt;          /* time step (> 0); mu = dx*dx/dt */
  double nu;          /* kinematic viscosity (>= 0), sets alpha_q */
  double omega_rho;   /* relaxation parameter of the density set, in (0, 2) */
  double omega_q;     /* relaxation parameter of the momentum sets, in (0, 2) */
  double alpha_rho;   /* equilibrium weight of the density set, in [0, 1/(2 dim)] */
  double gamma;       /* pressure exponent; the GPU engine supports gamma == 1 */
  double rho_ref;     /* reference density: default rho0 and deviation reference */
} lbm_params;

typedef struct lbm_diag {
  int64_t step;        /* time steps taken since lbm_init */
  double time;         /* step * dt */
  double mass;         /* dx^dim sum rho                               (FP64) */
  double mom[3];       /* dx^dim sum q_j                               (FP64) */
  double kinetic;      /* 1/2 dx^dim sum |q|^2 / rho                   (FP64) */
  double enstrophy;    /* 1/2 dx^dim sum |curl_h u|^2, centred diffs   (FP64) */
  double div_l2;       /* sqrt(dx^dim sum (div_h u)^2), centred diffs  (FP64) */
  double max_u;        /* max |u|, u = q / rho */
  double rho_min, rho_max;
  int64_t nonfinite;   /* cells holding at least one non-finite population */
  uint32_t flags;      /* LBM_WARN_* bits of the parameters */
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Host-only validation.  Computes mu = dx^2/dt and alpha_q from the viscosity
 * relation; either output pointer may be NULL.  No device work. */
lbm_status lbm_check_params(const lbm_params* p, double* mu, double* alpha_q, uint32_t* flags);

/* Device workspace bytes needed for parameters p (0 if p is invalid). */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a context and set every population to its equilibrium of the initial
 * moments (end of Section 2): W0 = (rho0, dx rho0 u0).
 *   u0     host FP64 [dim][cells] physical velocity (required)
 *   rho0   host FP64 [cells] density, or NULL for rho_ref everywhere
 *   workspace / ws_bytes  caller-owned device memory
 *   hip_stream            stream for all work of this context
 * Synchronises the stream once so that launch errors are reported here. */
lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, const double* u0, const double* rho0,
                    void* workspace, size_t ws_bytes, void* hip_stream);

/* Advance nsteps >= 0 time steps (relaxation then transport, Section 2).
 * Each launch fuses relaxation and transport.  One launch may advance
 * several steps (lbm_set_fusion): in 2D each tile and a border as wide as the
 * steps still to come are advanced on chip, the border shrinking by one cell
 * per step; in 3D a column tile marches along z with one plane per step in
 * flight.  Only the final state is written back.  A remainder shorter than
 * the fusion depth runs as two-step and single-step launches.  The result is
 * bit-identical for any fusion setting.  Asynchronous. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Time steps per launch, 1 .. 6.  In 2D, 2 .. 6 in any storage but LBM_F64
 * (3 .. 6 only while a plane holds at most 2^32 bytes, i.e. 2^30 FP32 cells);
 * in 3D, 2 and 3 for the population storages LBM_F32, LBM_F32_RAW and the
 * four 16-bit deviation storages, 2 for LBM_F32_MOMENTS while an x-y plane
 * holds at most 2^30 cells (kernels that march along z); channel boundaries
 * allow 1 only.  LBM_EINVAL otherwise.  Default in 2D: from 2^20 cells on 6
 * for LBM_F32, LBM_F32_RAW, LBM_F16_DEV_R32 and LBM_BF16_DEV_R32, 4 for
 * LBM_F32_MOMENTS and 5 for the other storages, below that 2 where
 * available, else 1.  Default in 3D: the largest of 3 and 2 whose launch has
 * at least 128 blocks (one per 64 x 8 or, for LBM_F32_MOMENTS, 64 x 11
 * column tile and segment along z; 128^3 runs three steps per launch
 * in the population storages and two in LBM_F32_MOMENTS, 64^3 one), else 1. */
lbm_status lbm_set_fusion(lbm_ctx* ctx, int32_t steps_per_launch);

/* The current number of time steps per launch (0 for a NULL context). */
int32_t lbm_fusion(const lbm_ctx* ctx);

/* Moments of the current state: rho [cells] and q [dim][cells] = (1/dx) sum f_q,
 * summed in FP64 from the stored populations.  Host FP64 outputs; q may be
 * NULL.  Synchronises. */
lbm_status lbm_moments(lbm_ctx* ctx, double* rho, double* q);

/* Same moments into caller-owned device FP32 memory out[(1+dim)][cells]
 * (rho first, then q_j).  Asynchronous. */
lbm_status lbm_moments_device(lbm_ctx* ctx, float* out);

/* FP64 reductions of the current state, see lbm_diag.  Deterministic (fixed
 * reduction order).  Returns LBM_ENONFINITE when out->nonfinite > 0 (the
 * struct is filled either way).  Synchronises. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out);

/* Allocation-free diagnostics, for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid allocation): the results of
 * lbm_diagnostics, bit for bit (same kernels, same fixed reduction order),
 * with the per-block partials and the final slots in a static device array
 * of the library instead of the context's workspace: at most 2048 partials of
 * 16 doubles plus the final slots, 262 KB per GPU, held until the process
 * ends.  lbm_init looks up the array's device address once per device.
 * Nothing is allocated and nothing needs clearing (every slot read is written
 * earlier in the same call).  Calls that overlap on one GPU (several threads
 * or streams) share the array and race: serialise them.  LBM_EINVAL for NULL
 * arguments or a partial count above the array's capacity; LBM_EDEVICE if the
 * address lookup failed; LBM_ENONFINITE as lbm_diagnostics.  Synchronises. */
lbm_status lbm_diagnostics_noalloc(lbm_ctx* ctx, lbm_diag* out);

/* Size of a full state snapshot: every population plane (without padding:
 * the D+1 rest planes of cells x rest element, then the (D+1) 2D moving planes
 * of cells x moving element, in the element types of the storage mode), then
 * the step count as int64, then for LBM_F16_NEQ the four FP32 per-set scales. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
/* Copy the full state to / from host memory (synchronises).  Restarting from
 * moments alone is not a continuation (the non-equilibrium part is lost), so
 * the snapshot holds every population plane. */
lbm_status lbm_save_state(lbm_ctx* ctx, void* host, size_t bytes);
lbm_status lbm_load_state(lbm_ctx* ctx, const void* host, size_t bytes);

/* Channel boundaries (2D; the numerical boundary conditions of the Poiseuille
 * test, Section 5.2) in place of the periodic ones, on the box [0, nx dx] x
 * [0, ny dx]:
 *   inlet  x = 0:  ghost moments rho_g = 2 rho(0) - rho(1),
 *                  q_g = 2 rho_ref u_in(y) - q(0)           (enters: +x)
 *   outlet x = L:  rho_g = 2 rho_out - rho(nx-1),
 *                  q_g = 2 q(nx-1) - q(nx-2)                (enters: -x)
 *   walls  y = 0, L: rho_g = 2 rho(wall row) - rho(next row),
 *                  q_g = (2 rho_ref u_wall - q_x, -q_y)(wall row) (enters: +y / -y)
 * The entering post-relaxation population of every set is the equilibrium of
 * the ghost moments; with `correction` the walls add the non-equilibrium part
 * f* - f^eq(W) of the same population in the wall row (second order when
 * omega_q != 1).  Moments are those of the time level the step starts from.
 *   walls   NULL restores periodic boundaries
 *   u_in    host FP64 [2][ny]: inlet velocity (x, then y component), copied
 * While the walls are set every launch advances one step (lbm_set_fusion(2)
 * returns LBM_EINVAL); diagnostics keep their periodic centred differences.
 * LBM_EINVAL for 3D contexts, LBM_F16_NEQ storage, nx or ny < 3, a NULL u_in
 * or non-finite values.  Synchronises (the profile copy). */
typedef struct lbm_walls {
  double rho_out;      /* outlet density target, rho_ref (1 + dx^2 p_out) */
  double u_bottom;     /* tangential velocity of the wall at y = 0 */
  double u_top;        /* tangential velocity of the wall at y = L */
  int32_t correction;  /* 1: non-equilibrium correction on the two walls */
} lbm_walls;

lbm_status lbm_set_walls(lbm_ctx* ctx, const lbm_walls* walls, const double* u_in);

/* Steps taken so far. */
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Release the host-side context (the workspace stays with the caller). */
void lbm_destroy(lbm_ctx* ctx);

const char* lbm_strerror(lbm_status s);

/* Measurement probe: copy `bytes` (multiple of 16, 16-byte aligned device
 * pointers) from src to dst with the library's streaming copy kernel,
 * enqueued on hip_stream.  It is the denominator of the HBM-bandwidth
 * fraction: its achieved read+write bandwidth is the measured peak. */
lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
