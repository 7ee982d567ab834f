/*
 * lbm_batch.h - many independent runs of the vectorial lattice Boltzmann
 * scheme (paper, Section 2) advanced together on one GPU.
 *
 * Every run is an independent periodic problem with its own grid and its own
 * scheme parameters (dx, dt, nu, omega, alpha); all runs share the dimension
 * and the storage mode (lbm_storage of lbm.h).  One time step of the whole
 * batch is ONE launch of a persistent kernel whose blocks walk a list of
 * 256-cell tiles covering every run; the tile shape of each size class
 * (64x4, 128x2 or 256x1 cells in 2D) is chosen by lbm_batch_autotune.  Steps
 * are replayed from a HIP graph.  In 2D two more persistent kernels advance
 * several steps per launch (lbm_batch_set_fusion): one walks 64 x 8-cell tiles
 * and advances two steps (each tile and its one-cell border by one step into
 * LDS, the tile by the second); the default one walks the single-run engine's
 * multi-step tiles and advances K steps (the tile and a (K-1)-cell border by
 * one step into LDS, K-2 more steps inside LDS on shrinking regions, the tile
 * by the last): K = 6 in LBM_F32 and LBM_F32_RAW when at least half of the
 * batch's cells belong to runs of 2^20 cells or more (as the single-run
 * engine), else 5.  The per-cell update is the same device code as lbm_step, so a
 * run advanced in a batch is bit-identical to the same run advanced alone,
 * with any setting.  The split FP16 (LBM_F16_NEQ) and FP64
 * storages are not available in a batch.
 *
 * Conventions are those of lbm.h: status codes only, caller-owned device
 * workspace (never allocated by the library), caller's stream, FP64 host
 * arrays copied during the call.
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_batch lbm_batch;

/* One run.  Same meaning and validity rules as the fields of lbm_params. */
typedef struct lbm_run_spec {
  int64_t n[3];       /* cells along x, y, z (n[2] = 1 in 2D) */
  double dx, dt, nu;  /* mu = dx^2/dt; nu sets alpha_q */
  double omega_rho, omega_q, alpha_rho;
  double rho_ref;
} lbm_run_spec;

/* Device workspace bytes for the batch (0 if any run is invalid). */
size_t lbm_batch_workspace_bytes(int32_t dim, int32_t storage, int32_t nruns,
                                 const lbm_run_spec* runs);

/* Create the batch and set every run to the equilibrium of its initial moments.
 *   u0[r]    host FP64 [dim][cells_r] velocity of run r (required)
 *   rho0     NULL, or an array whose entries are NULL (rho_ref) or FP64 [cells_r]
 * Returns LBM_EINVAL / LBM_EUNSTABLE for the first invalid run (its index in
 * *bad_run if bad_run != NULL); a 2D run of more than 2^30 cells is invalid in
 * a batch (the multi-step tiles address a plane with 32-bit byte offsets).
 * Synchronises once. */
lbm_status lbm_batch_init(lbm_batch** out, int32_t dim, int32_t storage, int32_t nruns,
                          const lbm_run_spec* runs, const double* const* u0,
                          const double* const* rho0, void* workspace, size_t ws_bytes,
                          void* hip_stream, int32_t* bad_run);

/* Choose the tile shape of every size class (runs grouped by nx rounded up to
 * a power of two), then the number of blocks of the persistent launch (4, 8,
 * 16 or 32 per compute unit, or one per tile), and in 2D the number of blocks
 * of the two-step launch (1, 2, 4 or 8 per compute unit, or one per tile) and
 * the K-step tile shape of every size class (each shape timed on the class's
 * runs alone, as a graph launch), by timing each candidate on the batch's own
 * buffers; the state is not changed.  The K-step launches keep one block per
 * tile (lbm_batch_set_fused_grid changes that).
 * If cache_path is non-NULL (else the environment
 * variable LBM_AUTOTUNE_CACHE, if set) previously tuned shapes for this
 * device, dimension and storage are read from that text file and new ones are
 * appended.  Rebuilds the step graph.  Synchronises. */
lbm_status lbm_batch_autotune(lbm_batch* b, const char* cache_path);

/* Advance every run by nsteps >= 0 steps.  Asynchronous (graph replays). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Moments of run r, as lbm_moments.  Synchronises. */
lbm_status lbm_batch_moments(lbm_batch* b, int32_t run, double* rho, double* q);

/* Total cells over all runs, and number of 256-cell tiles per step. */
lbm_status lbm_batch_info(const lbm_batch* b, int64_t* total_cells, int64_t* tiles,
                          int64_t* steps);

/* Tile width (cells along x) chosen for run r's size class. */
int32_t lbm_batch_tile_width(const lbm_batch* b, int32_t run);

/* Blocks of the persistent step launch (a grid of at least the tile count
 * means one block per tile); chosen by lbm_batch_autotune. */
int32_t lbm_batch_grid(const lbm_batch* b);

/* Blocks of the current multi-step launch: the K-step kernel's (summed over
 * its tile shapes) when the fusion is K, else the two-step kernel's (0 if the
 * batch has none, i.e. in 3D).  The two-step grid is chosen by
 * lbm_batch_autotune; the K-step grid is one block per tile unless
 * lbm_batch_set_fused_grid set a persistent one. */
int32_t lbm_batch_fused_grid(const lbm_batch* b);

/* Cell tile (tx x ty) of run r in the K-step launches (2D population
 * storages; LBM_EINVAL otherwise).  Three shapes exist per storage (4-byte
 * planes: 32x32 at K = 5 or 32x28 at K = 6, 32x16, 16x16; 16-bit planes:
 * 64x16, 32x32, 32x16); lbm_batch_autotune picks one per size class, the
 * first one otherwise. */
lbm_status lbm_batch_fused_tile(const lbm_batch* b, int32_t run, int32_t* tx, int32_t* ty);

/* Use fused tile shape `shape` (0, 1 or 2, in the order above) for every run
 * (results do not depend on it).  Rebuilds the step graphs.  Synchronises. */
lbm_status lbm_batch_set_fused_shape(lbm_batch* b, int32_t shape);

/* Blocks per compute unit of each K-step launch (1..64; each block then
 * walks several tiles), or 0 for one block per tile (the default); results do
 * not depend on it.  A persistent grid is slower here: the launch's per-shape
 * graph nodes run concurrently and share the compute units.  2D population
 * storages only (LBM_EINVAL otherwise).  Rebuilds the step graphs.
 * Synchronises. */
lbm_status lbm_batch_set_fused_grid(lbm_batch* b, int32_t blocks_per_cu);

/* Steps per launch: 1 (one-step kernel), 2 (two-step kernel) or the batch's K
 * (the K-step kernel, the default: 5 or 6, fixed when the batch is created);
 * 2 and K in 2D only; LBM_EINVAL otherwise.  Every setting gives the same
 * states.  A remainder shorter than the setting runs as shorter launches. */
lbm_status lbm_batch_set_fusion(lbm_batch* b, int32_t steps_per_launch);

/* The current number of steps per launch (0 for NULL). */
int32_t lbm_batch_fusion(const lbm_batch* b);

void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_BATCH_H */
