/*
 * lbm_closure.h - device-side pieces of the learned coarse-grid correction.
 *
 * The paper has no closure; these entry points connect a coarse run of the
 * scheme (an lbm_ctx) with the correction network of lbm_cnn.h:
 *
 *   restriction   fine moments -> coarse moments (block averages)
 *   features      coarse moments -> normalised network input
 *   reset         populations <- equilibrium of given device moments
 *   correction    populations += f^eq(W + dW) - f^eq(W) behind a guard
 *
 * Moments are device FP32 planes [(1 + dim)][cells] holding rho, then the
 * physical momentum q_j (as lbm_moments_device writes them).  Every call is
 * enqueued on the context's stream (or the given one) and is asynchronous,
 * except lbm_closure_report which synchronises.
 */
#ifndef LBM_CLOSURE_H
#define LBM_CLOSURE_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 2D restriction by r x r block averages (nfx, nfy multiples of r):
 *   q_c = mean(q_f),  rho_c = rho_ref + r^2 (mean(rho_f) - rho_ref)
 * The density deviation carries the pressure, rho - rho_ref ~ dx^2 Phi
 * (Proposition 1), so the same pressure field has an r^2 larger density
 * deviation on the r-times coarser grid. */
lbm_status lbm_restrict(const float* fine, int64_t nfx, int64_t nfy, int32_t r, double rho_ref,
                        float* coarse, void* stream);

/* Network input x[(1 + dim)][cells]: x0 = (rho - rho_ref)/s_rho, x_{1+j} = (q_j/rho)/s_u. */
lbm_status lbm_closure_features(const float* moments, int32_t dim, int64_t cells, double rho_ref,
                                float s_rho, float s_u, float* x, void* stream);

/* Training target of a window (2D): t0 = (rho_next - rho_now)/s_drho,
 * t_{1+j} = (q_next_j - q_now_j)/s_dq, for [3][cells] moment planes. */
lbm_status lbm_closure_target(const float* m_next, const float* m_now, int64_t cells, float s_drho,
                              float s_dq, float* t, void* stream);

/* Divergence-free training target of a window (2D, n x n periodic, 1 <= n <= 1024):
 *   out_rho = now_rho,   out_q = now_q + P(fine_q - now_q)
 * for [3][n][n] device moment planes (rho, q_x, q_y), where P is the spectral
 * Helmholtz projection onto divergence-free fields, d^(k) - k (k . d^(k)) / |k|^2
 * for every wavenumber k != 0 (signed: k = m for m < n/2, m - n otherwise) with
 * the mean kept.  The artificial compressibility of the scheme carries
 * acoustic waves at a speed ~1/dx that differs on every grid; the projection
 * keeps the incompressible dynamics a coarse correction can learn.  Computed
 * in FP64 (discrete Fourier sums), rounded to FP32 once.  scratch: device
 * memory of lbm_closure_project_scratch_bytes(n) bytes (0 for an invalid n);
 * out must not alias the inputs.  Asynchronous on `stream`. */
size_t lbm_closure_project_scratch_bytes(int32_t n);
lbm_status lbm_closure_project(const float* m_fine, const float* m_now, int32_t n, float* out, void* scratch,
                               void* stream);

/* Replace the state of ctx by the equilibrium of the device moments (end of
 * Section 2: populations at equilibrium); the step count is kept. */
lbm_status lbm_set_equilibrium_device(lbm_ctx* ctx, const float* moments);

/* Guarded correction of a 2D context from the network output y[3][cells]:
 *   dW = (y0 s_drho, y1 s_dq, y2 s_dq), each channel minus its grid mean (so
 *   mass and momentum are unchanged);
 *   accept iff every corrected value is finite and
 *   ||div_h u'||_2 <= guard_factor ||div_h u||_2, u = q/rho, u' = (q+dq)/(rho+drho),
 *   centred differences on the periodic grid, u from `moments`;
 *   if accepted, every population gets f^eq(W + dW) - f^eq(W) added, W being
 *   the moments of the current state (the non-equilibrium part is kept).
 * The decision is taken on the device (no host round trip); read it with
 * lbm_closure_report. */
lbm_status lbm_closure_apply(lbm_ctx* ctx, const float* moments, const float* y, float s_drho, float s_dq,
                             float guard_factor);

/* One whole correction of a 2D context, in five launches on its stream:
 *   moments (written to `moments`, [3][cells] FP32, as lbm_moments_device),
 *   the network output y = lbm_net_infer(moments, rho_ref of ctx, s_rho, s_u,
 *   packed, bias) ([3][cells] FP32),
 *   the guard and the update of lbm_closure_apply(ctx, moments, y, s_drho,
 *   s_dq, guard_factor).
 * The same result as those calls made one by one, except that the grid means
 * of y are summed per 16 x 16 tile first (a different FP64 summation order).
 * nx and ny must be multiples of 16; packed and bias are host arrays of the
 * four layers' device pointers (lbm_cnn.h).  Nothing in it needs the host,
 * so a caller can capture it in a graph. */
lbm_status lbm_closure_correct(lbm_ctx* ctx, const void* const* packed, const float* const* bias,
                               float s_rho, float s_u, float s_drho, float s_dq, float guard_factor,
                               float* moments, float* y);

typedef struct lbm_closure_report {
  int64_t n_accepted; /* corrections applied since lbm_init */
  int64_t n_rejected; /* corrections refused by the guard since lbm_init */
  int32_t accepted;   /* 1 if the last correction was applied */
  double div_before;  /* ||div_h u||_2 before */
  double div_after;   /* ||div_h u'||_2 of the proposed correction */
  double mean[3];     /* grid means removed from the three output channels (physical units) */
} lbm_closure_report;

/* Report of the last lbm_closure_apply on ctx.  Synchronises. */
lbm_status lbm_closure_report_get(lbm_ctx* ctx, lbm_closure_report* out);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CLOSURE_H */
