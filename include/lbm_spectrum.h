/*
 * lbm_spectrum.h - batched linear stability analysis of the vectorial scheme
 * (paper, Section 4): the amplification matrix E(theta) of the scheme
 * linearised about a constant reference state, and its eigenvalues, for many
 * (reference state, frequency) points at once on one GPU.
 *
 * A Fourier mode f_hat e^{i xi . x} of the linearised scheme evolves as
 * f_hat(t + dt) = E(theta) f_hat(t), theta = xi dx, with
 *
 *   E(theta) = S(theta) [ diag(1 - omega) + diag(omega) J M ]
 *
 * where M sums each set's populations into its conserved moment
 * W = (rho, dx q_1, .., dx q_d), J is the Jacobian of the equilibria
 * (Section 2) with respect to W at the reference state, and
 * S(theta) = diag(exp(-i theta . c_l)) transports the population of velocity
 * c_l by one cell.  The order of E is n = (d + 1)(2d + 1): 15 in 2D, 28 in 3D.
 * Population index: set i (0 = rho, 1 + j = q_j) times (2d + 1) plus velocity
 * l (0 = rest, 1 + 2j = +e_j, 2 + 2j = -e_j).  The matrix is the same whether
 * the momentum populations are counted in units of q or of W = dx q (a
 * similarity), so its eigenvalues do not depend on that choice.
 *
 * Conventions: every array argument is device memory of the current device
 * (caller-owned; the library allocates nothing); calls are enqueued on
 * `stream` (hipStream_t as void*, NULL for the null stream) and are
 * asynchronous.  Status codes as in lbm.h: LBM_EINVAL for a bad dimension,
 * count or pointer; LBM_EDEVICE if the launch fails.
 */
#ifndef LBM_SPECTRUM_H
#define LBM_SPECTRUM_H

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A reference state and the scheme's parameters (Section 2, linearisation of
 * Section 4).  The momentum sets share omega_q and alpha_q. */
typedef struct lbm_lin_state {
  double mu;                  /* dx^2 / dt */
  double dx;                  /* space step: the advection terms of J scale with dx q_bar */
  double omega_rho, omega_q;  /* relaxation parameters */
  double alpha_rho, alpha_q;  /* linear-equilibrium parameters */
  double rho_bar;             /* reference density (> 0) */
  double q_bar[3];            /* reference momentum q (unused components ignored) */
  double dp_drho;             /* P'(rho_bar) of the pressure law in the momentum
                                 fluxes (1 for the scheme's P(rho) = rho) */
} lbm_lin_state;

/* Order n of E(theta) for a dimension (2 or 3); 0 otherwise. */
int32_t lbm_spectrum_order(int32_t dim);

/* E(theta) for npts points.  Point p uses states[state_of_point[p]]
 * (state_of_point may be NULL: state 0 for every point) and the frequency
 * theta[p * dim .. p * dim + dim - 1].  Output E[p][r][c][2] (row-major,
 * real and imaginary parts interleaved), n * n * 2 doubles per point.  A
 * point whose state index is outside [0, nstates) gets NaN entries.
 * npts = 0 enqueues nothing and returns LBM_OK (array pointers unchecked). */
lbm_status lbm_spectrum_matrix(int32_t dim, int64_t npts, const lbm_lin_state* states, int32_t nstates,
                               const int32_t* state_of_point, const double* theta, double* E,
                               void* stream);

/* Eigenvalues of E(theta) for npts points (arguments as lbm_spectrum_matrix),
 * by Householder reduction to Hessenberg form and the single-shift complex
 * QR algorithm, in FP64; a subdiagonal entry is deflated once it is below
 * DBL_EPSILON times the largest row sum of |Re| + |Im| of E (a backward
 * error of that size, like the rounding of the reduction).  Outputs, each
 * optional (NULL) but
 * not all NULL:
 *   eig[p][k][2]  the n eigenvalues of point p (real, imaginary); entry k
 *                 is the one that deflated at position k of the Schur form
 *   radius[p]     largest modulus among them (the spectral radius)
 *   info[p]       QR sweeps used (>= 0); -1 if the iteration did not
 *                 converge within 30 max(10, n) sweeps (the outputs then hold
 *                 the current diagonal); -2 for a state index outside
 *                 [0, nstates) (outputs NaN)
 *   flops[p]      real floating-point operations of the reflections and
 *                 rotations applied (the O(n^3) work), counted by the kernel
 * One wavefront per point. */
lbm_status lbm_spectrum_eigs(int32_t dim, int64_t npts, const lbm_lin_state* states, int32_t nstates,
                             const int32_t* state_of_point, const double* theta, double* eig,
                             double* radius, int32_t* info, double* flops, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SPECTRUM_H */
