// Batched amplification matrices of the linearised scheme and their
// eigenvalues (Section 4).  Contract in include/lbm_spectrum.h.
//
// One 64-lane wavefront (one workgroup) per point.  E(theta) lives in LDS as
// FP64 complex entries; lane t owns row t or column t of the current update:
//   1. build: lane r writes row r of E = S (diag(1 - omega) + diag(omega) J M);
//   2. Householder reduction to upper Hessenberg form: for column k the
//      reflector is formed redundantly by every lane from column k (broadcast
//      reads), applied from the left (lane = column) and from the right
//      (lane = row);
//   3. single-shift complex QR with Wilkinson shifts on the active window
//      [l, hi] of the Hessenberg matrix: the deflation test runs on all
//      subdiagonal entries at once (one lane each, combined with a ballot),
//      and each bulge-chasing Givens rotation updates two rows (lane = column)
//      and then two columns (lane = row).
// Every loop bound and branch condition is uniform across the wavefront, so
// the barriers are reached by the whole workgroup; the QR loop is capped at
// 30 max(10, n) sweeps.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_spectrum.h"

namespace {

struct cplx {
  double re, im;
};

__device__ inline cplx cx(double r, double i) { return {r, i}; }
__device__ inline cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cplx operator-(cplx a) { return {-a.re, -a.im}; }
__device__ inline cplx operator*(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ inline cplx conj(cplx a) { return {a.re, -a.im}; }
__device__ inline double abs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ inline double abs1(cplx a) { return fabs(a.re) + fabs(a.im); }
// conj(a) * b
__device__ inline cplx cmulc(cplx a, cplx b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }

// a / b by Smith's scaling (no overflow of |b|^2 for large entries)
__device__ inline cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// principal square root
__device__ inline cplx csqrt(cplx z) {
  const double m = hypot(z.re, z.im);
  if (m == 0.0) return {0.0, 0.0};
  if (z.re >= 0.0) {
    const double r = sqrt(0.5 * (m + z.re));
    return {r, z.im / (2.0 * r)};
  }
  const double i = sqrt(0.5 * (m - z.re));
  return {fabs(z.im) / (2.0 * i), copysign(i, z.im)};
}

template <int D>
struct Shape {
  static constexpr int NV = 2 * D + 1;       // velocities per set
  static constexpr int N = (D + 1) * NV;     // order of E
  static constexpr int LD = N | 1;           // LDS row stride (odd, in complex entries)
};

// Row r of the equilibrium Jacobian with respect to W = (rho, dx q) at the
// reference state, from the equilibria of Section 2:
//   density set   rest  (1 - 2d a_rho) W_rho
//                 +-e_j a_rho W_rho +- W_j / (2 mu)
//   momentum W_a  rest  (1 - 2d a_q) W_a
//                 +-e_j a_q W_a +- (W_a W_j / W_rho + delta_aj P(rho)) / (2 mu)
template <int D>
__device__ inline void jacobian_row(const lbm_lin_state& s, int r, double J[D + 1]) {
  constexpr int NV = Shape<D>::NV;
  const int set = r / NV, l = r % NV;
#pragma unroll
  for (int k = 0; k < D + 1; ++k) J[k] = 0.0;
  const int j = (l - 1) >> 1;
  const double sg = (l & 1) ? 1.0 : -1.0;        // l = 1 + 2j: +e_j; l = 2 + 2j: -e_j
  const double h = 1.0 / (2.0 * s.mu);
  if (set == 0) {
    if (l == 0) {
      J[0] = 1.0 - 2.0 * D * s.alpha_rho;
    } else {
      J[0] = s.alpha_rho;
      J[1 + j] = sg * h;
    }
    return;
  }
  const int a = set - 1;
  if (l == 0) {
    J[set] = 1.0 - 2.0 * D * s.alpha_q;
    return;
  }
  const double wa = s.dx * s.q_bar[a], wj = s.dx * s.q_bar[j], rb = s.rho_bar;
  J[set] += s.alpha_q;
  J[set] += sg * h * wj / rb;
  J[1 + j] += sg * h * wa / rb;
  J[0] -= sg * h * wa * wj / (rb * rb);
  if (a == j) J[0] += sg * h * s.dp_drho;
}

// exp(-i theta . c_l) of velocity l
template <int D>
__device__ inline cplx transport_phase(const double* th, int l) {
  if (l == 0) return {1.0, 0.0};
  const int j = (l - 1) >> 1;
  double sn, cs;
  sincos(th[j], &sn, &cs);
  return (l & 1) ? cx(cs, -sn) : cx(cs, sn);
}

// E[r][c] for c = 0..N-1 of row r, handed to emit(c, value)
template <int D, typename Emit>
__device__ inline void build_row(const lbm_lin_state& s, const double* th, int r, Emit emit) {
  constexpr int NV = Shape<D>::NV;
  double J[D + 1];
  jacobian_row<D>(s, r, J);
  const int set = r / NV;
  const double w = set == 0 ? s.omega_rho : s.omega_q;
  const cplx ph = transport_phase<D>(th, r % NV);
#pragma unroll
  for (int k = 0; k < D + 1; ++k) {
    const double wj = w * J[k];
#pragma unroll
    for (int c = k * NV; c < (k + 1) * NV; ++c) emit(c, (c == r ? 1.0 - w + wj : wj) * ph);
  }
}

__device__ inline bool state_ok(const int32_t* sidx, int32_t nstates, int64_t p, int32_t* si) {
  const int32_t k = sidx ? sidx[p] : 0;
  *si = k;
  return k >= 0 && k < nstates;
}

template <int D>
__global__ __launch_bounds__(256) void k_spectrum_matrix(const lbm_lin_state* __restrict__ states, int32_t nstates,
                                                         const int32_t* __restrict__ sidx,
                                                         const double* __restrict__ theta, int64_t npts,
                                                         double* __restrict__ E) {
  constexpr int N = Shape<D>::N;
  const int64_t r_all = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r_all >= npts * N) return;
  const int64_t p = r_all / N;
  const int r = static_cast<int>(r_all % N);
  double* out = E + (p * N + r) * N * 2;
  int32_t si;
  if (!state_ok(sidx, nstates, p, &si)) {
    for (int c = 0; c < 2 * N; ++c) out[c] = __builtin_nan("");
    return;
  }
  const lbm_lin_state s = states[si];
  double th[D];
#pragma unroll
  for (int j = 0; j < D; ++j) th[j] = theta[p * D + j];
  build_row<D>(s, th, r, [&](int c, cplx v) {
    out[2 * c] = v.re;
    out[2 * c + 1] = v.im;
  });
}

constexpr double kUlp = 2.220446049250313e-16;   // DBL_EPSILON
constexpr double kSmall = 1e-290;                 // absolute deflation floor

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G [x; y] = [r; 0].
__device__ inline void givens(cplx x, cplx y, double* c, cplx* s, cplx* r) {
  const double ax = sqrt(abs2(x)), nu = sqrt(abs2(x) + abs2(y));
  if (nu == 0.0) {
    *c = 1.0;
    *s = cx(0.0, 0.0);
    *r = cx(0.0, 0.0);
  } else if (ax == 0.0) {
    *c = 0.0;
    *s = (1.0 / nu) * conj(y);
    *r = cx(nu, 0.0);
  } else {
    const cplx ph = (1.0 / ax) * x;
    *c = ax / nu;
    *s = (1.0 / nu) * (ph * conj(y));
    *r = nu * ph;
  }
}

template <int D>
__global__ __launch_bounds__(64) void k_spectrum_eigs(const lbm_lin_state* __restrict__ states, int32_t nstates,
                                                      const int32_t* __restrict__ sidx,
                                                      const double* __restrict__ theta, int64_t npts,
                                                      double* __restrict__ eig, double* __restrict__ radius,
                                                      int32_t* __restrict__ info, double* __restrict__ flops) {
  constexpr int N = Shape<D>::N, LD = Shape<D>::LD;
  constexpr int kMaxSweeps = 30 * (N > 10 ? N : 10);
  __shared__ cplx A[N * LD];
  const int t = threadIdx.x;
  for (int64_t p = blockIdx.x; p < npts; p += gridDim.x) {
    int32_t si;
    if (!state_ok(sidx, nstates, p, &si)) {
      if (t < N && eig) {
        eig[(p * N + t) * 2] = __builtin_nan("");
        eig[(p * N + t) * 2 + 1] = __builtin_nan("");
      }
      if (t == 0) {
        if (radius) radius[p] = __builtin_nan("");
        if (info) info[p] = -2;
        if (flops) flops[p] = 0.0;
      }
      continue;
    }
    const lbm_lin_state s = states[si];
    double th[D];
#pragma unroll
    for (int j = 0; j < D; ++j) th[j] = theta[p * D + j];
    __syncthreads();                         // the previous point is done with A
    double rowsum = 0.0;                     // sum of |re| + |im| over row t
    if (t < N) build_row<D>(s, th, t, [&](int c, cplx v) {
      A[t * LD + c] = v;
      rowsum += abs1(v);
    });
    // hnorm = max row sum (a norm of E, the same on every lane)
    double hnorm = rowsum;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) hnorm = fmax(hnorm, __shfl_xor(hnorm, o));
    __syncthreads();

    double work = 0.0;
    // ---- Householder reduction to upper Hessenberg form ----
    for (int k = 0; k < N - 2; ++k) {
      // reflector from x = A[k+1 .., k]: H = I - tau v v^H, H x = beta e_1,
      // v = (x_0 - beta, x_1, ..); every lane forms it from the same reads
      double sig = 0.0;
      for (int i = k + 2; i < N; ++i) sig += abs2(A[i * LD + k]);
      if (sig == 0.0) continue;              // already reduced in this column
      const cplx x0 = A[(k + 1) * LD + k];
      const double a0 = sqrt(abs2(x0)), nrm = sqrt(a0 * a0 + sig);
      const cplx ph = a0 > 0.0 ? (1.0 / a0) * x0 : cx(1.0, 0.0);
      const cplx beta = -nrm * ph;
      const cplx v0 = (a0 + nrm) * ph;       // x_0 - beta
      const double tau = 2.0 / ((a0 + nrm) * (a0 + nrm) + sig);
      const int m = N - k - 1;               // reflector length
      // left: columns k+1 .. N-1, lane = column
      if (t > k && t < N) {
        cplx w = cmulc(v0, A[(k + 1) * LD + t]);
        for (int i = k + 2; i < N; ++i) w = w + cmulc(A[i * LD + k], A[i * LD + t]);
        w = tau * w;
        A[(k + 1) * LD + t] = A[(k + 1) * LD + t] - v0 * w;
        for (int i = k + 2; i < N; ++i) A[i * LD + t] = A[i * LD + t] - A[i * LD + k] * w;
      }
      __syncthreads();
      // right: all rows, lane = row
      if (t < N) {
        cplx u = A[t * LD + k + 1] * v0;
        for (int j = k + 2; j < N; ++j) u = u + A[t * LD + j] * A[j * LD + k];
        u = tau * u;
        A[t * LD + k + 1] = A[t * LD + k + 1] - u * conj(v0);
        for (int j = k + 2; j < N; ++j) A[t * LD + j] = A[t * LD + j] - u * conj(A[j * LD + k]);
      }
      __syncthreads();
      // column k becomes (beta, 0, ..) below the diagonal; no later step reads
      // the rest of column k before the QR phase
      if (t == k + 1) A[t * LD + k] = beta;
      else if (t > k + 1 && t < N) A[t * LD + k] = cx(0.0, 0.0);
      work += 16.0 * m * (N - k - 1) + 16.0 * m * N;
    }
    __syncthreads();

    // ---- single-shift complex QR on the Hessenberg matrix ----
    int hi = N - 1, its = 0, sweeps = 0;
    double rad = 0.0;
    bool failed = false;
    while (hi >= 0) {
      if (hi == 0) {
        const cplx z = A[0];
        if (t == 0 && eig) {
          eig[p * N * 2] = z.re;
          eig[p * N * 2 + 1] = z.im;
        }
        rad = fmax(rad, sqrt(abs2(z)));
        break;
      }
      // deflation: the largest k in [1, hi] with a negligible A[k][k-1], that
      // is below ulp times the norm of E (setting it to zero is a backward
      // error of that size, as the rounding of the reduction already is)
      bool small = false;
      if (t >= 1 && t <= hi) small = abs1(A[t * LD + t - 1]) <= fmax(kUlp * hnorm, kSmall);
      const uint64_t mask = __ballot(small);
      const int l = mask ? 63 - __clzll(static_cast<long long>(mask)) : 0;
      if (l == hi) {
        const cplx z = A[hi * LD + hi];
        if (t == 0 && eig) {
          eig[(p * N + hi) * 2] = z.re;
          eig[(p * N + hi) * 2 + 1] = z.im;
        }
        rad = fmax(rad, sqrt(abs2(z)));
        --hi;
        its = 0;
        continue;
      }
      if (sweeps == kMaxSweeps) {
        failed = true;
        break;
      }
      // shift: eigenvalue of the trailing 2x2 block closer to its last entry;
      // an exceptional shift every tenth sweep without deflation
      const cplx a = A[(hi - 1) * LD + hi - 1], b = A[(hi - 1) * LD + hi];
      const cplx c = A[hi * LD + hi - 1], d = A[hi * LD + hi];
      cplx sigma;
      if (its > 0 && its % 10 == 0) {
        sigma = d + cx(0.75 * abs1(c), 0.0);
      } else {
        const cplx tt = 0.5 * (a - d), bc = b * c;
        cplx disc = csqrt(tt * tt + bc);
        if (tt.re * disc.re + tt.im * disc.im < 0.0) disc = -disc;
        const cplx den = tt + disc;
        sigma = abs1(den) == 0.0 ? d : d - cdiv(bc, den);
      }
      // implicit QR sweep over [l, hi]: chase the bulge with Givens rotations
      cplx x = A[l * LD + l] - sigma, y = A[(l + 1) * LD + l];
      for (int k = l; k < hi; ++k) {
        if (k > l) {
          x = A[k * LD + k - 1];
          y = A[(k + 1) * LD + k - 1];
        }
        double gc;
        cplx gs, gr;
        givens(x, y, &gc, &gs, &gr);
        // rows k, k+1 over columns max(l, k-1) .. hi, lane = column
        const int c0 = k > l ? k - 1 : l;
        if (t >= c0 && t <= hi) {
          if (k > l && t == k - 1) {
            A[k * LD + t] = gr;
            A[(k + 1) * LD + t] = cx(0.0, 0.0);
          } else {
            const cplx h0 = A[k * LD + t], h1 = A[(k + 1) * LD + t];
            A[k * LD + t] = gc * h0 + gs * h1;
            A[(k + 1) * LD + t] = gc * h1 - conj(gs) * h0;
          }
        }
        __syncthreads();
        // columns k, k+1 over rows l .. min(k+2, hi), lane = row
        const int r1 = k + 2 < hi ? k + 2 : hi;
        if (t >= l && t <= r1) {
          const cplx h0 = A[t * LD + k], h1 = A[t * LD + k + 1];
          A[t * LD + k] = gc * h0 + conj(gs) * h1;
          A[t * LD + k + 1] = gc * h1 - gs * h0;
        }
        __syncthreads();
        work += 20.0 * (hi - c0 + 1) + 20.0 * (r1 - l + 1);
      }
      ++its;
      ++sweeps;
    }
    if (failed) {
      // report the current diagonal of the unconverged window
      for (int i = 0; i <= hi; ++i) {
        const cplx z = A[i * LD + i];
        if (t == 0 && eig) {
          eig[(p * N + i) * 2] = z.re;
          eig[(p * N + i) * 2 + 1] = z.im;
        }
        rad = fmax(rad, sqrt(abs2(z)));
      }
    }
    if (t == 0) {
      if (radius) radius[p] = rad;
      if (info) info[p] = failed ? -1 : sweeps;
      if (flops) flops[p] = work;
    }
  }
}

bool dims_ok(int32_t dim) { return dim == 2 || dim == 3; }

int64_t grid_of(int64_t npts) {
  // one workgroup per point up to a cap; the kernel loops over the rest
  const int64_t cap = int64_t{1} << 20;
  return npts < cap ? npts : cap;
}

}  // namespace

extern "C" {

int32_t lbm_spectrum_order(int32_t dim) { return dims_ok(dim) ? (dim + 1) * (2 * dim + 1) : 0; }

lbm_status lbm_spectrum_matrix(int32_t dim, int64_t npts, const lbm_lin_state* states, int32_t nstates,
                               const int32_t* state_of_point, const double* theta, double* E, void* stream) {
  if (!dims_ok(dim) || npts < 0 || nstates < 1) return LBM_EINVAL;
  if (npts == 0) return LBM_OK;
  if (!states || !theta || !E) return LBM_EINVAL;
  const int n = lbm_spectrum_order(dim);
  const int64_t rows = npts * n;
  const int64_t blocks = (rows + 255) / 256;
  if (blocks > INT32_MAX) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dim == 2)
    hipLaunchKernelGGL(k_spectrum_matrix<2>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, states, nstates,
                       state_of_point, theta, npts, E);
  else
    hipLaunchKernelGGL(k_spectrum_matrix<3>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, states, nstates,
                       state_of_point, theta, npts, E);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_spectrum_eigs(int32_t dim, int64_t npts, const lbm_lin_state* states, int32_t nstates,
                             const int32_t* state_of_point, const double* theta, double* eig, double* radius,
                             int32_t* info, double* flops, void* stream) {
  if (!dims_ok(dim) || npts < 0 || nstates < 1) return LBM_EINVAL;
  if (npts == 0) return LBM_OK;
  if (!states || !theta || (!eig && !radius && !info && !flops)) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<uint32_t>(grid_of(npts)));
  if (dim == 2)
    hipLaunchKernelGGL(k_spectrum_eigs<2>, grid, dim3(64), 0, s, states, nstates, state_of_point, theta, npts, eig,
                       radius, info, flops);
  else
    hipLaunchKernelGGL(k_spectrum_eigs<3>, grid, dim3(64), 0, s, states, nstates, state_of_point, theta, npts, eig,
                       radius, info, flops);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

}  // extern "C"
