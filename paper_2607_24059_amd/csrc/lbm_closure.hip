// Device-side pieces of the learned coarse-grid correction (contract in
// include/lbm_closure.h): restriction, network features, reset to equilibrium
// and the guarded moment correction.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "lbm.h"
#include "lbm_closure.h"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

constexpr int kThreads = 256;

// closure scratch slots (doubles) in the context workspace
constexpr int kSlotMean = 0;      // 0..3: grid means of the three channels (physical units)
constexpr int kSlotAccept = 4;    // 1.0 if accepted
constexpr int kSlotDiv0 = 5;      // ||div u||
constexpr int kSlotDiv1 = 6;      // ||div u'||
constexpr int kSlotNacc = 7;      // running count of accepted corrections
constexpr int kSlotNrej = 8;      // running count of rejected corrections

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  return s;
}

// --------------------------------------------------------------------------
__global__ void k_restrict(const float* __restrict__ fine, int nfx, int nfy, int r, double rho_ref,
                           float* __restrict__ coarse) {
  const int ncx = nfx / r, ncy = nfy / r;
  const int64_t cc = static_cast<int64_t>(ncx) * ncy;
  const int64_t fc = static_cast<int64_t>(nfx) * nfy;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 3 * cc) return;
  const int ch = static_cast<int>(idx / cc);
  const int64_t c = idx % cc;
  const int cx = static_cast<int>(c % ncx), cy = static_cast<int>(c / ncx);
  double s = 0.0;
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < r; ++i) s += fine[ch * fc + static_cast<int64_t>(cy * r + j) * nfx + cx * r + i];
  const double mean = s / (static_cast<double>(r) * r);
  coarse[idx] = static_cast<float>(ch == 0 ? rho_ref + static_cast<double>(r) * r * (mean - rho_ref) : mean);
}

__global__ void k_target(const float* __restrict__ mn, const float* __restrict__ m0, int64_t cells, float s_drho,
                         float s_dq, float* __restrict__ t) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 3 * cells) return;
  t[i] = (mn[i] - m0[i]) / (i < cells ? s_drho : s_dq);
}

__global__ void k_features(const float* __restrict__ m, int dim, int64_t cells, double rho_ref, float s_rho,
                           float s_u, float* __restrict__ x) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const float rho = m[c];
  x[c] = static_cast<float>((rho - rho_ref) / s_rho);
  for (int j = 0; j < dim; ++j) x[(1 + j) * cells + c] = (m[(1 + j) * cells + c] / rho) / s_u;
}

// --------------------------------------------------------------------------
// reset to the equilibrium of FP32 device moments (W = (rho, dx q))
// --------------------------------------------------------------------------
template <int D, typename TR, typename TM>
__global__ __launch_bounds__(256) void k_set_eq(const float* __restrict__ m, int64_t cells, int64_t stride,
                                                double dx, TR* __restrict__ rest, TM* __restrict__ move,
                                                CoefT<double> k) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const double rho = m[c];
  double W[D + 1];
  W[0] = rho - k.ref;
#pragma unroll
  for (int j = 0; j < D; ++j) W[1 + j] = dx * static_cast<double>(m[(1 + j) * cells + c]);
  if constexpr (StoresMoments<TM>::value) {  // the moments, no non-equilibrium part
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      store_real(rest + i * stride + c, W[i]);
      if constexpr (IsNeq<TM>::value) {
#pragma unroll
        for (int v = 0; v < 2 * D; ++v) store_f32(move + (i * 2 * D + v) * stride + c, 0.0f);
      }
    }
  } else {
    double eq[D + 1][2 * D + 1];
    equilibrium<D, double>(W, 1.0 / rho, k, eq);
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      store_real(rest + i * stride + c, eq[i][0]);
#pragma unroll
      for (int v = 0; v < 2 * D; ++v) store_real(move + (i * 2 * D + v) * stride + c, eq[i][1 + v]);
    }
  }
}

// --------------------------------------------------------------------------
// guarded correction (2D)
// --------------------------------------------------------------------------
// Deterministic reductions in two stages: per-block (or per-tile) FP64
// partials of 4 doubles in the context's diagnostics scratch, summed in a
// fixed order by every block of the next launch, so no launch is spent on
// the final sums alone.
constexpr int kRedSlots = 4;

// per-block sums of the three output channels
__global__ __launch_bounds__(kThreads) void k_cl_means(const float* __restrict__ y, int64_t cells,
                                                       double* __restrict__ part) {
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; c < cells;
         c += static_cast<int64_t>(gridDim.x) * kThreads)
      acc += static_cast<double>(y[ch * cells + c]);
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x * kRedSlots + ch] = s;
  }
}

// ---- the guard in two launches -------------------------------------------
// Sums of the first three entries of `count` 4-double partials, in a fixed
// order; every thread of the block receives them.
__device__ void reduce_partials3(const double* __restrict__ part, int64_t count, double (&out)[3]) {
  __shared__ double bc[3];
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kThreads) acc += part[i * kRedSlots + ch];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) bc[ch] = s;
  }
  __syncthreads();
  for (int ch = 0; ch < 3; ++ch) out[ch] = bc[ch];
  __syncthreads();
}

// Every block: the grid means of the output channels from their partial sums,
// then the divergence sums of u and u' over its cells (grid-stride) into
// div_part.  Block 0 records the means in the slots.
__global__ __launch_bounds__(kThreads) void k_cl_guard2(const float* __restrict__ m, const float* __restrict__ y,
                                                        int nx, int ny, double dx, float s_drho, float s_dq,
                                                        const double* __restrict__ mean_part, int64_t n_mean_part,
                                                        double* __restrict__ slots, double* __restrict__ div_part) {
  const int64_t cells = static_cast<int64_t>(nx) * ny;
  double sums[3];
  reduce_partials3(mean_part, n_mean_part, sums);
  double mean[3];
  for (int ch = 0; ch < 3; ++ch) mean[ch] = sums[ch] / static_cast<double>(cells) * (ch == 0 ? s_drho : s_dq);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int ch = 0; ch < 3; ++ch) slots[kSlotMean + ch] = mean[ch];
  auto uplain = [&](int x, int yy, int j) {
    const int64_t c = static_cast<int64_t>(yy) * nx + x;
    return static_cast<double>(m[(1 + j) * cells + c]) / static_cast<double>(m[c]);
  };
  auto ucorr = [&](int x, int yy, int j) {
    const int64_t c = static_cast<int64_t>(yy) * nx + x;
    const double rho = static_cast<double>(m[c]) + (static_cast<double>(y[c]) * s_drho - mean[0]);
    const double dq = static_cast<double>(y[(1 + j) * cells + c]) * s_dq - mean[1 + j];
    return (static_cast<double>(m[(1 + j) * cells + c]) + dq) / rho;
  };
  double a0 = 0.0, a1 = 0.0, bad = 0.0;
  const double inv2dx = 1.0 / (2.0 * dx);
  for (int64_t c = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; c < cells;
       c += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int x = static_cast<int>(c % nx), yy = static_cast<int>(c / nx);
    const int xp = wrapi(x + 1, nx), xm = wrapi(x - 1, nx), yp = wrapi(yy + 1, ny), ym = wrapi(yy - 1, ny);
    const double d0 = (uplain(xp, yy, 0) - uplain(xm, yy, 0)) * inv2dx + (uplain(x, yp, 1) - uplain(x, ym, 1)) * inv2dx;
    const double d1 = (ucorr(xp, yy, 0) - ucorr(xm, yy, 0)) * inv2dx + (ucorr(x, yp, 1) - ucorr(x, ym, 1)) * inv2dx;
    a0 += d0 * d0;
    a1 += d1 * d1;
    if (!isfinite(ucorr(x, yy, 0)) || !isfinite(ucorr(x, yy, 1))) bad += 1.0;
  }
  const double s0 = block_sum(a0);
  const double s1 = block_sum(a1);
  const double sb = block_sum(bad);
  if (threadIdx.x == 0) {
    div_part[blockIdx.x * kRedSlots + 0] = s0;
    div_part[blockIdx.x * kRedSlots + 1] = s1;
    div_part[blockIdx.x * kRedSlots + 2] = sb;
    div_part[blockIdx.x * kRedSlots + 3] = 0.0;
  }
}

// Every block takes the decision from the divergence partials (the same in
// all blocks), block 0 records it, and accepted corrections update the cells
// (one thread per cell): g += f^eq(W + dW) - f^eq(W).
template <int D, typename TR, typename TM>
__global__ __launch_bounds__(256) void k_cl_apply2(const float* __restrict__ y, int64_t cells, int64_t stride,
                                                   double dx, double ref, TR* __restrict__ rest,
                                                   TM* __restrict__ move, CoefT<double> k, float s_drho,
                                                   float s_dq, double* __restrict__ slots,
                                                   const double* __restrict__ div_part, int64_t n_div_part,
                                                   float factor) {
  double sums[3];
  reduce_partials3(div_part, n_div_part, sums);
  const double div0 = sqrt(dx * dx * sums[0]), div1 = sqrt(dx * dx * sums[1]);
  const bool ok = sums[2] == 0.0 && isfinite(div1) && div1 <= static_cast<double>(factor) * div0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    slots[kSlotDiv0] = div0;
    slots[kSlotDiv1] = div1;
    slots[kSlotAccept] = ok ? 1.0 : 0.0;
    slots[ok ? kSlotNacc : kSlotNrej] += 1.0;
  }
  if (!ok) return;
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  if constexpr (StoresMoments<TM>::value) {
    // split and moment-only storage: f + f^eq(W + dW) - f^eq(W) has moments
    // W + dW and the same non-equilibrium part, so only the moment planes change
    store_real(rest + c, load_f64(rest + c) + (static_cast<double>(y[c]) * s_drho - slots[kSlotMean]));
#pragma unroll
    for (int j = 0; j < D; ++j) {
      float* pr = rest + (1 + j) * stride + c;
      store_real(pr, load_f64(pr) + dx * (static_cast<double>(y[(1 + j) * cells + c]) * s_dq - slots[kSlotMean + 1 + j]));
    }
  } else {
    double W[D + 1];
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      double a = load_f64(rest + i * stride + c);
#pragma unroll
      for (int v = 0; v < 2 * D; ++v) a += load_f64(move + (i * 2 * D + v) * stride + c);
      W[i] = a;
    }
    W[0] += ref;  // full density; k.ref = 0 so both equilibria below are the plain ones
    double W1[D + 1];
    W1[0] = W[0] + (static_cast<double>(y[c]) * s_drho - slots[kSlotMean]);
#pragma unroll
    for (int j = 0; j < D; ++j)
      W1[1 + j] = W[1 + j] + dx * (static_cast<double>(y[(1 + j) * cells + c]) * s_dq - slots[kSlotMean + 1 + j]);
    double e0[D + 1][2 * D + 1], e1[D + 1][2 * D + 1];
    equilibrium<D, double>(W, 1.0 / W[0], k, e0);
    equilibrium<D, double>(W1, 1.0 / W1[0], k, e1);
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      TR* pr = rest + i * stride + c;
      store_real(pr, load_f64(pr) + (e1[i][0] - e0[i][0]));
#pragma unroll
      for (int v = 0; v < 2 * D; ++v) {
        TM* pm = move + (i * 2 * D + v) * stride + c;
        store_real(pm, load_f64(pm) + (e1[i][1 + v] - e0[i][1 + v]));
      }
    }
  }
}

template <int D, typename TR, typename TM, bool DEV>
struct ClosureImpl {
  static hipError_t set_eq(lbm_ctx* c, const float* m) {
    auto p = planes_of<TR, TM>(c->cur, c->g.rest_bytes);
    const CoefT<double> k = make_coef<double>(c->coef, D, DEV);
    hipLaunchKernelGGL((k_set_eq<D, TR, TM>), dim3(static_cast<unsigned>((c->g.cells + 255) / 256)), dim3(256),
                       0, c->stream, m, c->g.cells, c->g.stride, c->coef.dx, p.rest, p.move, k);
    return hipGetLastError();
  }
  static hipError_t apply(lbm_ctx* c, const float* y, float s_drho, float s_dq, double* slots,
                          const double* div_part, int64_t n_div_part, float factor) {
    auto p = planes_of<TR, TM>(c->cur, c->g.rest_bytes);
    const CoefT<double> k = make_coef<double>(c->coef, D, false);
    hipLaunchKernelGGL((k_cl_apply2<D, TR, TM>), dim3(static_cast<unsigned>((c->g.cells + 255) / 256)),
                       dim3(256), 0, c->stream, y, c->g.cells, c->g.stride, c->coef.dx, DEV ? c->coef.ref : 0.0,
                       p.rest, p.move, k, s_drho, s_dq, slots, div_part, n_div_part, factor);
    return hipGetLastError();
  }
};

template <int D>
hipError_t dispatch_set_eq(lbm_ctx* c, const float* m) {
  switch (c->p.storage) {
    case LBM_F32: return ClosureImpl<D, float, float, true>::set_eq(c, m);
    case LBM_F32_RAW: return ClosureImpl<D, float, float, false>::set_eq(c, m);
    case LBM_F16_DEV: return ClosureImpl<D, _Float16, _Float16, true>::set_eq(c, m);
    case LBM_BF16_DEV: return ClosureImpl<D, bf16, bf16, true>::set_eq(c, m);
    case LBM_F16_DEV_R32: return ClosureImpl<D, float, _Float16, true>::set_eq(c, m);
    case LBM_BF16_DEV_R32: return ClosureImpl<D, float, bf16, true>::set_eq(c, m);
    case LBM_F64: return ClosureImpl<D, double, double, true>::set_eq(c, m);
    case LBM_F16_NEQ: return ClosureImpl<D, float, neq16, true>::set_eq(c, m);
    case LBM_F32_MOMENTS: return ClosureImpl<D, float, mom0, true>::set_eq(c, m);
  }
  return hipErrorInvalidValue;
}

hipError_t dispatch_apply(lbm_ctx* c, const float* y, float s_drho, float s_dq, double* slots,
                          const double* div_part, int64_t n, float factor) {
  switch (c->p.storage) {
    case LBM_F32: return ClosureImpl<2, float, float, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F32_RAW: return ClosureImpl<2, float, float, false>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F16_DEV: return ClosureImpl<2, _Float16, _Float16, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_BF16_DEV: return ClosureImpl<2, bf16, bf16, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F16_DEV_R32: return ClosureImpl<2, float, _Float16, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_BF16_DEV_R32: return ClosureImpl<2, float, bf16, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F64: return ClosureImpl<2, double, double, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F16_NEQ: return ClosureImpl<2, float, neq16, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
    case LBM_F32_MOMENTS: return ClosureImpl<2, float, mom0, true>::apply(c, y, s_drho, s_dq, slots, div_part, n, factor);
  }
  return hipErrorInvalidValue;
}

// Guard blocks: one per 256 cells, at most 256 (each block reduces every
// partial of the previous stage, so their number is kept small).
int guard_blocks(int64_t cells) {
  int64_t nb = cells / 256;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return static_cast<int>(nb);
}

// The guard and the guarded update, from per-tile (or per-block) FP64 sums of
// the network output in mean_part; the divergence partials go after them in
// the context's scratch.
hipError_t guard_and_apply(lbm_ctx* c, const float* moments, const float* y, float s_drho, float s_dq, float factor,
                           const double* mean_part, int64_t n_mean_part, double* div_part) {
  const int nbg = guard_blocks(c->g.cells);
  hipLaunchKernelGGL(k_cl_guard2, dim3(nbg), dim3(kThreads), 0, c->stream, moments, y, c->g.nx, c->g.ny, c->p.dx,
                     s_drho, s_dq, mean_part, n_mean_part, c->closure_slots, div_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return dispatch_apply(c, y, s_drho, s_dq, c->closure_slots, div_part, nbg, factor);
}

// --------------------------------------------------------------------------
// divergence-free part of a momentum difference (2D, n x n periodic): the
// spectral Helmholtz projection d^(k) - k (k . d^(k)) / |k|^2 for k != 0, with
// signed wavenumbers k = m for m < n/2 and m - n otherwise, the mean kept.
// Three launches of FP64 discrete Fourier sums (the transform of the row, of
// the column with the projection and the inverse column transform, and the
// inverse row transform), each block holding the twiddles exp(-2 pi i m / n),
// m < n, in LDS; O(n^3) work, a fraction of a millisecond at 256^2.
// --------------------------------------------------------------------------
constexpr int kProjMaxN = 1024;

__device__ __forceinline__ void load_twiddles(double2* tw, int n) {
  for (int m = threadIdx.x; m < n; m += kThreads) {
    double sn, cs;
    sincospi(2.0 * m / n, &sn, &cs);
    tw[m] = make_double2(cs, -sn);
  }
}

// A[c][y][kx] = sum_x d_c(x, y) exp(-2 pi i kx x / n), d = fine - now (q planes)
__global__ __launch_bounds__(kThreads) void k_proj_rows(const float* __restrict__ fine, const float* __restrict__ now,
                                                        int n, double2* __restrict__ A) {
  __shared__ double2 tw[kProjMaxN];
  __shared__ double d[kProjMaxN];
  const int y = blockIdx.x, c = blockIdx.y;  // c = 0, 1: q_x, q_y (moment planes 1, 2)
  const int64_t cells = static_cast<int64_t>(n) * n;
  load_twiddles(tw, n);
  for (int x = threadIdx.x; x < n; x += kThreads) {
    const int64_t i = (1 + c) * cells + static_cast<int64_t>(y) * n + x;
    d[x] = static_cast<double>(fine[i]) - static_cast<double>(now[i]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += kThreads) {
    double re = 0.0, im = 0.0;
    int m = 0;  // k x mod n
    for (int x = 0; x < n; ++x) {
      re = fma(d[x], tw[m].x, re);
      im = fma(d[x], tw[m].y, im);
      m += k;
      if (m >= n) m -= n;
    }
    A[(static_cast<int64_t>(c) * n + y) * n + k] = make_double2(re, im);
  }
}

// Column kx of both components: forward transform along y, projection,
// inverse transform along y (unnormalised), back into A.
__global__ __launch_bounds__(kThreads) void k_proj_cols(int n, double2* __restrict__ A) {
  __shared__ double2 tw[kProjMaxN];
  __shared__ double2 col[2][kProjMaxN];
  __shared__ double2 hat[2][kProjMaxN];
  const int kx = blockIdx.x;
  const int sx = kx < (n + 1) / 2 ? kx : kx - n;  // signed wavenumber, as numpy's fftfreq
  load_twiddles(tw, n);
  for (int y = threadIdx.x; y < n; y += kThreads)
    for (int c = 0; c < 2; ++c) col[c][y] = A[(static_cast<int64_t>(c) * n + y) * n + kx];
  __syncthreads();
  for (int ky = threadIdx.x; ky < n; ky += kThreads) {
    double2 h[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    int m = 0;  // ky y mod n
    for (int y = 0; y < n; ++y) {
      const double2 t = tw[m];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        h[c].x = fma(col[c][y].x, t.x, fma(-col[c][y].y, t.y, h[c].x));
        h[c].y = fma(col[c][y].x, t.y, fma(col[c][y].y, t.x, h[c].y));
      }
      m += ky;
      if (m >= n) m -= n;
    }
    const int sy = ky < (n + 1) / 2 ? ky : ky - n;
    const double k2 = static_cast<double>(sx) * sx + static_cast<double>(sy) * sy;
    if (k2 > 0.0) {
      const double dre = (sx * h[0].x + sy * h[1].x) / k2, dim = (sx * h[0].y + sy * h[1].y) / k2;
      h[0].x -= sx * dre;
      h[0].y -= sx * dim;
      h[1].x -= sy * dre;
      h[1].y -= sy * dim;
    }
    hat[0][ky] = h[0];
    hat[1][ky] = h[1];
  }
  __syncthreads();
  for (int y = threadIdx.x; y < n; y += kThreads) {
    double2 v[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    int m = 0;  // ky y mod n; the inverse uses the conjugate twiddle
    for (int ky = 0; ky < n; ++ky) {
      const double2 t = tw[m];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        v[c].x = fma(hat[c][ky].x, t.x, fma(hat[c][ky].y, t.y, v[c].x));
        v[c].y = fma(hat[c][ky].y, t.x, fma(-hat[c][ky].x, t.y, v[c].y));
      }
      m += y;
      if (m >= n) m -= n;
    }
    for (int c = 0; c < 2; ++c) A[(static_cast<int64_t>(c) * n + y) * n + kx] = v[c];
  }
}

// Inverse transform along x, real part, 1/n^2: out_q = now_q + P(d); out_rho = now_rho.
__global__ __launch_bounds__(kThreads) void k_proj_out(const float* __restrict__ now, int n,
                                                       const double2* __restrict__ A, float* __restrict__ out) {
  __shared__ double2 tw[kProjMaxN];
  __shared__ double2 row[kProjMaxN];
  const int y = blockIdx.x, c = blockIdx.y;
  const int64_t cells = static_cast<int64_t>(n) * n;
  load_twiddles(tw, n);
  for (int k = threadIdx.x; k < n; k += kThreads) row[k] = A[(static_cast<int64_t>(c) * n + y) * n + k];
  __syncthreads();
  const double scale = 1.0 / (static_cast<double>(n) * n);
  for (int x = threadIdx.x; x < n; x += kThreads) {
    double re = 0.0;
    int m = 0;  // k x mod n
    for (int k = 0; k < n; ++k) {
      re = fma(row[k].x, tw[m].x, fma(row[k].y, tw[m].y, re));  // real part of row[k] conj(tw[m])
      m += x;
      if (m >= n) m -= n;
    }
    const int64_t i = static_cast<int64_t>(y) * n + x;
    out[(1 + c) * cells + i] = static_cast<float>(static_cast<double>(now[(1 + c) * cells + i]) + re * scale);
    if (c == 0) out[i] = now[i];
  }
}

lbm_status dev(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

lbm_status lbm_restrict(const float* fine, int64_t nfx, int64_t nfy, int32_t r, double rho_ref, float* coarse,
                        void* stream) {
  if (!fine || !coarse || r < 1 || nfx < r || nfy < r || nfx % r || nfy % r || nfx > (1 << 30) || nfy > (1 << 30))
    return LBM_EINVAL;
  const int64_t n = 3 * (nfx / r) * (nfy / r);
  hipLaunchKernelGGL(k_restrict, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), fine, static_cast<int>(nfx), static_cast<int>(nfy), r, rho_ref,
                     coarse);
  return dev(hipGetLastError());
}

lbm_status lbm_closure_features(const float* moments, int32_t dim, int64_t cells, double rho_ref, float s_rho,
                                float s_u, float* x, void* stream) {
  if (!moments || !x || (dim != 2 && dim != 3) || cells < 1 || !(s_rho > 0) || !(s_u > 0)) return LBM_EINVAL;
  hipLaunchKernelGGL(k_features, dim3(static_cast<unsigned>((cells + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), moments, dim, cells, rho_ref, s_rho, s_u, x);
  return dev(hipGetLastError());
}

lbm_status lbm_closure_target(const float* m_next, const float* m_now, int64_t cells, float s_drho, float s_dq,
                              float* t, void* stream) {
  if (!m_next || !m_now || !t || cells < 1 || !(s_drho > 0) || !(s_dq > 0)) return LBM_EINVAL;
  hipLaunchKernelGGL(k_target, dim3(static_cast<unsigned>((3 * cells + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), m_next, m_now, cells, s_drho, s_dq, t);
  return dev(hipGetLastError());
}

size_t lbm_closure_project_scratch_bytes(int32_t n) {
  if (n < 1 || n > kProjMaxN) return 0;
  return 2 * static_cast<size_t>(n) * n * sizeof(double2);
}

lbm_status lbm_closure_project(const float* m_fine, const float* m_now, int32_t n, float* out, void* scratch,
                               void* stream) {
  if (!m_fine || !m_now || !out || !scratch || n < 1 || n > kProjMaxN) return LBM_EINVAL;
  if (out == m_fine || out == m_now) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double2* A = static_cast<double2*>(scratch);
  hipLaunchKernelGGL(k_proj_rows, dim3(n, 2), dim3(kThreads), 0, s, m_fine, m_now, n, A);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_proj_cols, dim3(n), dim3(kThreads), 0, s, n, A);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_proj_out, dim3(n, 2), dim3(kThreads), 0, s, m_now, n, A, out);
    e = hipGetLastError();
  }
  return dev(e);
}

lbm_status lbm_set_equilibrium_device(lbm_ctx* c, const float* moments) {
  if (!c || !moments) return LBM_EINVAL;
  return dev(c->p.dim == 2 ? dispatch_set_eq<2>(c, moments) : dispatch_set_eq<3>(c, moments));
}

lbm_status lbm_closure_apply(lbm_ctx* c, const float* moments, const float* y, float s_drho, float s_dq,
                             float guard_factor) {
  if (!c || !moments || !y || c->p.dim != 2 || !(guard_factor > 0)) return LBM_EINVAL;
  // the context's partials region: mean partials, then divergence partials
  double* part = c->partials;
  const int nbm = guard_blocks(c->g.cells);
  if (static_cast<int64_t>(2 * nbm) * kRedSlots > c->part_doubles) return LBM_EINVAL;
  hipLaunchKernelGGL(k_cl_means, dim3(nbm), dim3(kThreads), 0, c->stream, y, c->g.cells, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = guard_and_apply(c, moments, y, s_drho, s_dq, guard_factor, part, nbm, part + nbm * kRedSlots);
  return dev(e);
}

lbm_status lbm_closure_correct(lbm_ctx* c, const void* const* packed, const float* const* bias, float s_rho,
                               float s_u, float s_drho, float s_dq, float guard_factor, float* moments, float* y) {
  if (!c || !packed || !bias || !moments || !y || c->p.dim != 2 || !(guard_factor > 0) || !(s_rho > 0) ||
      !(s_u > 0))
    return LBM_EINVAL;
  for (int l = 0; l < 4; ++l)
    if (!packed[l] || !bias[l]) return LBM_EINVAL;
  const int64_t tiles = net_infer_tiles(c->g.ny, c->g.nx);
  const int nbg = guard_blocks(c->g.cells);
  if (tiles == 0 || (tiles + nbg) * kRedSlots > c->part_doubles) return LBM_EINVAL;
  double* part = c->partials;
  hipError_t e = c->ops->moments(c->g, c->coef, c->cur, nullptr, moments, c->stream);
  if (e == hipSuccess)
    e = net_infer_launch(moments, c->g.ny, c->g.nx, c->p.rho_ref, s_rho, s_u, packed, bias, y, part, c->stream);
  if (e == hipSuccess)
    e = guard_and_apply(c, moments, y, s_drho, s_dq, guard_factor, part, tiles, part + tiles * kRedSlots);
  return dev(e);
}

lbm_status lbm_closure_report_get(lbm_ctx* c, lbm_closure_report* out) {
  if (!c || !out) return LBM_EINVAL;
  double s[16];
  hipError_t e = hipMemcpyAsync(s, c->closure_slots, sizeof(s), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return LBM_EDEVICE;
  memset(out, 0, sizeof(*out));
  out->n_accepted = static_cast<int64_t>(s[kSlotNacc]);
  out->n_rejected = static_cast<int64_t>(s[kSlotNrej]);
  out->accepted = s[kSlotAccept] != 0.0;
  out->div_before = s[kSlotDiv0];
  out->div_after = s[kSlotDiv1];
  for (int i = 0; i < 3; ++i) out->mean[i] = s[kSlotMean + i];
  return LBM_OK;
}

}  // extern "C"
