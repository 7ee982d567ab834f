// 3x3 periodic convolutions on BF16 matrix cores, their gradients, MSE and
// Adam (contract in include/lbm_cnn.h).
//
// The convolution is an implicit GEMM per 64-pixel row segment:
//   D[p][co] = sum_k A[p][k] B[k][co],  k = tap * CIN_PAD + ci,
//   A[p][k]  = X[ci][y + dy(tap)][x0 + p + dx(tap)],  B[k][co] = W[co][ci][tap]
// with one v_mfma_f32_16x16x16_bf16 per (16 pixels, 16 output channels, 16 k).
// Operand fragments of a 64-lane wave (lane l, i = l % 16, q = l / 16):
//   A: row i, k = 4q .. 4q+3      B: column i, k = 4q .. 4q+3
//   D: column i, rows 4q .. 4q+3 (four FP32 accumulators)
// The input tile (3 rows x 66 columns, channel-last, BF16) and the packed
// weights live in LDS; k runs over CIN_PAD consecutive channels of one tap, so
// each fragment is one 8-byte LDS read.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_cnn.h"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct NetWeights {
  const uint16_t* packed[4];  // forward-packed BF16 operands of the four layers
  const float* bias[4];
};

constexpr int kSeg = 64;       // pixels per block row segment
constexpr int kThreads = 256;  // 4 waves, 16 pixels each
constexpr int kWgradRows = 16; // rows accumulated per weight-gradient block

__host__ __device__ constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }
__host__ __device__ constexpr int cin_pad(int cin) { return round_up(cin, 4); }
__host__ __device__ constexpr int cout_pad(int cout) { return round_up(cout, 16); }
__host__ __device__ constexpr int k_pad(int cinp) { return round_up(9 * cinp, 16); }

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ----------------------------------------------------------------------------
// weight packing: packed[co][k] (BF16 bits), k = tap * cin_pad + ci
// ----------------------------------------------------------------------------
__global__ void k_conv_pack(const float* __restrict__ w, int cin, int cout, int transpose,
                            uint16_t* __restrict__ packed) {
  // the packed operand has cin' = transpose ? cout : cin inputs and cout' outputs
  const int ci_n = transpose ? cout : cin;
  const int co_n = transpose ? cin : cout;
  const int cinp = cin_pad(ci_n), coutp = cout_pad(co_n), kp = k_pad(cinp);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= coutp * kp) return;
  const int co = idx / kp, k = idx % kp;
  const int tap = k / cinp, ci = k % cinp;
  float v = 0.0f;
  if (co < co_n && ci < ci_n && tap < 9) {
    // forward: W[co][ci][tap]; input gradient: W'[co'][ci'][tap] = W[ci'][co'][8 - tap]
    v = transpose ? w[(ci * cin + co) * 9 + (8 - tap)] : w[(co * cin + ci) * 9 + tap];
  }
  packed[idx] = bf16_bits(v);
}

// ----------------------------------------------------------------------------
// forward convolution
// ----------------------------------------------------------------------------
template <int CINP, int COUTP>
__global__ __launch_bounds__(kThreads) void k_conv_fwd(const float* __restrict__ x, int cin, int h, int w,
                                                      const uint16_t* __restrict__ packed, int cout,
                                                      const float* __restrict__ bias,
                                                      const float* __restrict__ mask, unsigned flags,
                                                      float* __restrict__ y) {
  constexpr int KP = k_pad(CINP);
  constexpr int NT = COUTP / 16;
  constexpr int KS = KP / 16;
  __shared__ __attribute__((aligned(16))) uint16_t xs[3][kSeg + 2][CINP];
  __shared__ __attribute__((aligned(16))) uint16_t ws[COUTP][KP];
  const int x0 = blockIdx.x * kSeg, row = blockIdx.y, b = blockIdx.z;
  const int64_t plane = static_cast<int64_t>(h) * w;
  const float* xb = x + static_cast<int64_t>(b) * cin * plane;

  for (int i = threadIdx.x; i < COUTP * KP; i += kThreads) (&ws[0][0])[i] = packed[i];
  for (int i = threadIdx.x; i < 3 * (kSeg + 2) * CINP; i += kThreads) {
    const int c = i % (kSeg + 2);
    const int r = (i / (kSeg + 2)) % 3;
    const int ci = i / (3 * (kSeg + 2));
    float v = 0.0f;
    if (ci < cin) {
      const int gy = wrapi(row + r - 1, h), gx = wrapi(x0 + c - 1, w);
      v = xb[ci * plane + static_cast<int64_t>(gy) * w + gx];
    }
    xs[r][c][ci] = bf16_bits(v);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int p0 = wave * 16;
  f4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k0 = ks * 16 + 4 * lq;
    const int tap = k0 / CINP, ci0 = k0 % CINP;
    s4 a = s4{0, 0, 0, 0};
    if (tap < 9) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      a = *reinterpret_cast<const s4*>(&xs[1 + dy][1 + p0 + li + dx][ci0]);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const s4 bb = *reinterpret_cast<const s4*>(&ws[nt * 16 + li][k0]);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[nt], 0, 0, 0);
    }
  }
  // epilogue: lane holds output channel co = nt*16 + li for pixels p0 + 4*lq + r
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int co = nt * 16 + li;
    if (co >= cout) continue;
    const float bv = bias ? bias[co] : 0.0f;
    const int64_t base = (static_cast<int64_t>(b) * cout + co) * plane + static_cast<int64_t>(row) * w + x0 + p0 + 4 * lq;
    float4 o;
    float* op = reinterpret_cast<float*>(&o);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v = acc[nt][r] + bv;
      if (flags & LBM_CONV_RELU) v = fmaxf(v, 0.0f);
      op[r] = v;
    }
    if (mask) {
      const float4 mv = *reinterpret_cast<const float4*>(mask + base);
      o.x = mv.x > 0.0f ? o.x : 0.0f;
      o.y = mv.y > 0.0f ? o.y : 0.0f;
      o.z = mv.z > 0.0f ? o.z : 0.0f;
      o.w = mv.w > 0.0f ? o.w : 0.0f;
    }
    *reinterpret_cast<float4*>(y + base) = o;
  }
}

// ----------------------------------------------------------------------------
// weight gradient: D[co][k] = sum_p dY[co][p] Xpatch[p][k] over the block's pixels
//   A[co][p] = dY (rows of the MFMA = output channels), B[p][k] = input patches
// ----------------------------------------------------------------------------
template <int CINP, int COUTP>
__global__ __launch_bounds__(kThreads) void k_conv_wgrad(const float* __restrict__ x,
                                                        const float* __restrict__ dy, int cin, int cout,
                                                        int h, int w, float* __restrict__ part_w,
                                                        float* __restrict__ part_b) {
  constexpr int KP = k_pad(CINP);
  constexpr int MT = COUTP / 16;
  constexpr int NTT = KP / 16;
  constexpr int TILES = MT * NTT;
  constexpr int TPW = (TILES + 3) / 4;  // output tiles per wave
  __shared__ __attribute__((aligned(16))) uint16_t xs[3][kSeg + 2][CINP];
  __shared__ __attribute__((aligned(16))) uint16_t ds[COUTP][kSeg];
  __shared__ float dbs[COUTP];
  const int x0 = blockIdx.x * kSeg, y0 = blockIdx.y * kWgradRows, b = blockIdx.z;
  const int64_t plane = static_cast<int64_t>(h) * w;
  const float* xb = x + static_cast<int64_t>(b) * cin * plane;
  const float* db_ = dy + static_cast<int64_t>(b) * cout * plane;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;

  f4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float dbsum = 0.0f;  // thread co < COUTP accumulates the bias gradient of channel co

  const int y1 = min(y0 + kWgradRows, h);
  for (int row = y0; row < y1; ++row) {
    __syncthreads();  // previous row's LDS reads are done
    for (int i = threadIdx.x; i < 3 * (kSeg + 2) * CINP; i += kThreads) {
      const int c = i % (kSeg + 2);
      const int r = (i / (kSeg + 2)) % 3;
      const int ci = i / (3 * (kSeg + 2));
      float v = 0.0f;
      if (ci < cin) {
        const int gy = wrapi(row + r - 1, h), gx = wrapi(x0 + c - 1, w);
        v = xb[ci * plane + static_cast<int64_t>(gy) * w + gx];
      }
      xs[r][c][ci] = bf16_bits(v);
    }
    for (int i = threadIdx.x; i < COUTP * kSeg; i += kThreads) {
      const int p = i % kSeg, co = i / kSeg;
      const float v = co < cout ? db_[co * plane + static_cast<int64_t>(row) * w + x0 + p] : 0.0f;
      ds[co][p] = bf16_bits(v);
    }
    if (threadIdx.x < COUTP && threadIdx.x < cout) {
      const float* src = db_ + threadIdx.x * plane + static_cast<int64_t>(row) * w + x0;
      float s = 0.0f;
      for (int p = 0; p < kSeg; ++p) s += src[p];
      dbsum += s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= TILES) break;
      const int mt = tile / NTT, nt = tile % NTT;
      const int co = mt * 16 + li;          // A row of this lane
      const int k = nt * 16 + li;           // B column of this lane
      const int tap = k / CINP, ci = k % CINP;
      const bool valid = tap < 9;
      const int dyo = valid ? tap / 3 - 1 : 0, dxo = valid ? tap % 3 - 1 : 0;
#pragma unroll
      for (int ps = 0; ps < kSeg / 16; ++ps) {
        const int p = ps * 16 + 4 * lq;
        const s4 a = *reinterpret_cast<const s4*>(&ds[co][p]);
        s4 bb = s4{0, 0, 0, 0};
        if (valid) {
#pragma unroll
          for (int r = 0; r < 4; ++r) bb[r] = static_cast<short>(xs[1 + dyo][1 + p + r + dxo][ci]);
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[t], 0, 0, 0);
      }
    }
  }
  // partials of this block: D[co][k] lives in lane (col = k), rows co = mt*16 + 4*lq + r
  const int64_t blk = (static_cast<int64_t>(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  float* pw = part_w + blk * (COUTP * KP);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= TILES) break;
    const int mt = tile / NTT, nt = tile % NTT;
#pragma unroll
    for (int r = 0; r < 4; ++r) pw[(mt * 16 + 4 * lq + r) * KP + nt * 16 + li] = acc[t][r];
  }
  if (threadIdx.x < COUTP) {
    dbs[threadIdx.x] = threadIdx.x < cout ? dbsum : 0.0f;
    part_b[blk * COUTP + threadIdx.x] = dbs[threadIdx.x];
  }
}

// fixed-order sum of the partials into dw[co][ci][tap] and db[co]
__global__ void k_wgrad_reduce(const float* __restrict__ part_w, const float* __restrict__ part_b,
                               int64_t nblocks, int cin, int cout, int cinp, int coutp, int kp,
                               float* __restrict__ dw, float* __restrict__ db) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = cout * cin * 9;
  if (idx < nw) {
    const int co = idx / (cin * 9), ci = (idx / 9) % cin, tap = idx % 9;
    const int k = tap * cinp + ci;
    float s = 0.0f;
    for (int64_t bl = 0; bl < nblocks; ++bl) s += part_w[bl * coutp * kp + co * kp + k];
    dw[idx] = s;
  } else if (idx < nw + cout) {
    const int co = idx - nw;
    float s = 0.0f;
    for (int64_t bl = 0; bl < nblocks; ++bl) s += part_b[bl * coutp + co];
    db[co] = s;
  }
}

// ----------------------------------------------------------------------------
// reductions (FP64, fixed order), MSE, Adam
// ----------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;

__device__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(kThreads) void k_mse(const float* __restrict__ out, const float* __restrict__ tgt,
                                                  int64_t n, float* __restrict__ grad, double* __restrict__ part) {
  double acc = 0.0;
  const float scale = 2.0f / static_cast<float>(n);
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const float d = out[i] - tgt[i];
    grad[i] = scale * d;
    acc += static_cast<double>(d) * d;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_sumsq(const float* __restrict__ x, int64_t n,
                                                    double* __restrict__ part) {
  double acc = 0.0;
  const float* xc = x + static_cast<int64_t>(blockIdx.y) * n;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    acc += static_cast<double>(xc[i]) * xc[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// out[c] = f(sum of part[c][0..nb)) with f = x / n (mean) or sqrt(x / n) (rms)
__global__ __launch_bounds__(kThreads) void k_finish(const double* __restrict__ part, int nb, int64_t n,
                                                     int root, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += part[blockIdx.x * nb + i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = root ? sqrt(s / static_cast<double>(n)) : s / static_cast<double>(n);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------------------
// fused inference of the correction network (3 -> 32 -> 32 -> 32 -> 3)
//
// One block computes a 16 x 16 output tile through all four layers.  The
// layers shrink the region by one pixel per side, so the block loads a
// 24 x 24 input region (periodic wrap) and keeps every intermediate
// activation (22^2, 20^2, 18^2 pixels x 32 channels, channel-last BF16) in
// LDS.  The recomputed borders cost (22^2 + 20^2 + 18^2) / (3 * 16^2) = 1.57x
// the MFMA work of the three inner layers, in exchange for no activation
// traffic to HBM and one launch instead of five.  Each wave keeps the B
// fragments (weights) of the current layer in registers and walks 16-pixel
// M-tiles of the layer's output region.  The k order, the MFMA sequence, the
// bias, the ReLU and the BF16 rounding of each activation are those of
// k_conv_fwd, so the output equals the layer-by-layer forward bit for bit.
// ----------------------------------------------------------------------------
constexpr int kInfT = 16;        // output tile edge
constexpr int kInfS0 = kInfT + 8;  // input region edge (halo 4)
constexpr int kInfCh = 32;       // hidden channels
constexpr int kInfStride = 40;   // LDS elements per pixel of a hidden activation (32 + 8 pad)
constexpr int kInferWaves = 8;   // waves per block
constexpr int kInferMP = 4;      // M-tiles in flight per wave (8 x 4 = 32 M-tiles: one round of the 22^2 layer)

// One layer on the block's LDS regions: input region SIN x SIN (pixel stride
// IN_STRIDE elements), output region SOUT = SIN - 2.  NW waves split the
// 16-pixel M-tiles; each wave carries MP M-tiles at once (MP x NT independent
// accumulator chains, to keep the matrix pipeline busy).
template <int CINP, int COUTP, int SIN, int IN_STRIDE, bool LAST, int NW, int MP>
__device__ __forceinline__ void infer_layer(const uint16_t* in, uint16_t* out, const uint16_t* __restrict__ packed,
                                            const float* __restrict__ bias, float* ys) {
  constexpr int SOUT = SIN - 2;
  constexpr int KP = k_pad(CINP);
  constexpr int KS = KP / 16;
  constexpr int NT = COUTP / 16;
  constexpr int NPIX = SOUT * SOUT;
  constexpr int MT = (NPIX + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  s4 bf[NT][KS];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      bf[nt][ks] = *reinterpret_cast<const s4*>(packed + (nt * 16 + li) * KP + ks * 16 + 4 * lq);
  for (int mt0 = wave * MP; mt0 < MT; mt0 += NW * MP) {
    int oy[MP], ox[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      int o = (mt0 + j) * 16 + li;
      if (o >= NPIX) o = NPIX - 1;  // padding rows of the last M-tile: read a valid pixel, result dropped
      oy[j] = o / SOUT;
      ox[j] = o % SOUT;
    }
    f4 acc[MP][NT];
#pragma unroll
    for (int j = 0; j < MP; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[j][nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k0 = ks * 16 + 4 * lq;
      const int tap = k0 / CINP, ci0 = k0 % CINP;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      s4 a[MP];
#pragma unroll
      for (int j = 0; j < MP; ++j) {
        a[j] = s4{0, 0, 0, 0};
        if (tap < 9) a[j] = *reinterpret_cast<const s4*>(in + ((oy[j] + 1 + dy) * SIN + (ox[j] + 1 + dx)) * IN_STRIDE + ci0);
      }
#pragma unroll
      for (int j = 0; j < MP; ++j)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[j][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[j], bf[nt][ks], acc[j][nt], 0, 0, 0);
    }
    // lane holds output channel nt*16 + li of pixels (mt0 + j)*16 + 4*lq + r
#pragma unroll
    for (int j = 0; j < MP; ++j) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + li;
        if (LAST && co >= 3) continue;
        const float bv = bias[co];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int op = (mt0 + j) * 16 + 4 * lq + r;
          if (op >= NPIX) continue;
          float v = acc[j][nt][r] + bv;
          if (LAST) {
            ys[co * NPIX + op] = v;
          } else {
            v = fmaxf(v, 0.0f);
            out[op * kInfStride + co] = bf16_bits(v);
          }
        }
      }
    }
  }
}

template <int NW, int MP>
__global__ __launch_bounds__(NW * 64) void k_net_infer(const float* __restrict__ m, int h, int w, double rho_ref,
                                                       float s_rho, float s_u, NetWeights nw,
                                                       float* __restrict__ y, double* __restrict__ part) {
  constexpr int NTH = NW * 64;
  __shared__ __attribute__((aligned(16))) uint16_t a0[kInfS0 * kInfS0 * 4];
  __shared__ __attribute__((aligned(16))) uint16_t a1[(kInfS0 - 2) * (kInfS0 - 2) * kInfStride];
  __shared__ __attribute__((aligned(16))) uint16_t a2[(kInfS0 - 4) * (kInfS0 - 4) * kInfStride];
  __shared__ float ys[3 * kInfT * kInfT];
  __shared__ double red[NW][3];
  const int tx0 = blockIdx.x * kInfT, ty0 = blockIdx.y * kInfT;
  const int64_t cells = static_cast<int64_t>(h) * w;
  // features of the input region, as lbm_closure_features computes them
  for (int i = threadIdx.x; i < kInfS0 * kInfS0; i += NTH) {
    const int ry = i / kInfS0, rx = i % kInfS0;
    const int gy = ((ty0 - 4 + ry) % h + h) % h, gx = ((tx0 - 4 + rx) % w + w) % w;
    const int64_t c = static_cast<int64_t>(gy) * w + gx;
    const float rho = m[c];
    a0[i * 4 + 0] = bf16_bits(static_cast<float>((rho - rho_ref) / s_rho));
    a0[i * 4 + 1] = bf16_bits((m[cells + c] / rho) / s_u);
    a0[i * 4 + 2] = bf16_bits((m[2 * cells + c] / rho) / s_u);
    a0[i * 4 + 3] = 0;
  }
  __syncthreads();
  infer_layer<4, kInfCh, kInfS0, 4, false, NW, MP>(a0, a1, nw.packed[0], nw.bias[0], nullptr);
  __syncthreads();
  infer_layer<kInfCh, kInfCh, kInfS0 - 2, kInfStride, false, NW, MP>(a1, a2, nw.packed[1], nw.bias[1], nullptr);
  __syncthreads();
  infer_layer<kInfCh, kInfCh, kInfS0 - 4, kInfStride, false, NW, MP>(a2, a1, nw.packed[2], nw.bias[2], nullptr);
  __syncthreads();
  infer_layer<kInfCh, 16, kInfS0 - 6, kInfStride, true, NW, MP>(a1, nullptr, nw.packed[3], nw.bias[3], ys);
  __syncthreads();
  // output tile and its per-channel FP64 sums (fixed order: pixels in thread
  // order within a wave by a shuffle tree, then waves in order)
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < kInfT * kInfT; t += NTH) {
    const int64_t c = static_cast<int64_t>(ty0 + t / kInfT) * w + tx0 + t % kInfT;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float v = ys[ch * kInfT * kInfT + t];
      y[ch * cells + c] = v;
      acc[ch] += static_cast<double>(v);
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc[ch] += __shfl_xor(acc[ch], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) red[wave][ch] = acc[ch];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t tile = static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      double s = 0.0;
      for (int wv = 0; wv < NW; ++wv) s += red[wv][ch];
      part[tile * 4 + ch] = s;
    }
    part[tile * 4 + 3] = 0.0;
  }
}

// ----------------------------------------------------------------------------
// dispatch on the padded channel counts
// ----------------------------------------------------------------------------
template <int CINP, int COUTP>
hipError_t fwd_launch(const float* x, int batch, int cin, int h, int w, const void* packed, int cout,
                      const float* bias, const float* mask, unsigned flags, float* y, hipStream_t s) {
  dim3 grid(w / kSeg, h, batch);
  hipLaunchKernelGGL((k_conv_fwd<CINP, COUTP>), grid, dim3(kThreads), 0, s, x, cin, h, w,
                     static_cast<const uint16_t*>(packed), cout, bias, mask, flags, y);
  return hipGetLastError();
}

template <int CINP, int COUTP>
hipError_t wgrad_launch(const float* x, const float* dy, int batch, int cin, int cout, int h, int w, float* dw,
                        float* db, void* scratch, hipStream_t s) {
  constexpr int KP = k_pad(CINP);
  dim3 grid(w / kSeg, (h + kWgradRows - 1) / kWgradRows, batch);
  const int64_t nblocks = static_cast<int64_t>(grid.x) * grid.y * grid.z;
  float* pw = static_cast<float*>(scratch);
  float* pb = pw + nblocks * COUTP * KP;
  hipLaunchKernelGGL((k_conv_wgrad<CINP, COUTP>), grid, dim3(kThreads), 0, s, x, dy, cin, cout, h, w, pw, pb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int total = cout * cin * 9 + cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((total + 255) / 256), dim3(256), 0, s, pw, pb, nblocks, cin, cout,
                     CINP, COUTP, KP, dw, db);
  return hipGetLastError();
}

// Supported padded shapes: CINP in {4, 8, 16, 32, 64}, COUTP in {16, 32, 48, 64}.
#define LBM_CONV_DISPATCH(FN, CINP_V, COUTP_V, ...)                                    \
  switch (CINP_V) {                                                                  \
    case 4: LBM_CONV_DISPATCH_OUT(FN, 4, COUTP_V, __VA_ARGS__); break;               \
    case 8: LBM_CONV_DISPATCH_OUT(FN, 8, COUTP_V, __VA_ARGS__); break;               \
    case 16: LBM_CONV_DISPATCH_OUT(FN, 16, COUTP_V, __VA_ARGS__); break;             \
    case 32: LBM_CONV_DISPATCH_OUT(FN, 32, COUTP_V, __VA_ARGS__); break;             \
    case 64: LBM_CONV_DISPATCH_OUT(FN, 64, COUTP_V, __VA_ARGS__); break;             \
    default: return hipErrorInvalidValue;                                            \
  }
#define LBM_CONV_DISPATCH_OUT(FN, CI, COUTP_V, ...)                 \
  switch (COUTP_V) {                                                \
    case 16: return FN<CI, 16>(__VA_ARGS__);                        \
    case 32: return FN<CI, 32>(__VA_ARGS__);                        \
    case 48: return FN<CI, 48>(__VA_ARGS__);                        \
    case 64: return FN<CI, 64>(__VA_ARGS__);                        \
    default: return hipErrorInvalidValue;                           \
  }

int pad_pow2_cin(int cin) {
  int c = 4;
  while (c < cin) c *= 2;
  return c;
}

hipError_t conv_forward(const float* x, int batch, int cin, int h, int w, const void* packed, int cout,
                        const float* bias, const float* mask, unsigned flags, float* y, hipStream_t s) {
  LBM_CONV_DISPATCH(fwd_launch, cin_pad(cin), cout_pad(cout), x, batch, cin, h, w, packed, cout, bias, mask,
                    flags, y, s)
}

hipError_t conv_wgrad(const float* x, const float* dy, int batch, int cin, int cout, int h, int w, float* dw,
                      float* db, void* scratch, hipStream_t s) {
  LBM_CONV_DISPATCH(wgrad_launch, cin_pad(cin), cout_pad(cout), x, dy, batch, cin, cout, h, w, dw, db, scratch,
                    s)
}

bool shape_ok(int cin, int cout) {
  const int cp = cin_pad(cin), op = cout_pad(cout);
  return cin >= 1 && cout >= 1 && cin <= 64 && cout <= 64 && (cp == 4 || cp == 8 || cp == 16 || cp == 32 || cp == 64) &&
         (op == 16 || op == 32 || op == 48 || op == 64);
}

lbm_status dev(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

}  // namespace

hipError_t net_infer_launch(const float* m, int h, int w, double rho_ref, float s_rho, float s_u,
                            const void* const* packed, const float* const* bias, float* y, double* part,
                            hipStream_t s) {
  NetWeights nw;
  for (int l = 0; l < 4; ++l) {
    nw.packed[l] = static_cast<const uint16_t*>(packed[l]);
    nw.bias[l] = bias[l];
  }
  constexpr int NW = kInferWaves, MP = kInferMP;
  hipLaunchKernelGGL((k_net_infer<NW, MP>), dim3(w / kInfT, h / kInfT), dim3(NW * 64), 0, s, m, h, w, rho_ref, s_rho,
                     s_u, nw, y, part);
  return hipGetLastError();
}

int64_t net_infer_tiles(int h, int w) {
  if (h < kInfT || w < kInfT || h % kInfT || w % kInfT) return 0;
  return static_cast<int64_t>(h / kInfT) * (w / kInfT);
}

namespace {

int red_blocks(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > kRedBlocks) b = kRedBlocks;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" {

size_t lbm_conv_packed_bytes(int32_t cin, int32_t cout) {
  if (cin < 1 || cout < 1 || cin > 64 || cout > 64) return 0;
  // either orientation fits: max of the forward and the transposed operand
  const size_t a = static_cast<size_t>(cout_pad(cout)) * k_pad(cin_pad(cin));
  const size_t b = static_cast<size_t>(cout_pad(cin)) * k_pad(cin_pad(cout));
  return 2 * (a > b ? a : b);
}

lbm_status lbm_conv_pack(const float* w, int32_t cin, int32_t cout, int32_t transpose, void* packed,
                         void* stream) {
  if (!w || !packed || cin < 1 || cout < 1 || cin > 64 || cout > 64) return LBM_EINVAL;
  const int ci_n = transpose ? cout : cin, co_n = transpose ? cin : cout;
  if (!shape_ok(ci_n, co_n)) return LBM_EINVAL;
  const int total = cout_pad(co_n) * k_pad(cin_pad(ci_n));
  hipLaunchKernelGGL(k_conv_pack, dim3((total + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), w,
                     cin, cout, transpose, static_cast<uint16_t*>(packed));
  return dev(hipGetLastError());
}

lbm_status lbm_conv_forward(const float* x, int32_t batch, int32_t cin, int32_t h, int32_t w, const void* packed,
                            int32_t cout, const float* bias, const float* mask, uint32_t flags, float* y,
                            void* stream) {
  if (!x || !packed || !y || batch < 1 || h < 1 || w < kSeg || w % kSeg != 0 || !shape_ok(cin, cout))
    return LBM_EINVAL;
  return dev(conv_forward(x, batch, cin, h, w, packed, cout, bias, mask, flags, y, static_cast<hipStream_t>(stream)));
}

size_t lbm_net_partials_bytes(int32_t h, int32_t w) {
  return static_cast<size_t>(net_infer_tiles(h, w)) * 4 * sizeof(double);
}

lbm_status lbm_net_infer(const float* moments, int32_t h, int32_t w, double rho_ref, float s_rho, float s_u,
                         const void* const* packed, const float* const* bias, float* y, double* partials,
                         void* stream) {
  if (!moments || !packed || !bias || !y || !partials || net_infer_tiles(h, w) == 0 || !(s_rho > 0) ||
      !(s_u > 0))
    return LBM_EINVAL;
  for (int l = 0; l < 4; ++l)
    if (!packed[l] || !bias[l]) return LBM_EINVAL;
  return dev(net_infer_launch(moments, h, w, rho_ref, s_rho, s_u, packed, bias, y, partials,
                              static_cast<hipStream_t>(stream)));
}

size_t lbm_conv_wgrad_scratch_bytes(int32_t batch, int32_t cin, int32_t cout, int32_t h, int32_t w) {
  if (batch < 1 || h < 1 || w < kSeg || w % kSeg != 0 || !shape_ok(cin, cout)) return 0;
  const int64_t nblocks = static_cast<int64_t>(w / kSeg) * ((h + kWgradRows - 1) / kWgradRows) * batch;
  const int cinp = cin_pad(cin), coutp = cout_pad(cout);
  return static_cast<size_t>(nblocks) * (static_cast<size_t>(coutp) * k_pad(cinp) + coutp) * sizeof(float);
}

lbm_status lbm_conv_wgrad(const float* x, const float* dy, int32_t batch, int32_t cin, int32_t cout, int32_t h,
                          int32_t w, float* dw, float* db, void* scratch, void* stream) {
  if (!x || !dy || !dw || !db || !scratch || lbm_conv_wgrad_scratch_bytes(batch, cin, cout, h, w) == 0)
    return LBM_EINVAL;
  return dev(conv_wgrad(x, dy, batch, cin, cout, h, w, dw, db, scratch, static_cast<hipStream_t>(stream)));
}

size_t lbm_reduce_scratch_bytes(int64_t n) {
  if (n < 1) return 0;
  return static_cast<size_t>(kRedBlocks) * 64 * sizeof(double);  // up to 64 channels of partials
}

lbm_status lbm_mse(const float* out, const float* target, int64_t n, float* grad, double* loss_dev, void* scratch,
                   void* stream) {
  if (!out || !target || !grad || !loss_dev || !scratch || n < 1) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = red_blocks(n);
  double* part = static_cast<double*>(scratch);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kThreads), 0, s, out, target, n, grad, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return LBM_EDEVICE;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kThreads), 0, s, part, nb, n, 0, loss_dev);
  return dev(hipGetLastError());
}

lbm_status lbm_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                    int32_t t, void* stream) {
  if (!p || !g || !m || !v || n < 1 || t < 1) return LBM_EINVAL;
  const float c1 = 1.0f - powf(b1, static_cast<float>(t));
  const float c2 = 1.0f - powf(b2, static_cast<float>(t));
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return dev(hipGetLastError());
}

lbm_status lbm_channel_rms(const float* x, int32_t channels, int64_t n, double* out_dev, void* scratch,
                           void* stream) {
  if (!x || !out_dev || !scratch || channels < 1 || channels > 64 || n < 1) return LBM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = red_blocks(n);
  double* part = static_cast<double*>(scratch);
  hipLaunchKernelGGL(k_sumsq, dim3(nb, channels), dim3(kThreads), 0, s, x, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return LBM_EDEVICE;
  hipLaunchKernelGGL(k_finish, dim3(channels), dim3(kThreads), 0, s, part, nb, n, 1, out_dev);
  return dev(hipGetLastError());
}

}  // extern "C"
