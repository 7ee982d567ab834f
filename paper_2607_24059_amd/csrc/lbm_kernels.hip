// Kernels of the single-run engine: initialisation, the fused
// relax-and-transport step, moments, FP64 diagnostics and the copy probe.
//
// Every kernel is templated on the dimension D and on the element types of
// the rest (TR) and moving (TM) planes; plain FP32 storage and the deviation
// storages run the same code (see lbm_device.hpp).
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

// ----------------------------------------------------------------------------
// init: every population at the equilibrium of W0 = (rho0, dx rho0 u0)
// ----------------------------------------------------------------------------
template <int D, typename TR, typename TM>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ u0,
                                              const double* __restrict__ rho0, double rho_ref,
                                              double dx, TR* __restrict__ rest,
                                              TM* __restrict__ move, int64_t cells,
                                              int64_t stride, CoefT<double> k) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  const double rho = rho0 ? rho0[c] : rho_ref;
  double W[D + 1];
  W[0] = rho - k.ref;  // deviation when k.ref = rho_ref, plain when 0
#pragma unroll
  for (int j = 0; j < D; ++j) W[1 + j] = dx * rho * u0[j * cells + c];
  if constexpr (StoresMoments<TM>::value) {  // the moments, no non-equilibrium part
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      store_real(rest + i * stride + c, W[i]);
      if constexpr (IsNeq<TM>::value) {
#pragma unroll
        for (int m = 0; m < 2 * D; ++m) store_f32(move + (i * 2 * D + m) * stride + c, 0.0f);
      }
    }
  } else {
    double eq[D + 1][2 * D + 1];
    equilibrium<D, double>(W, 1.0 / rho, k, eq);
#pragma unroll
    for (int i = 0; i < D + 1; ++i) {
      store_real(rest + i * stride + c, eq[i][0]);
#pragma unroll
      for (int m = 0; m < 2 * D; ++m) store_real(move + (i * 2 * D + m) * stride + c, eq[i][1 + m]);
    }
  }
}

// ----------------------------------------------------------------------------
// step: one thread per cell, pull transport fused with relaxation (step_cell)
// ----------------------------------------------------------------------------
template <int D, typename TR, typename TM>
__global__ __launch_bounds__(256) void k_step(const TR* __restrict__ sr,
                                              const TM* __restrict__ sm, TR* __restrict__ dr,
                                              TM* __restrict__ dm, int nx, int ny, int nz,
                                              int64_t stride, CoefT<typename ComputeOf<TM>::type> k,
                                              NeqScale<D> sc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  if constexpr (IsNeq<TM>::value)
    step_cell_neq<D>(sr, sm, dr, dm, x, y, z, nx, ny, nz, stride, k, sc);
  else if constexpr (IsMom<TM>::value)
    step_cell_mom<D>(sr, dr, x, y, z, nx, ny, nz, stride, k);
  else
    step_cell<D, TR, TM>(sr, sm, dr, dm, x, y, z, nx, ny, nz, stride, k);
}

// ----------------------------------------------------------------------------
// step with the channel boundaries (2D): the step of k_step, with the
// populations entering through the domain's sides replaced by their ghost
// values (wall_ghosts) before the relaxation
// ----------------------------------------------------------------------------
template <typename TR, typename TM>
__global__ __launch_bounds__(256) void k_step_walls(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                    TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                                    int64_t stride, CoefT<typename ComputeOf<TM>::type> k,
                                                    WallArgs w) {
  using R = typename ComputeOf<TM>::type;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t c = static_cast<int64_t>(y) * nx + x;
  R g[3][5];
  gather_cell<2, TR, TM, R>(sr, sm, x, y, 0, nx, ny, 1, stride, c, g);
  if (x == 0 || y == 0 || x == nx - 1 || y == ny - 1) wall_ghosts<TR, TM, R>(sr, sm, x, y, nx, ny, stride, k, w, g);
  collide<2, R>(g, k);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    store_stream(dr + i * stride + c, g[i][0]);
#pragma unroll
    for (int m = 0; m < 4; ++m) store_stream(dm + (i * 4 + m) * stride + c, g[i][1 + m]);
  }
}

// ----------------------------------------------------------------------------
// two steps in one launch (2D): the block advances its TX x TY tile plus a
// one-cell border by one step, keeps that intermediate state in LDS in the
// storage type (rounded exactly as a store to HBM would be), then advances the
// tile by the second step reading the border from LDS.  Each state value is
// read from HBM (TX+2)(TY+2)/(TX TY) times and written once per two steps, and
// the result is bit-identical to two single steps.
// ----------------------------------------------------------------------------
// The two-step tile in split storage.  Phase 1 advances the extended tile by
// one step from HBM (rebuilding the upwind neighbours' equilibria), rounds its
// non-equilibrium parts to the stored FP16 values, and keeps the populations
// they stand for, f* = f^eq(W) + n / s (rest: f^eq_rest(W) - sum_m n_m / s),
// in LDS as FP32: exactly the values the next step's gather would rebuild from
// HBM.  Phase 2 then gathers them like the plain kernel does, so the tile's
// second step needs no neighbour equilibria and the result equals two single
// steps bit for bit.
template <int TX, int TY, int NT>
__device__ __forceinline__ void step2_neq_tile(const float* __restrict__ sr, const neq16* __restrict__ sm,
                                               float* __restrict__ dr, neq16* __restrict__ dm, int nx, int ny,
                                               int64_t stride, const Coef& k, const NeqScale<2>& sc) {
  constexpr int EX = TX + 2, EY = TY + 2, EN = EX * EY;
  __shared__ float s_f[15][EN];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  for (int e = threadIdx.x; e < EN; e += NT) {
    const int ex = e % EX, ey = e / EX;
    int x = x0 - 1 + ex, y = y0 - 1 + ey;
    x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
    y = wrap_coord(y, ny);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
    int64_t src[4];
    upwind_sources<2>(x, y, 0, nx, ny, 1, c, src);
    auto w_at = [&](int i, int nb) { return sr[i * stride + (nb < 0 ? c : src[nb])]; };
    auto n_at = [&](int i, int m, int nb) { return load_f32(sm + (i * 4 + m) * stride + (nb < 0 ? c : src[nb])); };
    float g[3][5];
    gather_neq<2>(w_at, n_at, k, sc, g);
    float W[3], n[3][4], eq[3][5];
    collide_neq<2>(g, k, W, n, eq);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float nr[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) nr[m] = static_cast<float>(static_cast<_Float16>(n[i][m] * sc.s[i]));
      const float s = ((nr[0] + nr[1]) + nr[2]) + nr[3];
      s_f[i * 5][e] = (W[i] - ((i == 0) ? k.d2a_rho : k.d2a_q) * W[i]) - s * sc.inv[i];
#pragma unroll
      for (int m = 0; m < 4; ++m) s_f[i * 5 + 1 + m][e] = eq[i][1 + m] + nr[m] * sc.inv[i];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY; t += NT) {
    const int tx = t % TX, ty = t / TX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= nx || y >= ny) continue;
    const int e = (ty + 1) * EX + (tx + 1);
    float g[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[i][0] = s_f[i * 5][e];
      g[i][1] = s_f[i * 5 + 1][e - 1];   // +x from x-1
      g[i][2] = s_f[i * 5 + 2][e + 1];   // -x from x+1
      g[i][3] = s_f[i * 5 + 3][e - EX];  // +y from y-1
      g[i][4] = s_f[i * 5 + 4][e + EX];  // -y from y+1
    }
    float W[3], n[3][4], eq[3][5];
    collide_neq<2>(g, k, W, n, eq);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      store_stream(dr + i * stride + c, W[i]);
#pragma unroll
      for (int m = 0; m < 4; ++m) store_stream(dm + (i * 4 + m) * stride + c, n[i][m] * sc.s[i]);
    }
  }
}

// The two-step tile in moment-only storage: the intermediate moments of the
// extended tile (12 bytes per cell) in LDS.
template <int TX, int TY, int NT>
__device__ __forceinline__ void step2_mom_tile(const float* __restrict__ sr, float* __restrict__ dr, int nx, int ny,
                                               int64_t stride, const Coef& k) {
  constexpr int EX = TX + 2, EY = TY + 2, EN = EX * EY;
  __shared__ float s_w[3][EN];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  for (int e = threadIdx.x; e < EN; e += NT) {
    const int ex = e % EX, ey = e / EX;
    int x = x0 - 1 + ex, y = y0 - 1 + ey;
    x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
    y = wrap_coord(y, ny);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
    int64_t src[4];
    upwind_sources<2>(x, y, 0, nx, ny, 1, c, src);
    float out[3];
    step_moments<2>([&](int i, int nb) { return sr[i * stride + (nb < 0 ? c : src[nb])]; }, k, out);
#pragma unroll
    for (int i = 0; i < 3; ++i) s_w[i][e] = out[i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY; t += NT) {
    const int tx = t % TX, ty = t / TX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= nx || y >= ny) continue;
    const int e = (ty + 1) * EX + (tx + 1);
    const int off[4] = {-1, 1, -EX, EX};  // upwind neighbour of velocity +x, -x, +y, -y
    float out[3];
    step_moments<2>([&](int i, int nb) { return s_w[i][nb < 0 ? e : e + off[nb]]; }, k, out);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 3; ++i) store_stream(dr + i * stride + c, out[i]);
  }
}

// The two-step tile in the population storages: the intermediate state of the
// extended tile is kept in LDS in the storage types.
template <typename TR, typename TM, int TX, int TY, int NT>
__device__ __forceinline__ void step2_tile(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                           TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                           int64_t stride, const Coef& k) {
  constexpr int EX = TX + 2, EY = TY + 2, EN = EX * EY;
  __shared__ TR s_rest[3][EN];
  __shared__ TM s_move[12][EN];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  for (int e = threadIdx.x; e < EN; e += NT) {
    const int ex = e % EX, ey = e / EX;
    int x = x0 - 1 + ex, y = y0 - 1 + ey;
    x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
    y = wrap_coord(y, ny);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
    float g[3][5];
    gather_cell<2, TR, TM>(sr, sm, x, y, 0, nx, ny, 1, stride, c, g);
    collide<2>(g, k);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      store_f32(&s_rest[i][e], g[i][0]);
#pragma unroll
      for (int m = 0; m < 4; ++m) store_f32(&s_move[i * 4 + m][e], g[i][1 + m]);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY; t += NT) {
    const int tx = t % TX, ty = t / TX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= nx || y >= ny) continue;
    const int e = (ty + 1) * EX + (tx + 1);
    float g[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[i][0] = load_f32(&s_rest[i][e]);
      g[i][1] = load_f32(&s_move[i * 4 + 0][e - 1]);   // +x from x-1
      g[i][2] = load_f32(&s_move[i * 4 + 1][e + 1]);   // -x from x+1
      g[i][3] = load_f32(&s_move[i * 4 + 2][e - EX]);  // +y from y-1
      g[i][4] = load_f32(&s_move[i * 4 + 3][e + EX]);  // -y from y+1
    }
    collide<2>(g, k);
    const int64_t c = static_cast<int64_t>(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      store_stream(dr + i * stride + c, g[i][0]);
#pragma unroll
      for (int m = 0; m < 4; ++m) store_stream(dm + (i * 4 + m) * stride + c, g[i][1 + m]);
    }
  }
}

// ----------------------------------------------------------------------------
// two steps per launch in 3D, marching along z.  Each thread owns one (x, y)
// column of a (TX+2) x (TY+2) extended tile and walks the planes of one z
// segment [z0, z0 + ZS) plus one plane on each side.  At plane p it advances
// its column cell by the first step from HBM (the single-step gather); the
// in-plane moving populations (+-x, +-y of the four sets) of that result go to
// one of two LDS planes, the rest and +-z populations stay in the thread's
// registers.  The second step of plane p - 1 then gathers +-x, +-y from the
// neighbouring columns' LDS values of plane p - 1, the rest from its own
// registers, +z from its result of plane p - 2 and -z from that of plane p,
// and writes the tile's cells to HBM.  One barrier per plane.  Every first-step
// value is rounded to the storage type as a store to HBM would round it, so the
// result equals two single steps bit for bit; each state value is read about
// (TX+2)(TY+2)(ZS+2)/(TX TY ZS) times and written once per two steps.
// Columns are wave-aligned: wave r < TY+2 owns the 64 columns x0 .. x0+63 of
// extended row r, so its loads and stores cover whole 128-byte lines (a store
// that covers part of a line costs a partial-line write to HBM), and the last
// wave owns the 2 (TY+2) border columns x0-1 and x0+64.
// ----------------------------------------------------------------------------
template <typename TR, typename TM, int TX, int TY, int ZS, int NT>
__global__ __launch_bounds__(NT) void k_step2_3d(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                  TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny, int nz,
                                                  int64_t stride, Coef k) {
  constexpr int EX = TX + 2, EY = TY + 2, EN = EX * EY;
  static_assert(TX == 64 && NT == 64 * (EY + 1) && 2 * EY <= 64, "one wave per row plus one for the border");
  __shared__ TM s_in[2][16][EN];  // +-x, +-y populations of the four sets, two planes
  const int t = threadIdx.x;
  int ex, ey;
  bool col;
  if (t < 64 * EY) {
    ey = t / 64;
    ex = 1 + t % 64;
    col = true;
  } else {
    const int j = t - 64 * EY;
    ey = j / 2;
    ex = (j % 2) ? EX - 1 : 0;
    col = j < 2 * EY;
  }
  const int e = ey * EX + ex;  // the column's LDS slot (used only where col holds)
  // one-dimensional grid in XCD-major order: XCD j (block b runs on XCD b mod
  // 8) takes the j-th eighth of the tiles in raster order (x, then y, then
  // z), so the tiles that run together on one XCD are neighbours and share
  // their border lines through its L2 (38.5 against 37.4 GLUPS at 256^3)
  const int tx_n = (nx + TX - 1) / TX, ty_n = (ny + TY - 1) / TY;
  const int nt = tx_n * ty_n * ((nz + ZS - 1) / ZS);
  const int b = blockIdx.x;
  const int tt = static_cast<int>(xcd_major(b, nt));
  const int x0 = (tt % tx_n) * TX, y0 = ((tt / tx_n) % ty_n) * TY, z0 = (tt / (tx_n * ty_n)) * ZS;
  int x = x0 - 1 + ex, y = y0 - 1 + ey;
  x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
  y = wrap_coord(y, ny);
  const bool inner = col && ex >= 1 && ex <= TX && ey >= 1 && ey <= TY && x0 + ex - 1 < nx && y0 + ey - 1 < ny;
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const int64_t cxy = static_cast<int64_t>(y) * nx + x;
  const int zend = min(z0 + ZS, nz);
  float rest1[4], zp1[4], zp2[4];  // first-step results of planes p - 1 (rest, +z) and p - 2 (+z)
#pragma unroll
  for (int i = 0; i < 4; ++i) rest1[i] = zp1[i] = zp2[i] = 0.0f;
  for (int p = z0 - 1; p <= zend; ++p) {
    const int slot = (p - z0 + 1) & 1;
    float rest0[4], zp0[4], zm0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) rest0[i] = zp0[i] = zm0[i] = 0.0f;
    if (col) {
      const int pz = ((p % nz) + nz) % nz;
      const int64_t c = static_cast<int64_t>(pz) * plane + cxy;
      float g[4][7];
      gather_cell<3, TR, TM>(sr, sm, x, y, pz, nx, ny, nz, stride, c, g);
      collide<3>(g, k);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        TR r;
        TM a, b;
        store_f32(&r, g[i][0]);
        store_f32(&a, g[i][5]);
        store_f32(&b, g[i][6]);
        rest0[i] = load_f32(&r);
        zp0[i] = load_f32(&a);
        zm0[i] = load_f32(&b);
#pragma unroll
        for (int m = 0; m < 4; ++m) store_f32(&s_in[slot][i * 4 + m][e], g[i][1 + m]);
      }
    }
    if (p >= z0 + 1 && inner) {
      // second step of plane p - 1
      float g[4][7];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        g[i][0] = rest1[i];
        g[i][1] = load_f32(&s_in[slot ^ 1][i * 4 + 0][e - 1]);   // +x from x-1
        g[i][2] = load_f32(&s_in[slot ^ 1][i * 4 + 1][e + 1]);   // -x from x+1
        g[i][3] = load_f32(&s_in[slot ^ 1][i * 4 + 2][e - EX]);  // +y from y-1
        g[i][4] = load_f32(&s_in[slot ^ 1][i * 4 + 3][e + EX]);  // -y from y+1
        g[i][5] = zp2[i];                                        // +z from z-1
        g[i][6] = zm0[i];                                        // -z from z+1
      }
      collide<3>(g, k);
      const int64_t c = static_cast<int64_t>(p - 1) * plane + static_cast<int64_t>(y0 + ey - 1) * nx + (x0 + ex - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        store_stream(dr + i * stride + c, g[i][0]);
#pragma unroll
        for (int m = 0; m < 6; ++m) store_stream(dm + (i * 6 + m) * stride + c, g[i][1 + m]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      zp2[i] = zp1[i];
      zp1[i] = zp0[i];
      rest1[i] = rest0[i];
    }
    __syncthreads();
  }
}

// Pull gather of a 3D cell for the z-marching kernels: the rest populations
// at in-plane index c of plane offset zc, the in-plane moving ones from the
// upwind indices nb (x - 1, x + 1, y - 1, y + 1, wrapped), +z from the plane
// below (offset zm) and -z from the plane above (zp).  Plane offsets are
// common to the block and element indices are 32-bit, so a load is a block
// base plus a lane offset (planes of at most 2^30 cells); the loaded
// elements are those of gather_cell.
template <typename TR, typename TM>
__device__ __forceinline__ void gather_cell3_o32(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                 int64_t stride, int64_t zc, int64_t zm, int64_t zp, uint32_t c,
                                                 const uint32_t (&nb)[4], float (&g)[4][7]) {
  constexpr uint32_t BR = sizeof(TR), BM = sizeof(TM);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    g[i][0] = load_f32(at_byte(sr + i * stride + zc, c * BR));
#pragma unroll
    for (int m = 0; m < 4; ++m) g[i][1 + m] = load_f32(at_byte(sm + (i * 6 + m) * stride + zc, nb[m] * BM));
    g[i][5] = load_f32(at_byte(sm + (i * 6 + 4) * stride + zm, c * BM));
    g[i][6] = load_f32(at_byte(sm + (i * 6 + 5) * stride + zp, c * BM));
  }
}

// ----------------------------------------------------------------------------
// three steps per launch in 3D (4-byte planes), marching along z.  The tile
// is TX x TY columns; stage 1 runs over the tile plus a two-cell x/y border
// (EX x EY columns), stage 2 over the tile plus a one-cell border, stage 3
// over the tile.  At plane p the block advances plane p by stage 1 (from
// HBM), plane p - 1 by stage 2 and plane p - 2 by stage 3 (to HBM).  Each
// thread owns one column of the EX x EY region in all three stages: a stage's
// rest and +-z populations stay in the owner's registers (the +-z neighbours
// of the next stage are the owner's results of the planes below and above),
// and its 16 in-plane moving populations go to LDS, each into the slot of the
// neighbouring column that pulls it in the next stage (so the LDS holds one
// set per column of the next stage's region, 66 x (TY + 2) and TX x TY,
// double-buffered by plane parity: one barrier per plane).  Every
// stage stores its results as the storage type rounds them and relaxes with
// the same collide as the single step, so the result equals three single
// steps bit for bit.  Waves r < EY own the 64 columns x0 .. x0 + 63 of
// extended row r (whole 128-byte lines per access); the last wave owns the
// four border columns x0 - 2, x0 - 1, x0 + 64, x0 + 65 of every row.  A block
// walks zs planes (chosen per grid by zseg_for).
// ----------------------------------------------------------------------------
template <typename TR, typename TM, int TY>
__global__ __launch_bounds__(64 * (TY + 5)) void k_step3_3d(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                            TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                                            int nz, int zs, int64_t stride, Coef k) {
  constexpr int TX = 64, H = 2, EX = TX + 2 * H, EY = TY + 2 * H;
  constexpr int RX2 = TX + 2, RY2 = TY + 2, EN2 = RX2 * RY2;  // stage-2 region
  static_assert(4 * EY <= 64, "border columns of every row fit one wave");
  // a stage's moving populations wait in LDS in the slot of the next stage's
  // column that pulls them, by plane parity: 16 values per column of the
  // next stage's region, not of the writer's
  __shared__ TM s1[2][16][EN2];      // stage-1 results, in stage-2 slots
  __shared__ TM s2[2][16][TX * TY];  // stage-2 results, in stage-3 (tile) slots
  const int t = threadIdx.x;
  int ex, ey;
  bool col;
  if (t < 64 * EY) {
    ey = t / 64;
    ex = H + t % 64;
    col = true;
  } else {
    const int j = t - 64 * EY;
    ey = j / 4;
    const int c = j % 4;
    ex = c < 2 ? c : TX + c;  // 0, 1, EX - 2, EX - 1
    col = j < 4 * EY;
    if (!col) ey = 0;
  }
  const bool in2 = col && ex >= 1 && ex < EX - 1 && ey >= 1 && ey < EY - 1;
  const bool in3 = col && ex >= H && ex < H + TX && ey >= H && ey < H + TY;
  // own slots in the stage-2 and stage-3 regions, and the slots that the
  // four moving populations go to: +x to column (ex + 1, ey), -x to
  // (ex - 1, ey), +y to (ex, ey + 1), -y to (ex, ey - 1); -1 where that
  // column is outside the next stage's region
  const int e2 = in2 ? (ey - 1) * RX2 + (ex - 1) : 0;
  const int e3 = in3 ? (ey - H) * TX + (ex - H) : 0;
  int w1[4], w2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int tx = ex + (m == 0 ? 1 : m == 1 ? -1 : 0), ty = ey + (m == 2 ? 1 : m == 3 ? -1 : 0);
    w1[m] = (col && tx >= 1 && tx < EX - 1 && ty >= 1 && ty < EY - 1) ? (ty - 1) * RX2 + (tx - 1) : -1;
    w2[m] = (in2 && tx >= H && tx < H + TX && ty >= H && ty < H + TY) ? (ty - H) * TX + (tx - H) : -1;
  }
  const int tx_n = (nx + TX - 1) / TX, ty_n = (ny + TY - 1) / TY;
  const int nt = tx_n * ty_n * ((nz + zs - 1) / zs);
  const int b = blockIdx.x;
  const int tt = static_cast<int>(xcd_major(b, nt));
  const int x0 = (tt % tx_n) * TX, y0 = ((tt / tx_n) % ty_n) * TY, z0 = (tt / (tx_n * ty_n)) * zs;
  int x = x0 - H + ex, y = y0 - H + ey;
  x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
  y = wrap_coord(y, ny);
  const bool out = in3 && x0 + ex - H < nx && y0 + ey - H < ny;
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  // the column's in-plane index and its four in-plane upwind indices
  const uint32_t c32 = static_cast<uint32_t>(y) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x);
  const uint32_t row = static_cast<uint32_t>(nx), last = static_cast<uint32_t>(ny - 1) * row;
  uint32_t nb[4];
  nb[0] = (x == 0) ? c32 + (row - 1) : c32 - 1;       // +x from x - 1
  nb[1] = (x == nx - 1) ? c32 - (row - 1) : c32 + 1;  // -x from x + 1
  nb[2] = (y == 0) ? c32 + last : c32 - row;          // +y from y - 1
  nb[3] = (y == ny - 1) ? c32 - last : c32 + row;     // -y from y + 1
  // gather of wrapped plane pz (its neighbours wrap too)
  auto gather = [&](int pz, float (&gg)[4][7]) {
    const int zb = (pz == 0) ? nz - 1 : pz - 1, za = (pz == nz - 1) ? 0 : pz + 1;
    gather_cell3_o32<TR, TM>(sr, sm, stride, pz * plane, zb * plane, za * plane, c32, nb, gg);
  };
  const int zend = min(z0 + zs, nz);
  // stage histories: rest and +z of the previous plane, +z of the one before
  float r1p[4], z1p[4], z1pp[4], r2p[4], z2p[4], z2pp[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) r1p[i] = z1p[i] = z1pp[i] = r2p[i] = z2p[i] = z2pp[i] = 0.0f;
  // the stage-1 gather of the next plane is issued before the current plane's
  // work (45.6 against 45.0 GLUPS at 256^3); loads stay in flight across the
  // barrier, which waits on LDS only
  float gn[4][7];
  int pzn = wrap_coord(z0 - 2, nz);  // wrapped index of the next plane to gather
  if (col) gather(pzn, gn);
  pzn = (pzn + 1 == nz) ? 0 : pzn + 1;
  for (int p = z0 - 2; p <= zend + 1; ++p) {
    const int sl = p & 1;
    float g[4][7];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int l = 0; l < 7; ++l) g[i][l] = gn[i][l];
    if (col && p + 1 <= zend + 1) gather(pzn, gn);
    pzn = (pzn + 1 == nz) ? 0 : pzn + 1;
    // stage 1, plane p, from HBM
    float r1[4], zp1[4], zm1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) r1[i] = zp1[i] = zm1[i] = 0.0f;
    if (col) {
      collide<3>(g, k);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        TR a;
        TM bp, bm;
        store_f32(&a, g[i][0]);
        store_f32(&bp, g[i][5]);
        store_f32(&bm, g[i][6]);
        r1[i] = load_f32(&a);
        zp1[i] = load_f32(&bp);
        zm1[i] = load_f32(&bm);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (w1[m] >= 0)
#pragma unroll
          for (int i = 0; i < 4; ++i) store_f32(&s1[sl][i * 4 + m][w1[m]], g[i][1 + m]);
    }
    // stage 2, plane p - 1, from the stage-1 results
    float zm2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) zm2[i] = 0.0f;
    if (p >= z0 && in2) {
      float g[4][7];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        g[i][0] = r1p[i];
        g[i][1] = load_f32(&s1[sl ^ 1][i * 4 + 0][e2]);  // +x from x-1
        g[i][2] = load_f32(&s1[sl ^ 1][i * 4 + 1][e2]);  // -x from x+1
        g[i][3] = load_f32(&s1[sl ^ 1][i * 4 + 2][e2]);  // +y from y-1
        g[i][4] = load_f32(&s1[sl ^ 1][i * 4 + 3][e2]);  // -y from y+1
        g[i][5] = z1pp[i];                               // +z from z-1
        g[i][6] = zm1[i];                                // -z from z+1
      }
      collide<3>(g, k);
      float r2[4], zp2[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        TR a;
        TM bp, bm;
        store_f32(&a, g[i][0]);
        store_f32(&bp, g[i][5]);
        store_f32(&bm, g[i][6]);
        r2[i] = load_f32(&a);
        zp2[i] = load_f32(&bp);
        zm2[i] = load_f32(&bm);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (w2[m] >= 0)
#pragma unroll
          for (int i = 0; i < 4; ++i) store_f32(&s2[sl ^ 1][i * 4 + m][w2[m]], g[i][1 + m]);
      // stage 3, plane p - 2, from the stage-2 results, to HBM
      if (p >= z0 + 2 && out) {
        float h[4][7];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          h[i][0] = r2p[i];
          h[i][1] = load_f32(&s2[sl][i * 4 + 0][e3]);
          h[i][2] = load_f32(&s2[sl][i * 4 + 1][e3]);
          h[i][3] = load_f32(&s2[sl][i * 4 + 2][e3]);
          h[i][4] = load_f32(&s2[sl][i * 4 + 3][e3]);
          h[i][5] = z2pp[i];
          h[i][6] = zm2[i];
        }
        collide<3>(h, k);
        const int64_t zc = static_cast<int64_t>(p - 2) * plane;  // an output column does not wrap: c32 is its index
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          store_stream(at_byte(dr + i * stride + zc, c32 * static_cast<uint32_t>(sizeof(TR))), h[i][0]);
#pragma unroll
          for (int m = 0; m < 6; ++m)
            store_stream(at_byte(dm + (i * 6 + m) * stride + zc, c32 * static_cast<uint32_t>(sizeof(TM))), h[i][1 + m]);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z2pp[i] = z2p[i];
        z2p[i] = zp2[i];
        r2p[i] = r2[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z1pp[i] = z1p[i];
      z1p[i] = zp1[i];
      r1p[i] = r1[i];
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// one step of the 3D moment-only storage, marching along z.  A block owns a
// TX x TY column tile and a z segment; each thread keeps its column's W at
// planes z - 1, z and z + 1 in registers (the +-z neighbours of the stencil),
// and plane z of the tile plus a one-cell x/y halo goes to LDS for the
// in-plane neighbours (double-buffered: one barrier per plane).  Each plane
// of W is read once by the tile (plus the halo, mostly from L2) instead of
// by seven stencil points, and the stencil evaluates step_moments exactly as
// the cell-parallel kernel does, so the result is the same bit for bit.  The
// loads of plane z + 2 are issued before plane z is evaluated.
// Bound to 64 VGPRs (8 waves per SIMD) so that two 1024-thread blocks share
// a compute unit (one block per unit ran 110 against 134 GLUPS); plane bases
// common to the block with 32-bit lane offsets keep it at 58 without spills.
// ----------------------------------------------------------------------------
template <int TX, int TY, int ZS>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_step_mom_3d(
    const float* __restrict__ sr, float* __restrict__ dr, int nx, int ny, int nz, int64_t stride, Coef k) {
  constexpr int NT = TX * TY, EX = TX + 2, EY = TY + 2, EN = EX * EY;
  constexpr int NH = 2 * EX + 2 * TY;  // halo cells of a plane: two rows of EX, two columns of TY
  static_assert(NH <= NT, "one halo cell per thread at most");
  __shared__ float s_w[2][4][EN];
  const int t = static_cast<int>(threadIdx.x);
  // tile order: XCD-major over (x, y, z-segment) in raster order
  const int tx_n = (nx + TX - 1) / TX, ty_n = (ny + TY - 1) / TY;
  const int nt = tx_n * ty_n * ((nz + ZS - 1) / ZS);
  const int b = blockIdx.x;
  const int tt = static_cast<int>(xcd_major(b, nt));
  const int x0 = (tt % tx_n) * TX, y0 = ((tt / tx_n) % ty_n) * TY, z0 = (tt / (tx_n * ty_n)) * ZS;
  const int zend = min(z0 + ZS, nz);
  const int ox = t % TX, oy = t / TX;
  const int x = x0 + ox, y = y0 + oy;
  const bool own = x < nx && y < ny;
  const int e_own = (oy + 1) * EX + (ox + 1);
  // the thread's own column (wrapped, so that ragged tiles load valid cells),
  // as a 32-bit byte offset within a plane: addresses are a plane base common
  // to the block plus that offset (planes of at most 2^30 cells)
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const uint32_t o_own = (static_cast<uint32_t>(wrap_coord(y, ny)) * static_cast<uint32_t>(nx) +
                          static_cast<uint32_t>(wrap_coord(x, nx))) * 4u;
  // the thread's halo cell: rows y0 - 1 and y0 + TY (EX cells each, corners
  // included), then columns x0 - 1 and x0 + TX of the TY inner rows
  int e_h = -1;
  uint32_t o_h = 0;
  if (t < NH) {
    int hx, hy;
    if (t < 2 * EX) {
      hx = t % EX;
      hy = (t < EX) ? 0 : EY - 1;
    } else {
      const int u = t - 2 * EX;
      hx = (u % 2) ? EX - 1 : 0;
      hy = 1 + u / 2;
    }
    e_h = hy * EX + hx;
    o_h = (static_cast<uint32_t>(wrap_coord(y0 - 1 + hy, ny)) * static_cast<uint32_t>(nx) +
           static_cast<uint32_t>(wrap_coord(x0 - 1 + hx, nx))) * 4u;
  }
  // component i of plane z (periodic in z)
  auto pl = [&](int i, int z) { return sr + i * stride + static_cast<int64_t>(wrap_coord(z, nz)) * plane; };
  float wm[4], w0[4], wp[4], wn[4], h0[4], h1[4], hn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    wm[i] = *at_byte(pl(i, z0 - 1), o_own);
    w0[i] = *at_byte(pl(i, z0), o_own);
    wp[i] = *at_byte(pl(i, z0 + 1), o_own);
    h0[i] = (e_h >= 0) ? *at_byte(pl(i, z0), o_h) : 0.0f;
    h1[i] = (e_h >= 0) ? *at_byte(pl(i, z0 + 1), o_h) : 0.0f;
  }
  int buf = 0;
  // plane z + 2 wrapped into [0, nz), advanced by one per plane
  int zw2 = wrap_coord(z0 + 2, nz);
  for (int z = z0; z < zend; ++z) {
    // issue the loads of plane z + 2 (own column and halo cell) before this
    // plane's stencil: the halo rows are then read at the same time as the
    // neighbouring tiles read them as their own (141.6 against 139.2 GLUPS)
    const float* p2 = sr + static_cast<int64_t>(zw2) * plane;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      wn[i] = *at_byte(p2 + i * stride, o_own);
      hn[i] = (e_h >= 0) ? *at_byte(p2 + i * stride, o_h) : 0.0f;
    }
    zw2 = (zw2 + 1 == nz) ? 0 : zw2 + 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s_w[buf][i][e_own] = w0[i];
      if (e_h >= 0) s_w[buf][i][e_h] = h0[i];
    }
    __syncthreads();
    if (own) {
      const int off[4] = {-1, 1, -EX, EX};  // upwind neighbour of velocity +x, -x, +y, -y
      float out[4];
      step_moments<3>(
          [&](int i, int nb) {
            return nb < 0 ? w0[i] : nb == 4 ? wm[i] : nb == 5 ? wp[i] : s_w[buf][i][e_own + off[nb]];
          },
          k, out);
      const uint32_t o = (static_cast<uint32_t>(y) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x)) * 4u;
#pragma unroll
      for (int i = 0; i < 4; ++i) store_stream(at_byte(dr + i * stride + static_cast<int64_t>(z) * plane, o), out[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      wm[i] = w0[i];
      w0[i] = wp[i];
      wp[i] = wn[i];
      h0[i] = h1[i];
      h1[i] = hn[i];
    }
    buf ^= 1;
  }
}

// ----------------------------------------------------------------------------
// two steps of the 3D moment-only storage per launch, marching along z.  A
// block owns a 64 x TY column tile and a segment of zs planes.  Stage 1
// advances the tile plus a one-cell x/y border (66 x (TY + 2) columns) by one
// step from the stored W of the tile plus a two-cell border (68 x (TY + 4));
// stage 2 advances the tile from the stage-1 results, which stay on the chip.
// At plane p the block evaluates stage 1 at plane p and stage 2 at plane
// p - 1.  Each thread owns one column of the 68 x (TY + 4) region (waves
// r < TY + 4 the 64 inner columns of row r, the last wave the four border
// columns of every row, as in k_step3_3d) and keeps the column's stored W at
// planes p - 1, p, p + 1 and its stage-1 W at planes p - 2, p - 1, p in
// registers: the +-z neighbours of both stages.  The in-plane neighbours of a
// stage come from an LDS plane of that stage's input, double-buffered by
// plane parity, so a plane costs one barrier.  Each cell's 1 / rho is
// computed once per plane by its owner and kept beside its W (in LDS and in
// the column's registers) instead of once by each of its six neighbours
// (GLUPS at 256^3: 174.1 -> 184.8, 128^3: 116 -> 133).  Both stages evaluate
// the single step's stencil (step_moments_inv, with that same reciprocal), so
// the result equals two single steps bit for bit.  Loads and stores use a plane base common to the
// block plus the column's 32-bit byte offset (planes of at most 2^30 cells).
// ----------------------------------------------------------------------------
template <int TY>
__global__ __launch_bounds__(64 * (TY + 5)) void k_step2_mom_3d(const float* __restrict__ sr, float* __restrict__ dr,
                                                                int nx, int ny, int nz, int zs, int64_t stride,
                                                                Coef k) {
  constexpr int TX = 64, H = 2, EX = TX + 2 * H, EY = TY + 2 * H, E0 = EX * EY;
  constexpr int RX1 = TX + 2, RY1 = TY + 2, E1 = RX1 * RY1;
  static_assert(4 * EY <= 64, "border columns of every row fit one wave");
  __shared__ float s0[2][5][E0];  // stored W of plane p and its 1 / rho, over the 68 x (TY + 4) region
  __shared__ float s1[2][5][E1];  // stage-1 W of plane p and its 1 / rho, over the 66 x (TY + 2) region
  const int t = threadIdx.x;
  int ex, ey;
  bool col;
  if (t < 64 * EY) {
    ey = t / 64;
    ex = H + t % 64;
    col = true;
  } else {
    const int j = t - 64 * EY;
    ey = j / 4;
    const int c = j % 4;
    ex = c < 2 ? c : TX + c;  // 0, 1, EX - 2, EX - 1
    col = j < 4 * EY;
    if (!col) ey = 0;
  }
  const bool in1 = col && ex >= 1 && ex < EX - 1 && ey >= 1 && ey < EY - 1;
  const bool in2 = col && ex >= H && ex < H + TX && ey >= H && ey < H + TY;
  const int e0 = ey * EX + ex;
  const int e1 = in1 ? (ey - 1) * RX1 + (ex - 1) : 0;
  const int tx_n = (nx + TX - 1) / TX, ty_n = (ny + TY - 1) / TY;
  const int nt = tx_n * ty_n * ((nz + zs - 1) / zs);
  const int tt = static_cast<int>(xcd_major(blockIdx.x, nt));
  const int x0 = (tt % tx_n) * TX, y0 = ((tt / tx_n) % ty_n) * TY, z0 = (tt / (tx_n * ty_n)) * zs;
  const int x = wrap_coord(x0 - H + ex, nx), y = wrap_coord(y0 - H + ey, ny);  // may wrap several times
  const bool out = in2 && x0 + ex - H < nx && y0 + ey - H < ny;
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const uint32_t o = (static_cast<uint32_t>(y) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x)) * 4u;
  const int zend = min(z0 + zs, nz);
  // the column's stored W at wrapped plane q
  auto load = [&](int q, float (&w)[4]) {
    const float* base = sr + static_cast<int64_t>(q) * plane;
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = *at_byte(base + i * stride, o);
  };
  // stored W at planes p - 1, p, p + 1 and p + 2 (in flight); stage-1 W at p - 2, p - 1
  float a0[4], b0[4], c0[4], n0[4], a1[4], b1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) a0[i] = b0[i] = c0[i] = n0[i] = a1[i] = b1[i] = 0.0f;
  // 1 / rho of the column at those planes, computed once per cell and plane
  auto rinv = [&](const float (&w)[4]) { return recip_neq(w[0] + k.ref); };
  float ia0 = 0.0f, ib0 = 0.0f, ic0 = 0.0f, ia1 = 0.0f, ib1 = 0.0f;
  int q = wrap_coord(z0 - 2, nz);
  if (col) load(q, a0);
  q = (q + 1 == nz) ? 0 : q + 1;
  if (col) load(q, b0);
  q = (q + 1 == nz) ? 0 : q + 1;
  if (col) load(q, c0);
  q = (q + 1 == nz) ? 0 : q + 1;  // wrapped z0 + 1: the first plane issued ahead
  ia0 = rinv(a0);
  ib0 = rinv(b0);
  for (int p = z0 - 1; p <= zend; ++p) {
    const int sl = p & 1;
    // plane p + 2, consumed from the next plane on; in flight across the barrier
    if (col && p < zend) load(q, n0);
    q = (q + 1 == nz) ? 0 : q + 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) s0[sl][i][e0] = b0[i];
    s0[sl][4][e0] = ib0;
    ic0 = rinv(c0);
    __syncthreads();
    // stage 1 at plane p
    float c1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float ic1 = 0.0f;
    if (in1) {
      const int off[4] = {-1, 1, -EX, EX};  // upwind neighbour of velocity +x, -x, +y, -y
      step_moments_inv<3>(
          [&](int i, int nb) {
            return nb < 0 ? b0[i] : nb == 4 ? a0[i] : nb == 5 ? c0[i] : s0[sl][i][e0 + off[nb]];
          },
          [&](int nb) { return nb == 4 ? ia0 : nb == 5 ? ic0 : s0[sl][4][e0 + off[nb]]; }, k, c1);
      ic1 = rinv(c1);
#pragma unroll
      for (int i = 0; i < 4; ++i) s1[sl][i][e1] = c1[i];
      s1[sl][4][e1] = ic1;
    }
    // stage 2 at plane p - 1, to HBM
    if (out && p > z0) {
      const int off[4] = {-1, 1, -RX1, RX1};
      float w2[4];
      step_moments_inv<3>(
          [&](int i, int nb) {
            return nb < 0 ? b1[i] : nb == 4 ? a1[i] : nb == 5 ? c1[i] : s1[sl ^ 1][i][e1 + off[nb]];
          },
          [&](int nb) { return nb == 4 ? ia1 : nb == 5 ? ic1 : s1[sl ^ 1][4][e1 + off[nb]]; }, k, w2);
      const int64_t zc = static_cast<int64_t>(p - 1) * plane;  // an output column does not wrap
#pragma unroll
      for (int i = 0; i < 4; ++i) store_stream(at_byte(dr + i * stride + zc, o), w2[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a0[i] = b0[i];
      b0[i] = c0[i];
      c0[i] = n0[i];
      a1[i] = b1[i];
      b1[i] = c1[i];
    }
    ia0 = ib0;
    ib0 = ic0;
    ia1 = ib1;
    ib1 = ic1;
  }
}

// K >= 3 steps per launch: the tiles of lbm_fused.hpp
template <typename TR, typename TM, int TX, int TY, int NT, int K, bool XCD = false>
__global__ __launch_bounds__(NT) void k_stepK_2d(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                  TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                                  int64_t stride, Coef k) {
  using T = TileK<TR, TM, TX, TY, NT, K>;
  __shared__ TR s_rest[3][T::EN];
  __shared__ TM s_move[12][T::EN];
  int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  if constexpr (XCD) xcd_tile_origin(blockIdx.x, nx, ny, TX, TY, &x0, &y0);
  T::run(sr, sm, dr, dm, x0, y0, nx, ny, stride, k, s_rest, s_move);
}

template <typename TR, typename TM, int TX, int TY, int NT, int K, bool XCD = false>
__global__ __launch_bounds__(NT) void k_stepKr_2d(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                   TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                                   int64_t stride, Coef k) {
  using T = TileKr<TR, TM, TX, TY, NT, K>;
  __shared__ TM s_move[12][T::EN];
  int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  if constexpr (XCD) xcd_tile_origin(blockIdx.x, nx, ny, TX, TY, &x0, &y0);
  T::run(sr, sm, dr, dm, x0, y0, nx, ny, stride, k, s_move);
}

template <int TX, int TY, int NT, int K, bool XCD = false>
__global__ __launch_bounds__(NT) void k_stepK_neq_2d(const float* __restrict__ sr, const neq16* __restrict__ sm,
                                                      float* __restrict__ dr, neq16* __restrict__ dm, int nx, int ny,
                                                      int64_t stride, Coef k, NeqScale<2> sc) {
  using T = TileNeqK<TX, TY, NT, K>;
  __shared__ float s_f[15][T::EN];
  int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  if constexpr (XCD) xcd_tile_origin(blockIdx.x, nx, ny, TX, TY, &x0, &y0);
  T::run(sr, sm, dr, dm, x0, y0, nx, ny, stride, k, sc, s_f);
}

template <int TX, int TY, int NT, int K, bool XCD = false>
__global__ __launch_bounds__(NT) void k_stepK_mom_2d(const float* __restrict__ sr, float* __restrict__ dr, int nx,
                                                      int ny, int64_t stride, Coef k) {
  using T = TileMomK<TX, TY, NT, K>;
  __shared__ float s_w[3][T::EN];
  int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  if constexpr (XCD) xcd_tile_origin(blockIdx.x, nx, ny, TX, TY, &x0, &y0);
  T::run(sr, dr, x0, y0, nx, ny, stride, k, s_w);
}

template <typename TR, typename TM, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_step2_2d(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                                  TR* __restrict__ dr, TM* __restrict__ dm, int nx, int ny,
                                                  int64_t stride, Coef k, NeqScale<2> sc) {
  if constexpr (IsNeq<TM>::value)
    step2_neq_tile<TX, TY, NT>(sr, sm, dr, dm, nx, ny, stride, k, sc);
  else if constexpr (IsMom<TM>::value)
    step2_mom_tile<TX, TY, NT>(sr, dr, nx, ny, stride, k);
  else
    step2_tile<TR, TM, TX, TY, NT>(sr, sm, dr, dm, nx, ny, stride, k);
}

// ----------------------------------------------------------------------------
// moments: rho = ref + sum_l g_rho,l and q_j = (sum_l g_qj,l) / dx, in FP64
// ----------------------------------------------------------------------------
template <int D, typename TR, typename TM>
__device__ __forceinline__ void cell_sums(const TR* __restrict__ r, const TM* __restrict__ m,
                                          int64_t c, int64_t stride, double (&s)[D + 1]) {
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    double a = load_f64(r + i * stride + c);
    if constexpr (!StoresMoments<TM>::value) {  // these storages keep the moments themselves
#pragma unroll
      for (int v = 0; v < 2 * D; ++v) a += load_f64(m + (i * 2 * D + v) * stride + c);
    }
    s[i] = a;
  }
}

template <int D, typename TR, typename TM>
__global__ __launch_bounds__(256) void k_moments(const TR* __restrict__ r, const TM* __restrict__ m,
                                                 int64_t cells, int64_t stride, double ref, double dx,
                                                 double* __restrict__ out64,
                                                 float* __restrict__ out32) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cells) return;
  double s[D + 1];
  cell_sums<D>(r, m, c, stride, s);
  double v[D + 1];
  v[0] = ref + s[0];
#pragma unroll
  for (int j = 0; j < D; ++j) v[1 + j] = s[1 + j] / dx;
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    if (out64) out64[i * cells + c] = v[i];
    if (out32) out32[i * cells + c] = static_cast<float>(v[i]);
  }
}

// ----------------------------------------------------------------------------
// diagnostics: FP64 partials of a persistent grid, then one fixed-order pass
//   partial slots: 0 sum rho, 1..3 sum q_j, 4 sum |q|^2/rho, 5 sum |curl u|^2,
//   6 sum (div u)^2, 7 max |u|^2, 8 min rho, 9 max rho, 10 non-finite cells
// The grid has min(tiles, kDiagMaxBlocks) blocks; block b walks the tiles
// b, b + G, b + 2G, ... of the XCD-major tile order, so the blocks that run
// together on one XCD hold neighbouring tiles and share their halo lines in
// its L2.  Each thread accumulates its cells' contributions in that fixed
// order and the block reduces them once, so the result does not depend on
// timing, and the final pass reads at most kDiagMaxBlocks partials.
// ----------------------------------------------------------------------------
constexpr int kDiagSlots = 16;
constexpr int kDiagThreads = 256;

template <int D>
struct DiagTile;
template <>
struct DiagTile<2> {
  static constexpr int TX = 64, TY = 16, TZ = 1;
};
template <>
struct DiagTile<3> {
  static constexpr int TX = 32, TY = 8, TZ = 4;
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ void combine(double (&a)[kDiagSlots], const double (&b)[kDiagSlots]) {
#pragma unroll
  for (int s = 0; s < 7; ++s) a[s] += b[s];
  a[7] = fmax(a[7], b[7]);
  a[8] = fmin(a[8], b[8]);
  a[9] = fmax(a[9], b[9]);
  a[10] += b[10];
}

__device__ __forceinline__ void identity(double (&a)[kDiagSlots]) {
#pragma unroll
  for (int s = 0; s < kDiagSlots; ++s) a[s] = 0.0;
  a[8] = INFINITY;
  a[9] = -INFINITY;
}

// Reduce a[] over the 256 threads of the block in a fixed order; thread 0 ends
// with the result.
__device__ void block_reduce(double (&a)[kDiagSlots]) {
  __shared__ double red[kDiagThreads / 64][kDiagSlots];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double b[kDiagSlots];
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) b[s] = __shfl_xor(a[s], off, 64);
    combine(a, b);
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) red[wave][s] = a[s];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) a[s] = red[0][s];
    for (int w = 1; w < kDiagThreads / 64; ++w) {
      double b[kDiagSlots];
#pragma unroll
      for (int s = 0; s < kDiagSlots; ++s) b[s] = red[w][s];
      combine(a, b);
    }
  }
}

template <int D>
__host__ __device__ inline int64_t diag_tile_count(int nx, int ny, int nz) {
  using T = DiagTile<D>;
  return static_cast<int64_t>((nx + T::TX - 1) / T::TX) * ((ny + T::TY - 1) / T::TY) *
         (D == 3 ? (nz + T::TZ - 1) / T::TZ : 1);
}

template <int D, typename TR, typename TM>
__global__ __launch_bounds__(kDiagThreads) void k_diag(const TR* __restrict__ r,
                                                      const TM* __restrict__ m, int nx, int ny,
                                                      int nz, int64_t stride, double ref, double dx,
                                                      double* __restrict__ partials) {
  using T = DiagTile<D>;
  constexpr int HX = T::TX + 2, HY = T::TY + 2, HZ = (D == 3) ? T::TZ + 2 : 1;
  constexpr int HN = HX * HY * HZ;
  constexpr int CELLS = T::TX * T::TY * T::TZ;
  static_assert(CELLS % kDiagThreads == 0, "whole cells per thread");
  __shared__ double sw[D + 1][HN];  // rho, q_j on the tile plus a one-cell halo
  const int tiles_x = (nx + T::TX - 1) / T::TX, tiles_y = (ny + T::TY - 1) / T::TY;
  const int nt = static_cast<int>(diag_tile_count<D>(nx, ny, nz));
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const double inv2dx = 1.0 / (2.0 * dx);
  double a[kDiagSlots];
  identity(a);
  for (int sched = blockIdx.x; sched < nt; sched += gridDim.x) {
    // XCD-major tile order (a grid that is a multiple of 8 keeps each
    // block's schedule indices on its XCD)
    const int t = static_cast<int>(xcd_major(sched, nt));
    const int x0 = (t % tiles_x) * T::TX, y0 = ((t / tiles_x) % tiles_y) * T::TY;
    const int z0 = (D == 3) ? (t / (tiles_x * tiles_y)) * T::TZ : 0;
    __syncthreads();  // the previous tile's LDS values are no longer read
    for (int h = threadIdx.x; h < HN; h += kDiagThreads) {
      const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
      const int gx = wrap(x0 + hx - 1, nx), gy = wrap(y0 + hy - 1, ny);
      const int gz = (D == 3) ? wrap(z0 + hz - 1, nz) : 0;
      const int64_t c = static_cast<int64_t>(gz) * plane + static_cast<int64_t>(gy) * nx + gx;
      double s[D + 1];
      cell_sums<D>(r, m, c, stride, s);
      sw[0][h] = ref + s[0];
#pragma unroll
      for (int j = 0; j < D; ++j) sw[1 + j][h] = s[1 + j] / dx;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CELLS / kDiagThreads; ++k) {
      const int o = static_cast<int>(threadIdx.x) + k * kDiagThreads;
      const int tx = o % T::TX, ty = (o / T::TX) % T::TY, tz = o / (T::TX * T::TY);
      const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
      if (x >= nx || y >= ny || (D == 3 && z >= nz)) continue;
      const int h = ((tz + (D == 3 ? 1 : 0)) * HY + (ty + 1)) * HX + (tx + 1);
      const int sx = 1, sy = HX, sz = HX * HY;
      const double rho = sw[0][h];
      double q[D], q2 = 0.0;
      bool finite = isfinite(rho);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        q[j] = sw[1 + j][h];
        finite = finite && isfinite(q[j]);
        q2 += q[j] * q[j];
      }
      const double u2 = q2 / (rho * rho);
      // u_j at the neighbour at offset o
      auto U = [&](int j, int off) { return sw[1 + j][h + off] / sw[0][h + off]; };
      const int st[3] = {sx, sy, sz};
      double div = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) div += (U(j, st[j]) - U(j, -st[j])) * inv2dx;
      double curl2 = 0.0;
      if constexpr (D == 2) {
        const double w = (U(1, sx) - U(1, -sx)) * inv2dx - (U(0, sy) - U(0, -sy)) * inv2dx;
        curl2 = w * w;
      } else {
        const double wx = (U(2, sy) - U(2, -sy)) * inv2dx - (U(1, sz) - U(1, -sz)) * inv2dx;
        const double wy = (U(0, sz) - U(0, -sz)) * inv2dx - (U(2, sx) - U(2, -sx)) * inv2dx;
        const double wz = (U(1, sx) - U(1, -sx)) * inv2dx - (U(0, sy) - U(0, -sy)) * inv2dx;
        curl2 = wx * wx + wy * wy + wz * wz;
      }
      a[0] += rho;
#pragma unroll
      for (int j = 0; j < D; ++j) a[1 + j] += q[j];
      a[4] += q2 / rho;
      a[5] += curl2;
      a[6] += div * div;
      a[7] = fmax(a[7], u2);
      a[8] = fmin(a[8], rho);
      a[9] = fmax(a[9], rho);
      a[10] += finite ? 0.0 : 1.0;
    }
  }
  block_reduce(a);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) partials[static_cast<int64_t>(blockIdx.x) * kDiagSlots + s] = a[s];
  }
}

// The final pass: thread t combines partials t, t + 256, ... in order, then
// the block reduces them in a fixed order.
__global__ __launch_bounds__(kDiagThreads) void k_diag_final(const double* __restrict__ partials,
                                                            int64_t nblocks,
                                                            double* __restrict__ result) {
  double a[kDiagSlots];
  identity(a);
  for (int64_t b = threadIdx.x; b < nblocks; b += kDiagThreads) {
    double v[kDiagSlots];
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) v[s] = partials[b * kDiagSlots + s];
    combine(a, v);
  }
  block_reduce(a);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) result[s] = a[s];
  }
}

// ----------------------------------------------------------------------------
// copy probe: one 16-byte load and store per thread, one block per 4 KiB
// (the fastest of the copy shapes measured on MI355X: grid-stride loops and
// several vectors per thread were slower)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
// 3D three-step launch: 64 x k3Rows column tiles on 64 (k3Rows + 5) threads,
// one block per compute unit (FP32: 147 KB of LDS; 16-bit: the registers,
// 127-128 VGPRs of the 128 that 13 waves leave).
constexpr int k3Rows = 8;

}  // namespace

// Planes per block of a 3D z-marching launch of `stages` fused steps on
// 64 x ky column tiles, `per_cu` blocks per compute unit.  The launch runs in
// rounds of per_cu x cus blocks and a partial last round leaves the rest of
// the chip idle; a block also recomputes 2 (stages - s) extra planes of its
// stage s, over a (64 + 2 (stages - s)) x (ky + 2 (stages - s)) region, at the
// ends of its segment.  The segment length minimises rounds x the work of one
// block (256^3 on 256 units, three steps on 64 x 8 tiles: 128 planes, 256
// blocks in one round; 64- and 32-plane segments, in two and four rounds, ran
// 15% and 18% slower).
int32_t zseg_for(const Geometry& g, int ky, int stages, int per_cu, int cus) {
  const int64_t txy = static_cast<int64_t>((g.nx + 63) / 64) * ((g.ny + ky - 1) / ky);
  const int64_t slots = static_cast<int64_t>(std::max(per_cu, 1)) * std::max(cus, 1);
  int32_t best = 32;
  double best_cost = -1.0;
  for (int32_t zs = 8; zs <= std::max<int32_t>(8, g.nz); ++zs) {
    const int64_t blocks = txy * ((g.nz + zs - 1) / zs);
    const int64_t rounds = (blocks + slots - 1) / slots;
    double work = 0.0;
    for (int st = 1; st <= stages; ++st) {
      const int b = 2 * (stages - st);  // border cells per side of stage st
      work += static_cast<double>(zs + b) * static_cast<double>((64 + b) * (ky + b));
    }
    const double cost = static_cast<double>(rounds) * work;
    if (best_cost < 0.0 || cost < best_cost) {
      best_cost = cost;
      best = zs;
    }
  }
  return best;
}

namespace {

template <int D, typename TR, typename TM, bool DEV>
struct Impl {
  static hipError_t init(const Geometry& g, const RunCoef& r, const double* u0, const double* rho0,
                         void* dst, hipStream_t s) {
    auto p = planes_of<TR, TM>(dst, g.rest_bytes);
    const CoefT<double> k = make_coef<double>(r, D, DEV);
    const int64_t blocks = (g.cells + 255) / 256;
    hipLaunchKernelGGL((k_init<D, TR, TM>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, u0,
                       rho0, r.ref, r.dx, p.rest, p.move, g.cells, g.stride, k);
    return hipGetLastError();
  }

  // 3D moment-only storage: the z-marching kernel, 64 x 16 column tiles on
  // 1024 threads, 32-plane segments; two steps per launch: 64 x kM2Y column
  // tiles on 64 (kM2Y + 5) threads, kM2PerCU blocks per compute unit (75 KB
  // of LDS and 60 VGPRs each).  GLUPS at 256^3 by tile height: 64 x 11 (1024
  // threads) 177.9, 64 x 10 (960) 172.4, 64 x 8 (832) 141.6, against 143.3
  // for one step per launch; segment lengths of 16 to 52 planes within 2%.
  static constexpr int kM3X = 64, kM3Y = 16, kM3Z = 32;
  static constexpr int kM2Y = 11, kM2PerCU = 2;

  static hipError_t step(const Geometry& g, const RunCoef& r, const void* src, void* dst, int bx,
                         int by, hipStream_t s) {
    auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
    auto b = planes_of<TR, TM>(dst, g.rest_bytes);
    const auto k = make_coef<typename ComputeOf<TM>::type>(r, D, DEV);
    if constexpr (D == 3 && IsMom<TM>::value) {
      // the z-marching kernel where its launch fills the chip and its 32-bit
      // byte offsets cover a plane; else the cell-parallel kernel (the same
      // stencil, the same bits)
      const int64_t tiles = static_cast<int64_t>((g.nx + kM3X - 1) / kM3X) * ((g.ny + kM3Y - 1) / kM3Y) *
                            ((g.nz + kM3Z - 1) / kM3Z);
      if (tiles >= kMinZmarchBlocks3d && fused_offsets_fit(static_cast<int64_t>(g.nx) * g.ny, sizeof(float))) {
        hipLaunchKernelGGL((k_step_mom_3d<kM3X, kM3Y, kM3Z>), dim3(static_cast<uint32_t>(tiles)), dim3(kM3X * kM3Y),
                           0, s, a.rest, reinterpret_cast<float*>(b.rest), g.nx, g.ny, g.nz, g.stride, k);
        return hipGetLastError();
      }
    }
    dim3 block(bx, by, 1);
    dim3 grid((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, g.nz);
    hipLaunchKernelGGL((k_step<D, TR, TM>), grid, block, 0, s, a.rest, a.move, b.rest, b.move, g.nx,
                       g.ny, g.nz, g.stride, k, neq_scale_of<D>(r));
    return hipGetLastError();
  }

  // Tile of the two-step kernel by storage and grid size, from sweeps of this
  // kernel on MI355X (GLUPS; 128x8 on 512 threads / 256x8 on 1024 / 128x16 on
  // 1024 / 64x8 on 512): 4096^2 FP32 81.1 / 85.8 / 83.2 / 79.6, FP16 148.3 /
  // 137.9 / 121.0 / 128.6, BF16 132.7 / 121.4 / 113.0 / 121.8, FP16 + FP32 rest
  // 129.2 / 122.8 / 114.0 / 115.9; 2048^2 FP32 74.2 / 69.3 / 71.4 / 73.4.  So
  // 256x8 tiles only for 4-byte moving planes from 2^23 cells on.  Up to 256^2
  // cells the launch is latency-bound and 64x4 on 256 threads (256 blocks)
  // beats 128x8 (64 blocks): 20.4 vs 19.4 GLUPS FP32 at 256^2.  The split
  // storage is ALU-bound (it rebuilds the upwind equilibria) and runs 128x8
  // on 1024 threads: 91 vs 85 GLUPS for 128x8/512 (64x8/512: 72, 256x4/1024: 77).
  // 3D: the z-marching two-step kernel for 4-byte planes (FP32, raw FP32)
  // 3D: the z-marching kernels for the population storages (FP32 and the
  // 16-bit deviation storages; not FP64 or the split and moment-only ones)
  static constexpr bool k3DPop = D == 3 && !std::is_same<TM, double>::value && !IsNeq<TM>::value &&
                                 !IsMom<TM>::value;
  // 3D moment-only storage: the z-marching two-step kernel
  static constexpr bool k3DMom = D == 3 && IsMom<TM>::value;
  static constexpr bool kHasStep2 = (D == 2 && !std::is_same<TM, double>::value) || k3DPop || k3DMom;
  // 64 x 8 columns on 704 threads, 32-plane segments (GLUPS at 256^3: 31.5;
  // 32x16 / 640: 29.2, with 64-plane segments 28.2; 64x12 / 960: 27.5;
  // 96x8 / 1024: 28.0; 32x8 and 16x16 / 384: 25.3, 20.9; 16- and 24-plane
  // segments: 29.9, 30.2; one step per launch: 25.2).  The kernel needs 140
  // VGPRs (one block per CU); capping it at 128 or 96 spills.
  static constexpr int kT3X = 64, kT3Y = 8, kT3Z = 32, kT3N = 704;

  template <int TX, int TY, int NT>
  static hipError_t launch2(const Geometry& g, const RunCoef& r, const void* src, void* dst, hipStream_t s) {
    auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
    auto b = planes_of<TR, TM>(dst, g.rest_bytes);
    const Coef k = make_coef<float>(r, D, DEV);
    dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, 1);
    hipLaunchKernelGGL((k_step2_2d<TR, TM, TX, TY, NT>), grid, dim3(NT), 0, s, a.rest, a.move, b.rest, b.move, g.nx,
                       g.ny, g.stride, k, neq_scale_of<2>(r));
    return hipGetLastError();
  }

  static hipError_t step2(const Geometry& g, const RunCoef& r, const void* src, void* dst, hipStream_t s) {
    if constexpr (!kHasStep2) {
      return hipErrorInvalidValue;
    } else if constexpr (k3DMom) {
      // 32-bit byte offsets within a plane (lbm_set_fusion refuses larger planes)
      if (!fused_offsets_fit(static_cast<int64_t>(g.nx) * g.ny, sizeof(float))) return hipErrorInvalidValue;
      auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
      auto b = planes_of<TR, TM>(dst, g.rest_bytes);
      const Coef k = make_coef<float>(r, D, DEV);
      hipLaunchKernelGGL((k_step2_mom_3d<kM2Y>), dim3(static_cast<uint32_t>(launch_blocks(g, 2))),
                         dim3(64 * (kM2Y + 5)), 0, s, a.rest, reinterpret_cast<float*>(b.rest), g.nx, g.ny, g.nz,
                         g.zseg, g.stride, k);
      return hipGetLastError();
    } else if constexpr (D == 3) {
      auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
      auto b = planes_of<TR, TM>(dst, g.rest_bytes);
      const Coef k = make_coef<float>(r, D, DEV);
      const int64_t tiles = static_cast<int64_t>((g.nx + kT3X - 1) / kT3X) * ((g.ny + kT3Y - 1) / kT3Y) *
                            ((g.nz + kT3Z - 1) / kT3Z);
      dim3 grid(static_cast<uint32_t>(tiles), 1, 1);
      hipLaunchKernelGGL((k_step2_3d<TR, TM, kT3X, kT3Y, kT3Z, kT3N>), grid, dim3(kT3N), 0, s, a.rest, a.move, b.rest,
                         b.move, g.nx, g.ny, g.nz, g.stride, k);
      return hipGetLastError();
    } else if constexpr (IsNeq<TM>::value) {
      return launch2<128, 8, 1024>(g, r, src, dst, s);
    } else if constexpr (IsMom<TM>::value) {
      return launch2<256, 8, 1024>(g, r, src, dst, s);
    } else {
      if (sizeof(TM) == 4 && g.cells >= (int64_t(1) << 23)) return launch2<256, 8, 1024>(g, r, src, dst, s);
      if (g.cells <= (int64_t(1) << 16)) return launch2<64, 4, 256>(g, r, src, dst, s);
      return launch2<128, 8, 512>(g, r, src, dst, s);
    }
  }

  // K = 3 .. 6 steps per launch (2D population storages) in XCD-major tile
  // order.  4-byte planes: k_stepKr_2d (rest populations in registers), 32x16
  // tiles on 256 threads; 16-bit moving planes: k_stepK_2d, 64x16 tiles on
  // 512 threads (1024 threads ran FP16 + FP32 rest at 124 against 154 GLUPS
  // at 4096^2 in this library's build).  From
  // sweeps of the engine's instantiations on MI355X (GLUPS at 4096^2 / 2048^2 /
  // 1024^2, two steps per launch first): FP32 86.9 / 68.5 / 63.8 against 114.3 /
  // 121.7 / 118.6 for k_stepK_2d at K = 5 and 130.2 / 132.8 for k_stepKr_2d;
  // FP16 140.3 / 116.4 / 119.5 against 173.9 / 165.6 / 145.4; FP16 + FP32 rest
  // 124.5 / 108.5 / 100.9 against 197.9 / 189.6 / 163.4.
  // Deeper fusion moves fewer HBM bytes per step (the state is read about
  // (TX+2K)(TY+2K)/(TX TY) times and written once per K steps) at the price of
  // recomputing the shrinking borders; K = 6..8 and 32x16, 32x32 or 64x32
  // tiles were within a few percent or slower.
  static constexpr bool kHasStepK = (kHasStep2 && D == 2) || k3DPop;
  // most steps per launch: 6 in 2D, 3 for the 3D FP32 storages, else the
  // two-step kernel's 2 or one
  static constexpr int kMaxFuse = kHasStepK ? (D == 2 ? kMaxFusion : 3) : kHasStep2 ? 2 : 1;
  static constexpr int kRows3 = (D == 3 && kHasStepK) ? k3Rows : 0;

  // planes per block of the deepest 3D z-marching launch of this storage
  static int32_t zseg(const Geometry& g, int cus) {
    if constexpr (k3DMom) return zseg_for(g, kM2Y, 2, kM2PerCU, cus);
    return zseg_for(g, kRows3 > 0 ? kRows3 : 8, 3, 1, cus);
  }
  // threads of the 16-bit multi-step tile (64x16): 768 where the rest planes
  // are FP32 (FP16 + FP32 rest 194.8 -> 203.3, BF16 + FP32 rest 191.6 ->
  // 201.8 GLUPS at 4096^2), 512 for the all-16-bit storages (768 ran BF16 at
  // 201.4 against 212.8, FP16 equal)
  static constexpr int kStepKThreads = sizeof(TR) == 4 ? 768 : 512;

  static constexpr bool kRestInRegisters = sizeof(TR) == 4 && sizeof(TM) == 4;
  // split FP16 storage: 32x24 tiles on 1024 threads (GLUPS at 4096^2 / 2048^2
  // at K = 5: 139.9 / 135.1; on 768 threads 137.6 / 125.8; 32x16 on 512 116.4 /
  // 107.9; 64x8 on 512 107.6 / 102.2; 64x16 and 32x32 on 512 88.5 and 82.2;
  // 32x24 at K = 4: 119.2).  Its 77 KB of FP32 populations in LDS is the
  // largest five-step tile of which two fit in one CU.  Every stage rebuilds
  // the storage rounding, so the kernel is ALU-bound.
  struct NeqKTile {
    static constexpr int TX = 32, TY = 24, NT = 1024;
  };

  template <int K>
  static hipError_t launchK(const Geometry& g, const RunCoef& r, const void* src, void* dst, hipStream_t s) {
    auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
    auto b = planes_of<TR, TM>(dst, g.rest_bytes);
    const Coef k = make_coef<float>(r, D, DEV);
    if constexpr (IsNeq<TM>::value) {
      constexpr int TX = NeqKTile::TX, TY = NeqKTile::TY, NT = NeqKTile::NT;
      const int64_t tiles = static_cast<int64_t>((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
      hipLaunchKernelGGL((k_stepK_neq_2d<TX, TY, NT, K, true>), dim3(static_cast<uint32_t>(tiles)), dim3(NT), 0, s,
                         a.rest, a.move, b.rest, b.move, g.nx, g.ny, g.stride, k, neq_scale_of<2>(r));
    } else if constexpr (IsMom<TM>::value) {
      // moment-only storage: 64x32 tiles on 512 threads in raster order (sweep
      // at 4096^2 / 2048^2, GLUPS: two steps 264.9 / 223.8; four steps 363.2 /
      // 332.4; five steps with 64x16 tiles on 256 threads 352.3 / 314.3; XCD
      // order was a few percent slower here)
      constexpr int TX = 64, TY = 32, NT = 512;
      dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, 1);
      hipLaunchKernelGGL((k_stepK_mom_2d<TX, TY, NT, K, false>), grid, dim3(NT), 0, s, a.rest,
                         reinterpret_cast<float*>(b.rest), g.nx, g.ny, g.stride, k);
    } else if constexpr (kRestInRegisters) {
      // the tile per depth (inner-first cell order; GLUPS at 4096^2 / 2048^2):
      // K = 5: 32x32, 159.7 / 136.0 on 512 threads (its 77 KB of LDS lets two
      // blocks share a CU; 135.5 without the XCD order), against 145.3 / 136.4
      // for 32x16 on 256; on 768 threads (24 waves per CU instead of 16,
      // 60 VGPRs) 177.5 against 172.7 after the relaxation change (640: 115);
      // K = 4: 64x16 on 512, 139.3 / 132.9 against 125.0 / 122.1; K = 3:
      // 32x16 on 256 (102.2 at 4096^2); K = 6 (the FP32 default): 32x28 on 768
      // threads, 42x38 extended, 77 KB of LDS, two blocks per CU, 192.6 against 176.3 for
      // K = 5 in the same session (32x24: 182.2, 32x16 on 256: 152.8, 32x16
      // and 32x20 on 512 (three and two blocks per CU): 166, 32x28 on 832,
      // 896 or 1024 threads: 118-120; K = 7 on 32x24: 191.5, K = 8 on 32x20:
      // 177.8; 32x32 at K = 6 needs 85 KB per block and ran 108.6)
      constexpr int TX = K == 5 ? 32 : K == 4 ? 64 : 32;
      constexpr int TY = K == 5 ? 32 : K == 6 ? 28 : 16;
      constexpr int NT = K == 5 ? 768 : K == 4 ? 512 : K == 6 ? 768 : 256;
      const int64_t tiles = static_cast<int64_t>((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
      hipLaunchKernelGGL((k_stepKr_2d<TR, TM, TX, TY, NT, K, true>), dim3(static_cast<uint32_t>(tiles)), dim3(NT), 0,
                         s, a.rest, a.move, b.rest, b.move, g.nx, g.ny, g.stride, k);
    } else {
      // 64x16, or 64x20 at six steps with FP32 rest planes (80 KB of LDS, two
      // blocks per CU: FP16 + FP32 rest 210.0 GLUPS against 203.4 at five
      // steps on 64x16; 32x28 at six: 190.1; the all-16-bit storages stay at
      // five, BF16 214.5 against 210.7 at six on 64x20)
      constexpr int TX = 64, TY = (K == 6 && sizeof(TR) == 4) ? 20 : 16;
      const int64_t tiles = static_cast<int64_t>((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
      hipLaunchKernelGGL((k_stepK_2d<TR, TM, TX, TY, kStepKThreads, K, true>), dim3(static_cast<uint32_t>(tiles)),
                         dim3(kStepKThreads), 0, s, a.rest, a.move, b.rest, b.move, g.nx, g.ny, g.stride, k);
    }
    return hipGetLastError();
  }

  static hipError_t stepK(const Geometry& g, const RunCoef& r, int K, const void* src, void* dst,
                          hipStream_t s) {
    if constexpr (!kHasStepK) {
      return hipErrorInvalidValue;
    } else if constexpr (D == 3) {
      if (K != 3) return hipErrorInvalidValue;
      auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
      auto b = planes_of<TR, TM>(dst, g.rest_bytes);
      const Coef k = make_coef<float>(r, D, DEV);
      const int64_t tiles = launch_blocks(g, 3);
      constexpr int KY = k3Rows;
      hipLaunchKernelGGL((k_step3_3d<TR, TM, KY>), dim3(static_cast<uint32_t>(tiles)), dim3(64 * (KY + 5)), 0, s,
                         a.rest, a.move, b.rest, b.move, g.nx, g.ny, g.nz, g.zseg, g.stride, k);
      return hipGetLastError();
    } else {
      switch (K) {
        case 3: return launchK<3>(g, r, src, dst, s);
        case 4: return launchK<4>(g, r, src, dst, s);
        case 5: return launchK<5>(g, r, src, dst, s);
        case 6: return launchK<6>(g, r, src, dst, s);
      }
      return hipErrorInvalidValue;
    }
  }

  static constexpr bool kHasWalls = D == 2 && !StoresMoments<TM>::value;

  static hipError_t step_walls(const Geometry& g, const RunCoef& r, const void* src, void* dst, const WallArgs& w,
                               int bx, int by, hipStream_t s) {
    if constexpr (!kHasWalls) {
      return hipErrorInvalidValue;
    } else {
      auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
      auto b = planes_of<TR, TM>(dst, g.rest_bytes);
      const auto k = make_coef<typename ComputeOf<TM>::type>(r, D, DEV);
      dim3 block(bx, by, 1);
      dim3 grid((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, 1);
      hipLaunchKernelGGL((k_step_walls<TR, TM>), grid, block, 0, s, a.rest, a.move, b.rest, b.move, g.nx, g.ny,
                         g.stride, k, w);
      return hipGetLastError();
    }
  }

  static hipError_t moments(const Geometry& g, const RunCoef& r, const void* src, double* out64,
                            float* out32, hipStream_t s) {
    auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
    const int64_t blocks = (g.cells + 255) / 256;
    hipLaunchKernelGGL((k_moments<D, TR, TM>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       a.rest, a.move, g.cells, g.stride, DEV ? r.ref : 0.0, r.dx, out64, out32);
    return hipGetLastError();
  }

  static int64_t diag_blocks(const Geometry& g) {
    const int64_t nt = diag_tile_count<D>(g.nx, g.ny, g.nz);
    return nt < kDiagMaxBlocks ? nt : kDiagMaxBlocks;
  }

  static hipError_t diag(const Geometry& g, const RunCoef& r, const void* src, double* partials,
                         double* result, hipStream_t s) {
    auto a = planes_of<TR, TM>(const_cast<void*>(src), g.rest_bytes);
    hipLaunchKernelGGL((k_diag<D, TR, TM>), dim3(static_cast<uint32_t>(diag_blocks(g))), dim3(kDiagThreads), 0, s,
                       a.rest, a.move, g.nx, g.ny, g.nz, g.stride, DEV ? r.ref : 0.0, r.dx, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, s, partials, diag_blocks(g),
                       result);
    return hipGetLastError();
  }

  static int64_t launch_blocks(const Geometry& g, int depth) {
    if constexpr (D == 3) {
      if (depth >= 3 && kHasStepK)
        return static_cast<int64_t>((g.nx + 63) / 64) * ((g.ny + kRows3 - 1) / kRows3) *
               ((g.nz + g.zseg - 1) / g.zseg);
      if (depth == 2 && k3DMom)
        return static_cast<int64_t>((g.nx + 63) / 64) * ((g.ny + kM2Y - 1) / kM2Y) * ((g.nz + g.zseg - 1) / g.zseg);
      if (depth == 2 && kHasStep2)
        return static_cast<int64_t>((g.nx + kT3X - 1) / kT3X) * ((g.ny + kT3Y - 1) / kT3Y) *
               ((g.nz + kT3Z - 1) / kT3Z);
    }
    return INT64_MAX;
  }

  static const Ops* ops() {
    static const Ops o = {&init, &step, kHasStep2 ? &step2 : nullptr, &moments, &diag, &diag_blocks,
                          kHasWalls ? &step_walls : nullptr, kHasStepK ? &stepK : nullptr, kMaxFuse,
                          &launch_blocks, (k3DPop || k3DMom) ? &zseg : nullptr};
    return &o;
  }
};

}  // namespace

const Ops* ops_for(int dim, int storage) {
  if (dim == 2) {
    switch (storage) {
      case LBM_F32: return Impl<2, float, float, true>::ops();
      case LBM_F32_RAW: return Impl<2, float, float, false>::ops();
      case LBM_F16_DEV: return Impl<2, _Float16, _Float16, true>::ops();
      case LBM_BF16_DEV: return Impl<2, bf16, bf16, true>::ops();
      case LBM_F16_DEV_R32: return Impl<2, float, _Float16, true>::ops();
      case LBM_BF16_DEV_R32: return Impl<2, float, bf16, true>::ops();
      case LBM_F64: return Impl<2, double, double, true>::ops();
      case LBM_F16_NEQ: return Impl<2, float, neq16, true>::ops();
      case LBM_F32_MOMENTS: return Impl<2, float, mom0, true>::ops();
    }
  } else if (dim == 3) {
    switch (storage) {
      case LBM_F32: return Impl<3, float, float, true>::ops();
      case LBM_F32_RAW: return Impl<3, float, float, false>::ops();
      case LBM_F16_DEV: return Impl<3, _Float16, _Float16, true>::ops();
      case LBM_BF16_DEV: return Impl<3, bf16, bf16, true>::ops();
      case LBM_F16_DEV_R32: return Impl<3, float, _Float16, true>::ops();
      case LBM_BF16_DEV_R32: return Impl<3, float, bf16, true>::ops();
      case LBM_F64: return Impl<3, double, double, true>::ops();
      case LBM_F16_NEQ: return Impl<3, float, neq16, true>::ops();
      case LBM_F32_MOMENTS: return Impl<3, float, mom0, true>::ops();
    }
  }
  return nullptr;
}

bool storage_elems(int storage, size_t* rest_elem, size_t* move_elem) {
  switch (storage) {
    case LBM_F32:
    case LBM_F32_RAW: *rest_elem = 4; *move_elem = 4; return true;
    case LBM_F16_DEV:
    case LBM_BF16_DEV: *rest_elem = 2; *move_elem = 2; return true;
    case LBM_F16_DEV_R32:
    case LBM_BF16_DEV_R32:
    case LBM_F16_NEQ: *rest_elem = 4; *move_elem = 2; return true;
    case LBM_F64: *rest_elem = 8; *move_elem = 8; return true;
    case LBM_F32_MOMENTS: *rest_elem = 4; *move_elem = 0; return true;
  }
  return false;
}

Geometry make_geometry(int dim, int storage, const int64_t n[3]) {
  Geometry g;
  g.dim = dim;
  g.nx = static_cast<int32_t>(n[0]);
  g.ny = static_cast<int32_t>(n[1]);
  g.nz = static_cast<int32_t>(n[2]);
  g.cells = n[0] * n[1] * n[2];
  g.stride = (g.cells + 255) / 256 * 256;
  storage_elems(storage, &g.rest_elem, &g.move_elem);
  const int ns = dim + 1;
  auto align = [](size_t v) { return (v + 255) / 256 * 256; };
  g.rest_bytes = align(static_cast<size_t>(ns) * g.stride * g.rest_elem);
  g.buf_bytes = align(g.rest_bytes + static_cast<size_t>(ns) * 2 * dim * g.stride * g.move_elem);
  return g;
}

bool storage_is_deviation(int storage) { return storage != LBM_F32_RAW; }

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(bytes / 16);
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n);
  return hipGetLastError();
}

}  // namespace lbm
