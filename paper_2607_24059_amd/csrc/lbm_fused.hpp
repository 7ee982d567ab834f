// Tiles of the fused multi-step update (2D population storages), shared by
// the single-run kernels (lbm_kernels.hip) and the batch engine
// (lbm_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm {

// ----------------------------------------------------------------------------
// K >= 3 steps in one launch (2D, population storages): the block advances its
// TX x TY tile plus a (K-1)-cell border by one step from HBM into LDS, then
// K-2 more steps in LDS, each over a region one cell narrower on every side
// (the cells whose inputs are still valid), and the tile by the last step to
// HBM.  A step inside LDS gathers and relaxes its cells into registers, waits
// for every thread, and writes them back over the same LDS slots, so one LDS
// buffer serves all stages.  Every intermediate value is rounded to the
// storage type when it is written to LDS, as a store to HBM would round it, so
// the result equals K single steps bit for bit.  Each state value is read from
// HBM about (TX+2K)(TY+2K)/(TX TY) times and written once per K steps.
// ----------------------------------------------------------------------------
template <typename TR, typename TM, int EX, int EN>
__device__ __forceinline__ void gather_lds(const TR (&s_rest)[3][EN], const TM (&s_move)[12][EN], int e,
                                           float (&g)[3][5]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[i][0] = load_f32(&s_rest[i][e]);
    g[i][1] = load_f32(&s_move[i * 4 + 0][e - 1]);   // +x from x-1
    g[i][2] = load_f32(&s_move[i * 4 + 1][e + 1]);   // -x from x+1
    g[i][3] = load_f32(&s_move[i * 4 + 2][e - EX]);  // +y from y-1
    g[i][4] = load_f32(&s_move[i * 4 + 3][e + EX]);  // -y from y+1
  }
}

// one step inside LDS over the region [LO, EX - LO) x [LO, EY - LO)
template <typename TR, typename TM, int EX, int EY, int NT, int LO>
__device__ __forceinline__ void lds_stage(TR (&s_rest)[3][EX * EY], TM (&s_move)[12][EX * EY], const Coef& k) {
  constexpr int EN = EX * EY, RX = EX - 2 * LO, RY = EY - 2 * LO, RN = RX * RY;
  constexpr int PER = (RN + NT - 1) / NT;
  float keep[PER][3][5];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int t = static_cast<int>(threadIdx.x) + j * NT;
    if (t < RN) {
      const int e = (LO + t / RX) * EX + LO + t % RX;
      gather_lds<TR, TM, EX, EN>(s_rest, s_move, e, keep[j]);
      collide<2>(keep[j], k);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int t = static_cast<int>(threadIdx.x) + j * NT;
    if (t < RN) {
      const int e = (LO + t / RX) * EX + LO + t % RX;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        store_f32(&s_rest[i][e], keep[j][i][0]);
#pragma unroll
        for (int m = 0; m < 4; ++m) store_f32(&s_move[i * 4 + m][e], keep[j][i][1 + m]);
      }
    }
  }
  __syncthreads();
}

template <typename TR, typename TM, int EX, int EY, int NT, int LO, int LAST>
__device__ __forceinline__ void lds_stages(TR (&s_rest)[3][EX * EY], TM (&s_move)[12][EX * EY], const Coef& k) {
  if constexpr (LO <= LAST) {
    lds_stage<TR, TM, EX, EY, NT, LO>(s_rest, s_move, k);
    lds_stages<TR, TM, EX, EY, NT, LO + 1, LAST>(s_rest, s_move, k);
  }
}

// The first step of a tile reads its whole extended tile from HBM while the
// other block on the compute unit works in LDS; raising the wave priority over
// that step gets its loads issued ahead of the other block's arithmetic
// (five-step FP32 tiles at 4096^2: 168 against 159 GLUPS; raising it over the
// last step's stores as well: 165; moment-only tiles 311 against 264).
// Results do not depend on it.
__device__ __forceinline__ void hbm_phase_begin() { __builtin_amdgcn_s_setprio(1); }
__device__ __forceinline__ void hbm_phase_end() { __builtin_amdgcn_s_setprio(0); }

// origin of the tile that block b takes, in XCD-major order (xcd_major)
__device__ __forceinline__ void xcd_tile_origin(int b, int nx, int ny, int TX, int TY, int* x0, int* y0) {
  const int tiles_x = (nx + TX - 1) / TX;
  const int nt = tiles_x * ((ny + TY - 1) / TY);
  const int t = static_cast<int>(xcd_major(b, nt));
  *x0 = (t % tiles_x) * TX;
  *y0 = (t / tiles_x) * TY;
}

// The K-step tile with its origin (x0, y0); s_rest and s_move are the block's
// LDS tile (TileK<..>::EN cells).
template <typename TR, typename TM, int TX, int TY, int NT, int K>
struct TileK {
  static_assert(K >= 3, "two steps per launch use the two-step tile");
  static constexpr int H = K - 1, EX = TX + 2 * H, EY = TY + 2 * H, EN = EX * EY;

  __device__ static void run(const TR* __restrict__ sr, const TM* __restrict__ sm, TR* __restrict__ dr,
                             TM* __restrict__ dm, int x0, int y0, int nx, int ny, int64_t stride, const Coef& k,
                             TR (&s_rest)[3][EN], TM (&s_move)[12][EN]) {
    // first step, from HBM, over the whole extended tile
    hbm_phase_begin();
    for (int e = threadIdx.x; e < EN; e += NT) {
      const int ex = e % EX, ey = e / EX;
      int x = x0 - H + ex, y = y0 - H + ey;
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
    hbm_phase_end();
    __syncthreads();
    // steps 2 .. K-1 in LDS
    lds_stages<TR, TM, EX, EY, NT, 1, H - 1>(s_rest, s_move, k);
    // last step, from LDS to HBM, over the tile
    for (int t = threadIdx.x; t < TX * TY; t += NT) {
      const int tx = t % TX, ty = t / TX;
      const int x = x0 + tx, y = y0 + ty;
      if (x >= nx || y >= ny) continue;
      float g[3][5];
      gather_lds<TR, TM, EX, EN>(s_rest, s_move, (ty + H) * EX + (tx + H), g);
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
};

// Accesses at a byte offset from a plane base that is the same for the whole
// block: the compiler then keeps the 64-bit base in scalar registers and
// issues the scalar-base form of the load or store with a 32-bit lane offset,
// so no 64-bit address arithmetic runs on the vector ALU per access.  Valid
// while every byte offset within a plane fits in 32 bits (fused_offsets_fit).
template <typename T>
__device__ __forceinline__ const T* at_byte(const T* base, uint32_t off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ T* at_byte(T* base, uint32_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

// Pull gather of 2D cell c = y nx + x (periodic) with 32-bit plane offsets.
template <typename TR, typename TM>
__device__ __forceinline__ void gather_cell2_o32(const TR* __restrict__ sr, const TM* __restrict__ sm, int x, int y,
                                                 int nx, int ny, int64_t stride, float (&g)[3][5]) {
  const uint32_t c = static_cast<uint32_t>(y) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x);
  const uint32_t row = static_cast<uint32_t>(nx), last = static_cast<uint32_t>(ny - 1) * row;
  uint32_t src[4];
  src[0] = (x == 0) ? c + (row - 1) : c - 1;     // +x from x-1
  src[1] = (x == nx - 1) ? c - (row - 1) : c + 1; // -x from x+1
  src[2] = (y == 0) ? c + last : c - row;         // +y from y-1
  src[3] = (y == ny - 1) ? c - last : c + row;    // -y from y+1
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[i][0] = load_f32(at_byte(sr + i * stride, c * static_cast<uint32_t>(sizeof(TR))));
#pragma unroll
    for (int m = 0; m < 4; ++m)
      g[i][1 + m] = load_f32(at_byte(sm + (i * 4 + m) * stride, src[m] * static_cast<uint32_t>(sizeof(TM))));
  }
}

// Whether every element offset of a plane of `cells` values fits the 32-bit
// byte offsets of gather_cell2_o32 (host side).
__host__ __device__ inline bool fused_offsets_fit(int64_t cells, size_t elem_bytes) {
  return cells * static_cast<int64_t>(elem_bytes) <= (int64_t(1) << 32);
}

// Variant for 4-byte planes with the rest populations in registers: every
// thread owns the same cells of the extended tile in all K steps (ownership
// index threadIdx + j NT, mapped to cells by cell_of), so a cell's rest
// populations, which only that cell reads, never go through LDS; LDS holds the
// 12 moving planes only (48 B per cell in FP32, against 60 B).  Not used for 16-bit planes: there the compiler turns
// the last relaxation FMA and the rounding to FP16 into one fused instruction
// (one rounding) in some kernels and not in others (two roundings), and this
// kernel's register round trip of the rest values takes the two-rounding form,
// which differs from the single-step kernel in one FP16 ulp now and then.
template <typename TR, typename TM, int TX, int TY, int NT, int K>
struct TileKr {
  static_assert(K >= 2, "at least two steps");
  static constexpr int H = K - 1, EX = TX + 2 * H, EY = TY + 2 * H, EN = EX * EY;
  static constexpr int PER = (EN + NT - 1) / NT;

  // Cell of ownership index o: the TX x TY inner cells first, row by row (so
  // a wave owns whole rows of the tile and its last-step stores cover whole
  // 128-byte lines, and the last step runs on the first TX TY / NT indices
  // only), then the border cells in raster order of the extended tile.
  __device__ static __forceinline__ void cell_of(int o, int& ex, int& ey) {
    if (o < TX * TY) {
      ex = H + o % TX;
      ey = H + o / TX;
      return;
    }
    int b = o - TX * TY;
    if (b < H * EX) {
      ex = b % EX;
      ey = b / EX;
      return;
    }
    b -= H * EX;
    if (b < TY * 2 * H) {
      const int c = b % (2 * H);
      ex = c < H ? c : c + TX;
      ey = H + b / (2 * H);
      return;
    }
    b -= TY * 2 * H;
    ex = b % EX;
    ey = H + TY + b / EX;
  }

  __device__ static void run(const TR* __restrict__ sr, const TM* __restrict__ sm, TR* __restrict__ dr,
                             TM* __restrict__ dm, int x0, int y0, int nx, int ny, int64_t stride, const Coef& k,
                             TM (&s_move)[12][EN]) {
    float rest[PER][3];   // this thread's cells' rest populations (storage-rounded)
    float mv[PER][12];    // moving populations computed in the current step
    int e_of[PER];        // LDS slot of each of this thread's cells
    int d_of[PER];        // its distance from the inner tile (step st updates d <= K - st)
    // step 1 from HBM over the whole extended tile
    hbm_phase_begin();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int o = static_cast<int>(threadIdx.x) + j * NT;
      int ex, ey;
      cell_of(o, ex, ey);
      const int e = ey * EX + ex;
      e_of[j] = e;
      d_of[j] = o < EN ? max(max(max(H - ex, ex - (H + TX - 1)), max(H - ey, ey - (H + TY - 1))), 0) : K;
      if (o < EN) {
        int x = x0 - H + ex, y = y0 - H + ey;
        x = wrap_coord(x, nx);
        y = wrap_coord(y, ny);
        float g[3][5];
        gather_cell2_o32<TR, TM>(sr, sm, x, y, nx, ny, stride, g);
        collide<2>(g, k);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          TR rr;
          store_f32(&rr, g[i][0]);
          rest[j][i] = load_f32(&rr);
#pragma unroll
          for (int m = 0; m < 4; ++m) store_f32(&s_move[i * 4 + m][e], g[i][1 + m]);
        }
      }
    }
    hbm_phase_end();
    __syncthreads();
    // steps 2 .. K-1 in LDS over shrinking regions, then step K to HBM
#pragma unroll
    for (int st = 2; st <= K; ++st) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = e_of[j];
        const bool in = d_of[j] <= K - st;
        if (in) {
          float g[3][5];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            g[i][0] = rest[j][i];
            g[i][1] = load_f32(&s_move[i * 4 + 0][e - 1]);
            g[i][2] = load_f32(&s_move[i * 4 + 1][e + 1]);
            g[i][3] = load_f32(&s_move[i * 4 + 2][e - EX]);
            g[i][4] = load_f32(&s_move[i * 4 + 3][e + EX]);
          }
          collide<2>(g, k);
          if (st < K) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              TR rr;
              store_f32(&rr, g[i][0]);
              rest[j][i] = load_f32(&rr);
#pragma unroll
              for (int m = 0; m < 4; ++m) mv[j][i * 4 + m] = g[i][1 + m];
            }
          } else {
            // the last step updates the inner cells only: o < TX TY
            const int o = static_cast<int>(threadIdx.x) + j * NT;
            const int x = x0 + o % TX, y = y0 + o / TX;
            if (x < nx && y < ny) {
              const uint32_t c = static_cast<uint32_t>(y) * static_cast<uint32_t>(nx) + static_cast<uint32_t>(x);
#pragma unroll
              for (int i = 0; i < 3; ++i) {
                store_stream(at_byte(dr + i * stride, c * static_cast<uint32_t>(sizeof(TR))), g[i][0]);
#pragma unroll
                for (int m = 0; m < 4; ++m)
                  store_stream(at_byte(dm + (i * 4 + m) * stride, c * static_cast<uint32_t>(sizeof(TM))), g[i][1 + m]);
              }
            }
          }
        }
      }
      if (st < K) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          if (d_of[j] <= K - st) {
#pragma unroll
            for (int q = 0; q < 12; ++q) store_f32(&s_move[q][e_of[j]], mv[j][q]);
          }
        }
        __syncthreads();
      }
    }
  }
};

// K >= 3 steps of the moment-only storage (relaxation scheme, omega = 1) in
// one tile: the state is W (3 FP32 planes); the first step runs the stencil
// W(t+1, x) = sum_l f^eq_l(W(t, x - c_l)) from HBM over the tile plus a
// (K-1)-cell border into LDS (12 B per cell), the next K-2 steps run it inside
// LDS on regions one cell narrower per side (results staged in registers
// across a barrier, then written back over the same slots), and the last step
// writes the tile to HBM.  Every stage evaluates the same step_moments as the
// one- and two-step kernels, so the result equals K single steps bit for bit.
template <int TX, int TY, int NT, int K>
struct TileMomK {
  static_assert(K >= 3, "two steps per launch use the two-step tile");
  static constexpr int H = K - 1, EX = TX + 2 * H, EY = TY + 2 * H, EN = EX * EY;

  template <int LO>
  __device__ static void lds_stage(float (&s_w)[3][EN], const Coef& k) {
    constexpr int RX = EX - 2 * LO, RY = EY - 2 * LO, RN = RX * RY;
    constexpr int PER = (RN + NT - 1) / NT;
    float keep[PER][3];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = static_cast<int>(threadIdx.x) + j * NT;
      if (t < RN) {
        const int e = (LO + t / RX) * EX + LO + t % RX;
        const int off[4] = {-1, 1, -EX, EX};  // upwind neighbour of velocity +x, -x, +y, -y
        step_moments<2>([&](int i, int nb) { return s_w[i][nb < 0 ? e : e + off[nb]]; }, k, keep[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = static_cast<int>(threadIdx.x) + j * NT;
      if (t < RN) {
        const int e = (LO + t / RX) * EX + LO + t % RX;
#pragma unroll
        for (int i = 0; i < 3; ++i) s_w[i][e] = keep[j][i];
      }
    }
    __syncthreads();
    if constexpr (LO + 1 <= H - 1) lds_stage<LO + 1>(s_w, k);
  }

  __device__ static void run(const float* __restrict__ sr, float* __restrict__ dr, int x0, int y0, int nx, int ny,
                             int64_t stride, const Coef& k, float (&s_w)[3][EN]) {
    hbm_phase_begin();
    for (int e = threadIdx.x; e < EN; e += NT) {
      const int ex = e % EX, ey = e / EX;
      int x = x0 - H + ex, y = y0 - H + ey;
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
    hbm_phase_end();
    __syncthreads();
    lds_stage<1>(s_w, k);
    for (int t = threadIdx.x; t < TX * TY; t += NT) {
      const int tx = t % TX, ty = t / TX;
      const int x = x0 + tx, y = y0 + ty;
      if (x >= nx || y >= ny) continue;
      const int e = (ty + H) * EX + (tx + H);
      const int off[4] = {-1, 1, -EX, EX};
      float out[3];
      step_moments<2>([&](int i, int nb) { return s_w[i][nb < 0 ? e : e + off[nb]]; }, k, out);
      const int64_t c = static_cast<int64_t>(y) * nx + x;
#pragma unroll
      for (int i = 0; i < 3; ++i) store_stream(dr + i * stride + c, out[i]);
    }
  }
};

// K >= 3 steps of the split FP16 storage (W in FP32, scaled non-equilibrium
// parts n in FP16) in one tile.  The first step runs from HBM over the tile
// plus a (K-1)-cell border (rebuilding the upwind neighbours' equilibria) and
// keeps in LDS, as FP32, the populations that the stored values would stand
// for, f* = f^eq(W) + n / s with n rounded to FP16 (rest: f^eq_rest(W) -
// sum_m n_m / s): exactly what the next step's gather would rebuild from HBM.
// Each step inside LDS gathers those populations, relaxes, and rounds its
// result the same way before writing it back (staged in registers across a
// barrier), on regions one cell narrower per side; the last step writes W and
// the scaled FP16 parts of the tile to HBM.  The result equals K single steps
// bit for bit, and the upwind equilibria are rebuilt once per launch instead
// of once per step.
template <int TX, int TY, int NT, int K>
struct TileNeqK {
  static_assert(K >= 3, "two steps per launch use the two-step tile");
  static constexpr int H = K - 1, EX = TX + 2 * H, EY = TY + 2 * H, EN = EX * EY;

  // the populations a store of (W, n) and a reload would give
  __device__ static void stored_populations(const float (&W)[3], const float (&n)[3][4], const float (&eq)[3][5],
                                            const Coef& k, const NeqScale<2>& sc, float (&f)[15]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      float nr[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) nr[m] = static_cast<float>(static_cast<_Float16>(n[i][m] * sc.s[i]));
      const float s = ((nr[0] + nr[1]) + nr[2]) + nr[3];
      f[i * 5] = (W[i] - ((i == 0) ? k.d2a_rho : k.d2a_q) * W[i]) - s * sc.inv[i];
#pragma unroll
      for (int m = 0; m < 4; ++m) f[i * 5 + 1 + m] = eq[i][1 + m] + nr[m] * sc.inv[i];
    }
  }

  __device__ static void gather(const float (&s_f)[15][EN], int e, float (&g)[3][5]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[i][0] = s_f[i * 5][e];
      g[i][1] = s_f[i * 5 + 1][e - 1];   // +x from x-1
      g[i][2] = s_f[i * 5 + 2][e + 1];   // -x from x+1
      g[i][3] = s_f[i * 5 + 3][e - EX];  // +y from y-1
      g[i][4] = s_f[i * 5 + 4][e + EX];  // -y from y+1
    }
  }

  template <int LO>
  __device__ static void lds_stage(float (&s_f)[15][EN], const Coef& k, const NeqScale<2>& sc) {
    constexpr int RX = EX - 2 * LO, RY = EY - 2 * LO, RN = RX * RY;
    constexpr int PER = (RN + NT - 1) / NT;
    float keep[PER][15];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = static_cast<int>(threadIdx.x) + j * NT;
      if (t < RN) {
        const int e = (LO + t / RX) * EX + LO + t % RX;
        float g[3][5];
        gather(s_f, e, g);
        float W[3], n[3][4], eq[3][5];
        collide_neq<2>(g, k, W, n, eq);
        stored_populations(W, n, eq, k, sc, keep[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = static_cast<int>(threadIdx.x) + j * NT;
      if (t < RN) {
        const int e = (LO + t / RX) * EX + LO + t % RX;
#pragma unroll
        for (int q = 0; q < 15; ++q) s_f[q][e] = keep[j][q];
      }
    }
    __syncthreads();
    if constexpr (LO + 1 <= H - 1) lds_stage<LO + 1>(s_f, k, sc);
  }

  __device__ static void run(const float* __restrict__ sr, const neq16* __restrict__ sm, float* __restrict__ dr,
                             neq16* __restrict__ dm, int x0, int y0, int nx, int ny, int64_t stride, const Coef& k,
                             const NeqScale<2>& sc, float (&s_f)[15][EN]) {
    // (no raised priority here: this first step rebuilds the neighbours'
    // equilibria and is arithmetic-bound itself; with it, 117 against 130 GLUPS)
    for (int e = threadIdx.x; e < EN; e += NT) {
      const int ex = e % EX, ey = e / EX;
      int x = x0 - H + ex, y = y0 - H + ey;
      x = wrap_coord(x, nx);  // the border may wrap (several times on tiny grids)
      y = wrap_coord(y, ny);
      const int64_t c = static_cast<int64_t>(y) * nx + x;
      int64_t src[4];
      upwind_sources<2>(x, y, 0, nx, ny, 1, c, src);
      auto w_at = [&](int i, int nb) { return sr[i * stride + (nb < 0 ? c : src[nb])]; };
      auto n_at = [&](int i, int m, int nb) { return load_f32(sm + (i * 4 + m) * stride + (nb < 0 ? c : src[nb])); };
      float g[3][5];
      gather_neq<2>(w_at, n_at, k, sc, g);
      float W[3], n[3][4], eq[3][5], f[15];
      collide_neq<2>(g, k, W, n, eq);
      stored_populations(W, n, eq, k, sc, f);
#pragma unroll
      for (int q = 0; q < 15; ++q) s_f[q][e] = f[q];
    }
    __syncthreads();
    lds_stage<1>(s_f, k, sc);
    for (int t = threadIdx.x; t < TX * TY; t += NT) {
      const int tx = t % TX, ty = t / TX;
      const int x = x0 + tx, y = y0 + ty;
      if (x >= nx || y >= ny) continue;
      float g[3][5];
      gather(s_f, (ty + H) * EX + (tx + H), g);
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
};

}  // namespace lbm
