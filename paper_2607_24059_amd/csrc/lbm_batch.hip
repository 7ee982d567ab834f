// Batched engine: many independent runs, one persistent launch per step,
// replayed from a HIP graph (contract in include/lbm_batch.h).
//
// Work decomposition.  Every run is cut into tiles of exactly 256 cells:
// bx x (256 / bx) cells of one z-plane, with bx in {64, 128, 256} chosen per
// size class.  The tile list of the whole batch (runs in order, tiles of a run
// row-major) lives in device memory; a step is one launch of k_batch_step
// whose blocks walk the list with a static stride, so at any moment the
// resident blocks work on one contiguous stretch of it.  Each tile reads its
// run's descriptor (geometry, buffer offsets, coefficients) with scalar loads
// and updates its cells with the same step_cell as the single-run kernel.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_batch.h"
#include "lbm_device.hpp"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"

namespace lbm {
namespace {

constexpr int kTileCells = 256;
constexpr int kGraphSteps = 50;  // steps per replay of the main graph (even)

struct BatchRun {
  int32_t nx, ny, nz, pad;
  int64_t stride;
  int64_t rest_bytes;
  int64_t off[2];  // byte offsets of the two state buffers from the workspace base
  Coef k;
};

struct BatchTile {
  int32_t run;
  int32_t x0, y0;
  int16_t z;
  int16_t bx_log2;
};
static_assert(sizeof(BatchTile) == 16, "tile descriptor is 16 bytes");

template <int D, typename TR, typename TM>
__global__ __launch_bounds__(kTileCells) void k_batch_step(const BatchRun* __restrict__ runs,
                                                           const BatchTile* __restrict__ tiles,
                                                           int64_t ntiles, char* __restrict__ base,
                                                           int parity) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const BatchRun& r = runs[tl.run];
    const int bxl = tl.bx_log2;
    const int x = tl.x0 + (threadIdx.x & ((1 << bxl) - 1));
    const int y = tl.y0 + (threadIdx.x >> bxl);
    if (x < r.nx && y < r.ny) {
      char* src = base + r.off[parity];
      char* dst = base + r.off[parity ^ 1];
      const auto a = planes_of<TR, TM>(src, static_cast<size_t>(r.rest_bytes));
      const auto b = planes_of<TR, TM>(dst, static_cast<size_t>(r.rest_bytes));
      step_cell<D, TR, TM>(a.rest, a.move, b.rest, b.move, x, y, tl.z, r.nx, r.ny, r.nz, r.stride, r.k);
    }
  }
}

// Two steps per launch (2D): fused tiles of kT2X x kT2Y cells walked by a
// persistent grid; per tile the extended tile (one-cell border, periodic wrap
// in its run) is advanced one step into LDS in the storage types, then the
// tile by the second step from LDS, exactly as the single-run two-step kernel
// does, so the result equals two single steps bit for bit.
constexpr int kT2X = 64, kT2Y = 8, kT2N = 512;
constexpr int kFusedGraphLaunches = 24;  // fused launches per replay of the main graph (even)

template <typename TR, typename TM>
__global__ __launch_bounds__(kT2N) void k_batch_step2(const BatchRun* __restrict__ runs,
                                                      const BatchTile* __restrict__ tiles, int64_t ntiles,
                                                      char* __restrict__ base, int parity) {
  constexpr int EX = kT2X + 2, EY = kT2Y + 2, EN = EX * EY;
  __shared__ TR s_rest[3][EN];
  __shared__ TM s_move[12][EN];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const BatchRun& r = runs[tl.run];
    const int nx = r.nx, ny = r.ny;
    const int64_t stride = r.stride;
    const auto a = planes_of<TR, TM>(base + r.off[parity], static_cast<size_t>(r.rest_bytes));
    const auto b = planes_of<TR, TM>(base + r.off[parity ^ 1], static_cast<size_t>(r.rest_bytes));
    hbm_phase_begin();  // raised priority over the HBM phase (the 575-run sweep: 73.0 vs 75.1 ms)
    for (int e = threadIdx.x; e < EN; e += kT2N) {
      const int ex = e % EX, ey = e / EX;
      int x = tl.x0 - 1 + ex, y = tl.y0 - 1 + ey;
      x = wrap_coord(x, nx);  // the border may wrap (several times on tiny runs)
      y = wrap_coord(y, ny);
      const int64_t c = static_cast<int64_t>(y) * nx + x;
      float g[3][5];
      gather_cell<2, TR, TM>(a.rest, a.move, x, y, 0, nx, ny, 1, stride, c, g);
      collide<2>(g, r.k);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        store_f32(&s_rest[i][e], g[i][0]);
#pragma unroll
        for (int m = 0; m < 4; ++m) store_f32(&s_move[i * 4 + m][e], g[i][1 + m]);
      }
    }
    hbm_phase_end();
    __syncthreads();
    for (int q = threadIdx.x; q < kT2X * kT2Y; q += kT2N) {
      const int tx = q % kT2X, ty = q / kT2X;
      const int x = tl.x0 + tx, y = tl.y0 + ty;
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
      collide<2>(g, r.k);
      const int64_t c = static_cast<int64_t>(y) * nx + x;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        store_stream(b.rest + i * stride + c, g[i][0]);
#pragma unroll
        for (int m = 0; m < 4; ++m) store_stream(b.move + (i * 4 + m) * stride + c, g[i][1 + m]);
      }
    }
    __syncthreads();  // the next tile overwrites the LDS tile
  }
}

// K steps per launch (2D): the single-run engine's multi-step tiles
// (lbm_fused.hpp) walked by a persistent grid, each tile wrapping periodically
// in its own run, so again bit-identical to single steps.  Three tile shapes
// per storage; lbm_batch_autotune picks one per size class (the tiles of each
// shape are one launch of that shape's kernel, and the launches of one fused
// step are independent graph nodes).  K is 5, or 6 for the 4-byte storages
// where most cells belong to large runs (batch_depth).
constexpr int kShapes = 3;

template <typename TR, typename TM, int S, int K>
struct BatchKShape {
  static constexpr bool kRegs = sizeof(TR) == 4 && sizeof(TM) == 4;
  // 4-byte planes, rest populations in registers: 32x32 on 768 threads (the
  // single-run engine's tile, two blocks per compute unit; the 512-run batch
  // 178.8 against 170.7 GLUPS on 512 threads), 32x16 on 256 (three blocks per
  // compute unit), 16x16 on 256 (small runs: more tiles); 16-bit planes:
  // 64x16 on 512 (on 768 threads, the single-run engine's choice with FP32
  // rest planes, the 512-run FP16 + FP32 rest batch ran 183.0 against 199.6),
  // 32x32 on 512, 32x16 on 256.  At six steps the first 4-byte shape is the
  // single-run engine's 32x28 (its 42x38 extended tile keeps two blocks per
  // compute unit).
  static constexpr int TX = kRegs ? (S == 2 ? 16 : 32) : (S == 0 ? 64 : 32);
  static constexpr int TY = kRegs ? (S == 0 ? (K == 6 ? 28 : 32) : 16) : (S == 1 ? 32 : 16);
  static constexpr int NT = kRegs ? (S == 0 ? 768 : 256) : (S == 2 ? 256 : 512);
};
constexpr int kTKXmin = 16, kTKYmin = 16;  // smallest tile width and height (size the tile list)

template <typename TR, typename TM, int S, int K>
__global__ __launch_bounds__((BatchKShape<TR, TM, S, K>::NT)) void k_batch_stepK(const BatchRun* __restrict__ runs,
                                                                            const BatchTile* __restrict__ tiles,
                                                                            int64_t ntiles, char* __restrict__ base,
                                                                            int parity) {
  using SH = BatchKShape<TR, TM, S, K>;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const BatchRun& r = runs[tl.run];
    const auto a = planes_of<TR, TM>(base + r.off[parity], static_cast<size_t>(r.rest_bytes));
    const auto b = planes_of<TR, TM>(base + r.off[parity ^ 1], static_cast<size_t>(r.rest_bytes));
    if constexpr (SH::kRegs) {
      using T = TileKr<TR, TM, SH::TX, SH::TY, SH::NT, K>;
      __shared__ TM s_move[12][T::EN];
      T::run(a.rest, a.move, b.rest, b.move, tl.x0, tl.y0, r.nx, r.ny, r.stride, r.k, s_move);
    } else {
      using T = TileK<TR, TM, SH::TX, SH::TY, SH::NT, K>;
      __shared__ TR s_rest[3][T::EN];
      __shared__ TM s_move[12][T::EN];
      T::run(a.rest, a.move, b.rest, b.move, tl.x0, tl.y0, r.nx, r.ny, r.stride, r.k, s_rest, s_move);
    }
    __syncthreads();  // the next tile overwrites the LDS tile
  }
}

using BatchKernel = void (*)(const BatchRun*, const BatchTile*, int64_t, char*, int);

struct BatchKKernel {
  BatchKernel fn = nullptr;
  int tx = 0, ty = 0, threads = 0, depth = 0;
};

template <typename TR, typename TM, int S, int K>
BatchKKernel batch_k_shape() {
  using SH = BatchKShape<TR, TM, S, K>;
  return BatchKKernel{&k_batch_stepK<TR, TM, S, K>, SH::TX, SH::TY, SH::NT, K};
}

template <typename TR, typename TM, int K>
void batch_k_of(BatchKKernel (&out)[kShapes]) {
  out[0] = batch_k_shape<TR, TM, 0, K>();
  out[1] = batch_k_shape<TR, TM, 1, K>();
  out[2] = batch_k_shape<TR, TM, 2, K>();
}

// Steps per launch of a batch's multi-step kernel.  As in the single-run
// engine, six for the 4-byte storages where at least half of the cells belong
// to runs of 2^20 cells or more, else five: small runs (the 575 runs of 75^2
// of the parameter sweeps) keep the narrower border, and the 16-bit storages
// lost with six on the 512-run workload (FP16 + FP32 rest 189.4 against
// 199.2, BF16 195.0 against 205.7 GLUPS).
int batch_depth(int dim, int storage, int nruns, const lbm_run_spec* runs) {
  if (dim != 2 || (storage != LBM_F32 && storage != LBM_F32_RAW)) return 5;
  int64_t big = 0, all = 0;
  for (int r = 0; r < nruns; ++r) {
    const int64_t c = runs[r].n[0] * runs[r].n[1];
    all += c;
    if (c >= (int64_t(1) << 20)) big += c;
  }
  return 2 * big >= all && all > 0 ? 6 : 5;
}

// the multi-step kernels of a storage at `depth` steps per launch (all null
// where there are none)
void batch_kernelK(int dim, int storage, int depth, BatchKKernel (&out)[kShapes]) {
  for (auto& k : out) k = BatchKKernel{};
  if (dim != 2) return;
  switch (storage) {
    case LBM_F32: case LBM_F32_RAW:
      if (depth == 6) batch_k_of<float, float, 6>(out);
      else batch_k_of<float, float, 5>(out);
      return;
    case LBM_F16_DEV: batch_k_of<_Float16, _Float16, 5>(out); return;
    case LBM_BF16_DEV: batch_k_of<bf16, bf16, 5>(out); return;
    case LBM_F16_DEV_R32: batch_k_of<float, _Float16, 5>(out); return;
    case LBM_BF16_DEV_R32: batch_k_of<float, bf16, 5>(out); return;
  }
}

// multi-step tiles of one 2D run for a tx x ty tile (at most this many for any
// tile of at least kTKXmin x kTKYmin cells)
int64_t tilesK_of(const Geometry& g, int tx, int ty) {
  return static_cast<int64_t>((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
}

BatchKernel batch_kernel2(int dim, int storage) {
  if (dim != 2) return nullptr;
  switch (storage) {
    case LBM_F32: case LBM_F32_RAW: return &k_batch_step2<float, float>;
    case LBM_F16_DEV: return &k_batch_step2<_Float16, _Float16>;
    case LBM_BF16_DEV: return &k_batch_step2<bf16, bf16>;
    case LBM_F16_DEV_R32: return &k_batch_step2<float, _Float16>;
    case LBM_BF16_DEV_R32: return &k_batch_step2<float, bf16>;
  }
  return nullptr;
}

// fused tiles of one 2D run
int64_t tiles2_of(const Geometry& g) {
  return static_cast<int64_t>((g.nx + kT2X - 1) / kT2X) * ((g.ny + kT2Y - 1) / kT2Y);
}

BatchKernel batch_kernel(int dim, int storage) {
  if (dim == 2) {
    switch (storage) {
      case LBM_F32: case LBM_F32_RAW: return &k_batch_step<2, float, float>;
      case LBM_F16_DEV: return &k_batch_step<2, _Float16, _Float16>;
      case LBM_BF16_DEV: return &k_batch_step<2, bf16, bf16>;
      case LBM_F16_DEV_R32: return &k_batch_step<2, float, _Float16>;
      case LBM_BF16_DEV_R32: return &k_batch_step<2, float, bf16>;
    }
  } else if (dim == 3) {
    switch (storage) {
      case LBM_F32: case LBM_F32_RAW: return &k_batch_step<3, float, float>;
      case LBM_F16_DEV: return &k_batch_step<3, _Float16, _Float16>;
      case LBM_BF16_DEV: return &k_batch_step<3, bf16, bf16>;
      case LBM_F16_DEV_R32: return &k_batch_step<3, float, _Float16>;
      case LBM_BF16_DEV_R32: return &k_batch_step<3, float, bf16>;
    }
  }
  return nullptr;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

int pow2_class(int64_t nx) {
  int64_t c = 1;
  while (c < nx) c <<= 1;
  return static_cast<int>(c);
}

// tiles of one run for tile width bx
int64_t tiles_of(const Geometry& g, int bx) {
  const int by = kTileCells / bx;
  return static_cast<int64_t>((g.nx + bx - 1) / bx) * ((g.ny + by - 1) / by) * g.nz;
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace
}  // namespace lbm

using namespace lbm;

struct lbm_batch {
  int dim = 0, storage = 0, nruns = 0;
  std::vector<lbm_run_spec> specs;
  std::vector<Geometry> geo;
  std::vector<RunCoef> coef;
  std::vector<int64_t> off0, off1;
  std::vector<int> cls;           // size class (pow2 of nx) of each run
  std::map<int, int> bx_of_class; // tile width per class
  char* ws = nullptr;
  size_t ws_bytes = 0;
  BatchRun* d_runs = nullptr;
  BatchTile* d_tiles = nullptr;
  int64_t max_tiles = 0;
  int64_t ntiles = 0;
  BatchTile* d_tiles2 = nullptr;  // fused (two-step) tiles, 2D only
  int64_t ntiles2 = 0;
  int grid2 = 0;                  // persistent grid of the fused kernel
  int fuse = 1;                   // steps per launch: 1, 2 (two-step kernel) or kdepth
  int kdepth = 0;                 // steps per launch of the multi-step kernel (0: none)
  BatchKernel kernel2 = nullptr;
  BatchKKernel kernelK[kShapes];  // kdepth steps per launch (2D population storages), per tile shape
  std::map<int, int> shape_of_class;  // fused tile shape per size class
  BatchTile* d_tilesK = nullptr;
  int64_t ntilesK = 0;
  int64_t startK[kShapes] = {0, 0, 0}, countK[kShapes] = {0, 0, 0};  // tile ranges of the shapes
  int gridK = 0;                  // blocks per CU of each multi-step launch (0: one per tile)
  hipGraphExec_t exec_mainK[2] = {nullptr, nullptr};  // kFusedGraphLaunches K-step launches from parity p
  hipGraphExec_t exec_oneK[2] = {nullptr, nullptr};   // one K-step launch from parity p
  hipGraphExec_t exec_main2[2] = {nullptr, nullptr};  // kFusedGraphLaunches fused launches from parity p
  hipGraphExec_t exec_two[2] = {nullptr, nullptr};    // one fused launch from parity p
  int64_t total_cells = 0;
  int parity = 0;  // state buffer index holding the current step
  int grid = 0;    // persistent grid size (blocks); >= ntiles means one block per tile
  int cus = 256;   // compute units of the device
  hipStream_t stream = nullptr;
  BatchKernel kernel = nullptr;
  hipGraphExec_t exec_main = nullptr;  // kGraphSteps steps starting at parity 0
  hipGraphExec_t exec_one[2] = {nullptr, nullptr};
  int64_t steps = 0;
};

namespace {

lbm_params params_of(int dim, int storage, const lbm_run_spec& r) {
  lbm_params p;
  p.dim = dim;
  p.storage = storage;
  for (int a = 0; a < 3; ++a) p.n[a] = r.n[a];
  p.dx = r.dx;
  p.dt = r.dt;
  p.nu = r.nu;
  p.omega_rho = r.omega_rho;
  p.omega_q = r.omega_q;
  p.alpha_rho = r.alpha_rho;
  p.gamma = 1.0;
  p.rho_ref = r.rho_ref;
  return p;
}

int default_bx(const Geometry& g) {
  int bx = 256;
  while (bx > 64 && bx / 2 >= g.nx) bx /= 2;
  return bx;
}

struct Layout {
  size_t runs_off, tiles_off, tiles2_off, tilesK_off, bufs_off, total;
  int64_t max_tiles, tiles2, tilesK;
  std::vector<int64_t> off0, off1;
};

Layout layout(int dim, int storage, int nruns, const lbm_run_spec* runs) {
  Layout L;
  L.max_tiles = 0;
  L.tiles2 = 0;
  L.tilesK = 0;
  std::vector<Geometry> geo;
  for (int r = 0; r < nruns; ++r) {
    const Geometry g = make_geometry(dim, storage, runs[r].n);
    int64_t mt = 0;
    for (int bx = 64; bx <= 256; bx *= 2) mt = std::max(mt, tiles_of(g, bx));
    L.max_tiles += mt;
    if (dim == 2) {
      L.tiles2 += tiles2_of(g);
      L.tilesK += tilesK_of(g, kTKXmin, kTKYmin);
    }
    geo.push_back(g);
  }
  L.runs_off = 0;
  L.tiles_off = align256(sizeof(BatchRun) * nruns);
  L.tiles2_off = align256(L.tiles_off + sizeof(BatchTile) * L.max_tiles);
  L.tilesK_off = align256(L.tiles2_off + sizeof(BatchTile) * L.tiles2);
  L.bufs_off = align256(L.tilesK_off + sizeof(BatchTile) * L.tilesK);
  size_t off = L.bufs_off;
  for (int r = 0; r < nruns; ++r) {
    L.off0.push_back(static_cast<int64_t>(off));
    off += geo[r].buf_bytes;
    L.off1.push_back(static_cast<int64_t>(off));
    off += geo[r].buf_bytes;
  }
  L.total = off;
  return L;
}

lbm_status dev(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

// Build the host tile list for the runs selected by `use` (all if empty).
std::vector<BatchTile> build_tiles(const lbm_batch* b, const std::vector<char>& use) {
  std::vector<BatchTile> t;
  for (int r = 0; r < b->nruns; ++r) {
    if (!use.empty() && !use[r]) continue;
    const Geometry& g = b->geo[r];
    const int bx = b->bx_of_class.at(b->cls[r]);
    const int by = kTileCells / bx;
    const int16_t bl = static_cast<int16_t>(log2i(bx));
    for (int z = 0; z < g.nz; ++z)
      for (int y0 = 0; y0 < g.ny; y0 += by)
        for (int x0 = 0; x0 < g.nx; x0 += bx) t.push_back(BatchTile{r, x0, y0, static_cast<int16_t>(z), bl});
  }
  return t;
}

hipError_t upload_tiles(lbm_batch* b, const std::vector<BatchTile>& t) {
  if (static_cast<int64_t>(t.size()) > b->max_tiles) return hipErrorInvalidValue;
  b->ntiles = static_cast<int64_t>(t.size());
  if (t.empty()) return hipSuccess;
  hipError_t e = hipMemcpyAsync(b->d_tiles, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e;
}

hipError_t launch_step(lbm_batch* b, int parity, int64_t ntiles, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(ntiles, b->grid));
  hipLaunchKernelGGL(b->kernel, dim3(grid), dim3(kTileCells), 0, s, b->d_runs, b->d_tiles, ntiles, b->ws,
                     parity);
  return hipGetLastError();
}

hipError_t launch_step2(lbm_batch* b, int parity, hipStream_t s) {
  if (b->ntiles2 == 0) return hipSuccess;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(b->ntiles2, b->grid2));
  hipLaunchKernelGGL(b->kernel2, dim3(grid), dim3(kT2N), 0, s, b->d_runs, b->d_tiles2, b->ntiles2, b->ws, parity);
  return hipGetLastError();
}

// blocks of a multi-step launch over n tiles
unsigned gridK_for(const lbm_batch* b, int64_t n) {
  const int64_t cap = b->gridK > 0 ? static_cast<int64_t>(b->gridK) * b->cus : n;
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(n, std::min<int64_t>(cap, 0x7fffffff))));
}

void destroy_graphs(lbm_batch* b) {
  auto drop = [](hipGraphExec_t& e) {
    if (e) hipGraphExecDestroy(e);
    e = nullptr;
  };
  drop(b->exec_main);
  for (int p = 0; p < 2; ++p) {
    drop(b->exec_one[p]);
    drop(b->exec_main2[p]);
    drop(b->exec_two[p]);
    drop(b->exec_mainK[p]);
    drop(b->exec_oneK[p]);
  }
}

// A graph of `count` consecutive launches of `kernel` starting at `parity`
// (each launch flips the buffer parity): a chain of kernel nodes, no memset
// or copy nodes.
hipError_t make_graph(lbm_batch* b, BatchKernel kernel, const BatchTile* tiles, int64_t ntiles, int grid_max,
                      int threads, int parity, int count, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>(ntiles, 1), grid_max));
  for (int s = 0; s < count && e == hipSuccess; ++s) {
    int par = (parity + s) & 1;
    const BatchRun* runs = b->d_runs;
    int64_t nt = ntiles;
    char* base = b->ws;
    void* args[] = {&runs, &tiles, &nt, &base, &par};
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = reinterpret_cast<void*>(kernel);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(threads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}

// A graph of `count` consecutive multi-step launches starting at `parity`:
// each launch is one kernel node per tile shape in use (independent of each
// other), each depending on every node of the previous launch.
hipError_t make_graphK(lbm_batch* b, int parity, int count, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  std::vector<hipGraphNode_t> prev, cur;
  for (int l = 0; l < count && e == hipSuccess; ++l) {
    cur.clear();
    for (int sh = 0; sh < kShapes && e == hipSuccess; ++sh) {
      if (b->countK[sh] == 0) continue;
      int par = (parity + l) & 1;
      const BatchRun* runs = b->d_runs;
      const BatchTile* tiles = b->d_tilesK + b->startK[sh];
      int64_t nt = b->countK[sh];
      char* base = b->ws;
      void* args[] = {&runs, &tiles, &nt, &base, &par};
      hipKernelNodeParams kp;
      memset(&kp, 0, sizeof(kp));
      kp.func = reinterpret_cast<void*>(b->kernelK[sh].fn);
      kp.gridDim = dim3(gridK_for(b, nt));
      kp.blockDim = dim3(b->kernelK[sh].threads);
      kp.sharedMemBytes = 0;
      kp.kernelParams = args;
      kp.extra = nullptr;
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, g, prev.empty() ? nullptr : prev.data(), prev.size(), &kp);
      cur.push_back(node);
    }
    prev.swap(cur);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return e;
}

hipError_t rebuild(lbm_batch* b) {
  destroy_graphs(b);
  hipError_t e = upload_tiles(b, build_tiles(b, {}));
  const BatchTile* t1 = b->d_tiles;
  if (e == hipSuccess) e = make_graph(b, b->kernel, t1, b->ntiles, b->grid, kTileCells, 0, kGraphSteps, &b->exec_main);
  for (int p = 0; p < 2 && e == hipSuccess; ++p)
    e = make_graph(b, b->kernel, t1, b->ntiles, b->grid, kTileCells, p, 1, &b->exec_one[p]);
  if (b->kernel2) {
    for (int p = 0; p < 2 && e == hipSuccess; ++p) {
      e = make_graph(b, b->kernel2, b->d_tiles2, b->ntiles2, b->grid2, kT2N, p, kFusedGraphLaunches,
                     &b->exec_main2[p]);
      if (e == hipSuccess) e = make_graph(b, b->kernel2, b->d_tiles2, b->ntiles2, b->grid2, kT2N, p, 1, &b->exec_two[p]);
    }
  }
  if (b->kernelK[0].fn && b->ntilesK > 0) {
    for (int p = 0; p < 2 && e == hipSuccess; ++p) {
      e = make_graphK(b, p, kFusedGraphLaunches, &b->exec_mainK[p]);
      if (e == hipSuccess) e = make_graphK(b, p, 1, &b->exec_oneK[p]);
    }
  }
  return e;
}

// The multi-step tile list of the runs selected by `use` (all if empty): the
// tiles of each shape in one contiguous range, each range in XCD-major order
// (xcd_major: list slot s is taken by a block on XCD s % 8, with one block per
// tile or a persistent grid that is a multiple of 8, so neighbouring tiles
// share their border reads through one L2; a range whose length is not a
// multiple of 8 in raster order ran 5.07 against 4.12 ms per five-step launch
// of the 512-run FP32 batch).
hipError_t upload_tilesK(lbm_batch* b, const std::vector<char>& use = {}) {
  std::vector<BatchTile> all;
  for (int sh = 0; sh < kShapes; ++sh) {
    std::vector<BatchTile> t;
    const int tx = b->kernelK[sh].tx, ty = b->kernelK[sh].ty;
    for (int r = 0; r < b->nruns; ++r) {
      if ((!use.empty() && !use[r]) || b->shape_of_class.at(b->cls[r]) != sh) continue;
      const Geometry& g = b->geo[r];
      for (int y0 = 0; y0 < g.ny; y0 += ty)
        for (int x0 = 0; x0 < g.nx; x0 += tx) t.push_back(BatchTile{r, x0, y0, 0, static_cast<int16_t>(log2i(tx))});
    }
    const size_t n = t.size();
    b->startK[sh] = static_cast<int64_t>(all.size());
    b->countK[sh] = static_cast<int64_t>(n);
    for (size_t q = 0; q < n; ++q) all.push_back(t[xcd_major(static_cast<int64_t>(q), static_cast<int64_t>(n))]);
  }
  b->ntilesK = static_cast<int64_t>(all.size());
  if (all.empty()) return hipSuccess;
  hipError_t e = hipMemcpyAsync(b->d_tilesK, all.data(), all.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e;
}

// The fused tile list (fixed: it does not depend on the tuned tile widths).
hipError_t upload_tiles2(lbm_batch* b) {
  std::vector<BatchTile> t;
  for (int r = 0; r < b->nruns; ++r) {
    const Geometry& g = b->geo[r];
    for (int y0 = 0; y0 < g.ny; y0 += kT2Y)
      for (int x0 = 0; x0 < g.nx; x0 += kT2X) t.push_back(BatchTile{r, x0, y0, 0, static_cast<int16_t>(log2i(kT2X))});
  }
  b->ntiles2 = static_cast<int64_t>(t.size());
  if (t.empty()) return hipSuccess;
  hipError_t e = hipMemcpyAsync(b->d_tiles2, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e;
}

std::string device_key() {
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string k = prop.gcnArchName;
  for (auto& ch : k)
    if (ch == ' ' || ch == ':') ch = '_';
  return k;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t dim, int32_t storage, int32_t nruns, const lbm_run_spec* runs) {
  if (nruns <= 0 || !runs || !batch_kernel(dim, storage)) return 0;
  for (int r = 0; r < nruns; ++r) {
    lbm_params p = params_of(dim, storage, runs[r]);
    if (lbm_check_params(&p, nullptr, nullptr, nullptr) != LBM_OK) return 0;
  }
  return layout(dim, storage, nruns, runs).total;
}

lbm_status lbm_batch_init(lbm_batch** out, int32_t dim, int32_t storage, int32_t nruns,
                          const lbm_run_spec* runs, const double* const* u0, const double* const* rho0,
                          void* workspace, size_t ws_bytes, void* hip_stream, int32_t* bad_run) {
  if (!out || !runs || !u0 || !workspace || nruns <= 0) return LBM_EINVAL;
  *out = nullptr;
  if (!batch_kernel(dim, storage)) return LBM_EINVAL;  // no batched FP64 reference mode
  if (bad_run) *bad_run = -1;
  std::vector<RunCoef> coefs;
  for (int r = 0; r < nruns; ++r) {
    lbm_params p = params_of(dim, storage, runs[r]);
    double mu = 0, aq = 0;
    lbm_status st = lbm_check_params(&p, &mu, &aq, nullptr);
    if (st == LBM_OK && (!u0[r] || runs[r].n[2] > 32767)) st = LBM_EINVAL;  // tile z is 16-bit
    // the multi-step tiles address a plane with 32-bit byte offsets
    if (st == LBM_OK && dim == 2 && !fused_offsets_fit(runs[r].n[0] * runs[r].n[1], 4)) st = LBM_EINVAL;
    if (st != LBM_OK) {
      if (bad_run) *bad_run = r;
      return st;
    }
    coefs.push_back(RunCoef{runs[r].dx, mu, runs[r].alpha_rho, aq, runs[r].omega_rho, runs[r].omega_q,
                            runs[r].rho_ref});
  }
  const Layout L = layout(dim, storage, nruns, runs);
  if (ws_bytes < L.total) return LBM_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return LBM_EINVAL;

  lbm_batch* b = new (std::nothrow) lbm_batch;
  if (!b) return LBM_ENOMEM;
  b->dim = dim;
  b->storage = storage;
  b->nruns = nruns;
  b->specs.assign(runs, runs + nruns);
  b->coef = coefs;
  b->off0 = L.off0;
  b->off1 = L.off1;
  b->ws = static_cast<char*>(workspace);
  b->ws_bytes = ws_bytes;
  b->d_runs = reinterpret_cast<BatchRun*>(b->ws + L.runs_off);
  b->d_tiles = reinterpret_cast<BatchTile*>(b->ws + L.tiles_off);
  b->d_tiles2 = reinterpret_cast<BatchTile*>(b->ws + L.tiles2_off);
  b->d_tilesK = reinterpret_cast<BatchTile*>(b->ws + L.tilesK_off);
  b->max_tiles = L.max_tiles;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->kernel = batch_kernel(dim, storage);
  b->kernel2 = batch_kernel2(dim, storage);
  batch_kernelK(dim, storage, batch_depth(dim, storage, nruns, runs), b->kernelK);
  b->kdepth = b->kernelK[0].fn ? b->kernelK[0].depth : 0;
  b->fuse = b->kdepth ? b->kdepth : b->kernel2 ? 2 : 1;
  const Ops* ops = ops_for(dim, storage);
  const bool devn = storage_is_deviation(storage);

  std::vector<BatchRun> host_runs(nruns);
  hipError_t e = hipSuccess;
  for (int r = 0; r < nruns && e == hipSuccess; ++r) {
    const Geometry g = make_geometry(dim, storage, runs[r].n);
    b->geo.push_back(g);
    b->total_cells += g.cells;
    b->cls.push_back(pow2_class(g.nx));
    if (!b->bx_of_class.count(b->cls.back())) b->bx_of_class[b->cls.back()] = default_bx(g);
    b->shape_of_class[b->cls.back()] = 0;
    BatchRun& d = host_runs[r];
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.pad = 0;
    d.stride = g.stride;
    d.rest_bytes = static_cast<int64_t>(g.rest_bytes);
    d.off[0] = L.off0[r];
    d.off[1] = L.off1[r];
    d.k = make_coef<float>(coefs[r], dim, devn);
    // stage the initial fields in buffer 1 of the run, build the equilibrium in buffer 0
    double* su = reinterpret_cast<double*>(b->ws + L.off1[r]);
    double* sr = (rho0 && rho0[r]) ? su + static_cast<size_t>(dim) * g.cells : nullptr;
    e = hipMemcpyAsync(su, u0[r], static_cast<size_t>(dim) * g.cells * sizeof(double), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess && sr)
      e = hipMemcpyAsync(sr, rho0[r], static_cast<size_t>(g.cells) * sizeof(double), hipMemcpyHostToDevice,
                         b->stream);
    if (e == hipSuccess) e = ops->init(g, coefs[r], su, sr, b->ws + L.off0[r], b->stream);
    // pageable host copies: keep the staging buffer alive until it has been consumed
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_runs, host_runs.data(), sizeof(BatchRun) * nruns, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) {
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    b->cus = cus;
    b->grid = 8 * cus;  // 8 resident 256-thread blocks per CU at the kernel's register use
    b->grid2 = 2 * cus;  // two resident 512-thread fused blocks per CU (LDS tile of up to 40 KB)
    // one block per tile in each multi-step launch: the launch's per-shape
    // graph nodes run concurrently, and a persistent grid sized for the whole
    // chip then waits for the compute units the other node holds (2 blocks per
    // CU: 96 against 170 GLUPS for the 512-run FP32 batch)
    b->gridK = 0;
    if (b->kernel2) e = upload_tiles2(b);
    if (e == hipSuccess && b->kernelK[0].fn) e = upload_tilesK(b);
    if (e == hipSuccess) e = rebuild(b);
  }
  if (e != hipSuccess) {
    destroy_graphs(b);
    delete b;
    return LBM_EDEVICE;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, const char* cache_path) {
  if (!b) return LBM_EINVAL;
  if (!cache_path) cache_path = getenv("LBM_AUTOTUNE_CACHE");
  const std::string key = device_key();
  std::map<int, int> cached;
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char arch[128];
      int d, st, cl, bx;
      while (fscanf(f, "%127s %d %d %d %d", arch, &d, &st, &cl, &bx) == 5)
        if (key == arch && d == b->dim && st == b->storage && (cl < 0 || bx == 64 || bx == 128 || bx == 256))
          cached[cl] = bx;  // cl >= 0: one-step tile width; -1, -2: grids; -(1000 + cl): fused shape
      fclose(f);
    }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LBM_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return LBM_EDEVICE;
  }
  hipError_t e = hipSuccess;
  std::vector<std::pair<int, int>> fresh;
  for (auto& kv : b->bx_of_class) {
    const int cl = kv.first;
    if (cached.count(cl)) {
      kv.second = cached[cl];
      continue;
    }
    std::vector<char> use(b->nruns, 0);
    for (int r = 0; r < b->nruns; ++r) use[r] = (b->cls[r] == cl);
    float best = 1e30f;
    int best_bx = kv.second;
    for (int bx = 64; bx <= 256 && e == hipSuccess; bx *= 2) {
      if (bx > 64 && bx > cl) break;  // tiles wider than the class waste lanes
      kv.second = bx;
      const std::vector<BatchTile> t = build_tiles(b, use);
      e = upload_tiles(b, t);
      // a step only writes the idle buffer, so timing it leaves the state intact
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_step(b, b->parity, b->ntiles, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (int it = 0; it < 5 && e == hipSuccess; ++it) e = launch_step(b, b->parity, b->ntiles, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_bx = bx;
      }
    }
    kv.second = best_bx;
    fresh.emplace_back(cl, best_bx);
  }
  // persistent grid size for the whole list: blocks per CU, or one block per tile (0)
  if (e == hipSuccess) e = upload_tiles(b, build_tiles(b, {}));
  if (e == hipSuccess && cached.count(-1)) {
    const int per_cu = cached[-1];
    b->grid = per_cu > 0 ? per_cu * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles, 0x7fffffff));
  } else if (e == hipSuccess) {
    const int cands[] = {4, 8, 16, 32, 0};
    float best = 1e30f;
    int best_pc = 8;
    for (int pc : cands) {
      if (e != hipSuccess) break;
      b->grid = pc > 0 ? pc * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles, 0x7fffffff));
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_step(b, b->parity, b->ntiles, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (int it = 0; it < 5 && e == hipSuccess; ++it) e = launch_step(b, b->parity, b->ntiles, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_pc = pc;
      }
    }
    b->grid = best_pc > 0 ? best_pc * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles, 0x7fffffff));
    fresh.emplace_back(-1, best_pc);
  }
  // persistent grid of the fused kernel (class -2): blocks per CU, or one block per tile (0)
  if (e == hipSuccess && b->kernel2 && cached.count(-2)) {
    const int per_cu = cached[-2];
    b->grid2 = per_cu > 0 ? per_cu * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles2, 0x7fffffff));
  } else if (e == hipSuccess && b->kernel2) {
    const int cands[] = {1, 2, 4, 8, 0};
    float best = 1e30f;
    int best_pc = 2;
    for (int pc : cands) {
      if (e != hipSuccess) break;
      b->grid2 = pc > 0 ? pc * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles2, 0x7fffffff));
      // a fused launch reads the current buffer and writes the other: the state is kept
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_step2(b, b->parity, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (int it = 0; it < 5 && e == hipSuccess; ++it) e = launch_step2(b, b->parity, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_pc = pc;
      }
    }
    b->grid2 = best_pc > 0 ? best_pc * b->cus : static_cast<int>(std::min<int64_t>(b->ntiles2, 0x7fffffff));
    fresh.emplace_back(-2, best_pc);
  }
  // fused tile shape of every size class (cache key -(1000 + class)): each
  // candidate timed on the class's runs alone, one block per tile
  // each candidate is timed as the steps run: replays of a one-launch graph
  // whose per-shape nodes may overlap (timing plain launches in stream order
  // ranked persistent grids first that lose when the nodes overlap); every
  // replay reads the current buffer and writes the other: the state is kept
  auto time_K = [&](float* ms) {
    hipGraphExec_t g = nullptr;
    if (e == hipSuccess) e = make_graphK(b, b->parity, 1, &g);
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = hipGraphLaunch(g, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int it = 0; it < 6 && e == hipSuccess; ++it) e = hipGraphLaunch(g, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (g) {
      hipStreamSynchronize(b->stream);
      hipGraphExecDestroy(g);
    }
  };
  if (e == hipSuccess && b->kernelK[0].fn) {
    const int grid_keep = b->gridK;
    b->gridK = 0;
    for (auto& kv : b->shape_of_class) {
      const int cl = kv.first, key = -(1000 + cl);
      if (cached.count(key) && cached[key] >= 0 && cached[key] < kShapes) {
        kv.second = cached[key];
        continue;
      }
      std::vector<char> use(b->nruns, 0);
      for (int r = 0; r < b->nruns; ++r) use[r] = (b->cls[r] == cl);
      float best = 1e30f;
      int best_sh = kv.second;
      for (int sh = 0; sh < kShapes && e == hipSuccess; ++sh) {
        kv.second = sh;
        e = upload_tilesK(b, use);
        float ms = 0;
        time_K(&ms);
        if (e == hipSuccess && ms < best) {
          best = ms;
          best_sh = sh;
        }
      }
      kv.second = best_sh;
      fresh.emplace_back(key, best_sh);
    }
    b->gridK = grid_keep;
    if (e == hipSuccess) e = upload_tilesK(b);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e == hipSuccess) e = rebuild(b);
  if (e != hipSuccess) return LBM_EDEVICE;
  if (cache_path && !fresh.empty()) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      for (auto& p : fresh) fprintf(f, "%s %d %d %d %d\n", key.c_str(), b->dim, b->storage, p.first, p.second);
      fclose(f);
    }
  }
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  hipError_t e = hipSuccess;
  if (b->kdepth && b->fuse == b->kdepth) {
    // multi-step launches, then two-step and single-step ones for the remainder
    while (nsteps > 0 && e == hipSuccess) {
      int adv = 1, flip = 1;
      if (nsteps >= b->kdepth * kFusedGraphLaunches) {
        e = hipGraphLaunch(b->exec_mainK[b->parity], b->stream);  // even launch count: parity kept
        adv = b->kdepth * kFusedGraphLaunches;
        flip = 0;
      } else if (nsteps >= b->kdepth) {
        e = hipGraphLaunch(b->exec_oneK[b->parity], b->stream);
        adv = b->kdepth;
      } else if (nsteps >= 2) {
        e = hipGraphLaunch(b->exec_two[b->parity], b->stream);
        adv = 2;
      } else {
        e = hipGraphLaunch(b->exec_one[b->parity], b->stream);
      }
      if (e == hipSuccess) {
        nsteps -= adv;
        b->steps += adv;
        b->parity ^= flip;
      }
    }
    return dev(e);
  }
  if (b->fuse == 2) {
    // fused launches advance two steps and move the state to the other buffer
    while (nsteps > 0 && e == hipSuccess) {
      if (nsteps >= 2 * kFusedGraphLaunches) {
        e = hipGraphLaunch(b->exec_main2[b->parity], b->stream);  // even launch count: parity kept
        if (e == hipSuccess) {
          nsteps -= 2 * kFusedGraphLaunches;
          b->steps += 2 * kFusedGraphLaunches;
        }
      } else {
        const int two = nsteps >= 2;
        e = hipGraphLaunch(two ? b->exec_two[b->parity] : b->exec_one[b->parity], b->stream);
        if (e == hipSuccess) {
          nsteps -= two ? 2 : 1;
          b->steps += two ? 2 : 1;
          b->parity ^= 1;
        }
      }
    }
    return dev(e);
  }
  while (nsteps > 0 && e == hipSuccess) {
    if (b->parity == 0 && nsteps >= kGraphSteps) {
      e = hipGraphLaunch(b->exec_main, b->stream);
      if (e == hipSuccess) {
        nsteps -= kGraphSteps;
        b->steps += kGraphSteps;  // even count: parity unchanged
      }
    } else {
      e = hipGraphLaunch(b->exec_one[b->parity], b->stream);
      if (e == hipSuccess) {
        nsteps -= 1;
        b->steps += 1;
        b->parity ^= 1;
      }
    }
  }
  return dev(e);
}

lbm_status lbm_batch_moments(lbm_batch* b, int32_t run, double* rho, double* q) {
  if (!b || !rho || run < 0 || run >= b->nruns) return LBM_EINVAL;
  const Geometry& g = b->geo[run];
  const Ops* ops = ops_for(b->dim, b->storage);
  char* cur = b->ws + (b->parity ? b->off1[run] : b->off0[run]);
  double* st = reinterpret_cast<double*>(b->ws + (b->parity ? b->off0[run] : b->off1[run]));
  const size_t plane = static_cast<size_t>(g.cells) * sizeof(double);
  hipError_t e = ops->moments(g, b->coef[run], cur, st, nullptr, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(rho, st, plane, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess && q) e = hipMemcpyAsync(q, st + g.cells, plane * g.dim, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return dev(e);
}

lbm_status lbm_batch_info(const lbm_batch* b, int64_t* total_cells, int64_t* tiles, int64_t* steps) {
  if (!b) return LBM_EINVAL;
  if (total_cells) *total_cells = b->total_cells;
  if (tiles) *tiles = b->ntiles;
  if (steps) *steps = b->steps;
  return LBM_OK;
}

int32_t lbm_batch_grid(const lbm_batch* b) { return b ? b->grid : -1; }

int32_t lbm_batch_fused_grid(const lbm_batch* b) {
  if (!b) return -1;
  if (b->kdepth && b->fuse == b->kdepth) {
    int64_t blocks = 0;
    for (int sh = 0; sh < kShapes; ++sh)
      if (b->countK[sh]) blocks += gridK_for(b, b->countK[sh]);
    return static_cast<int32_t>(std::min<int64_t>(blocks, 0x7fffffff));
  }
  return b->kernel2 ? b->grid2 : 0;
}

lbm_status lbm_batch_fused_tile(const lbm_batch* b, int32_t run, int32_t* tx, int32_t* ty) {
  if (!b || run < 0 || run >= b->nruns || !b->kernelK[0].fn) return LBM_EINVAL;
  const BatchKKernel& k = b->kernelK[b->shape_of_class.at(b->cls[run])];
  if (tx) *tx = k.tx;
  if (ty) *ty = k.ty;
  return LBM_OK;
}

lbm_status lbm_batch_set_fused_shape(lbm_batch* b, int32_t shape) {
  if (!b || !b->kernelK[0].fn || shape < 0 || shape >= kShapes) return LBM_EINVAL;
  for (auto& kv : b->shape_of_class) kv.second = shape;
  hipError_t e = upload_tilesK(b);
  if (e == hipSuccess) e = rebuild(b);
  return dev(e);
}

lbm_status lbm_batch_set_fused_grid(lbm_batch* b, int32_t blocks_per_cu) {
  if (!b || !b->kernelK[0].fn || blocks_per_cu < 0 || blocks_per_cu > 64) return LBM_EINVAL;
  b->gridK = blocks_per_cu;
  return dev(rebuild(b));
}

lbm_status lbm_batch_set_fusion(lbm_batch* b, int32_t steps_per_launch) {
  if (!b) return LBM_EINVAL;
  if (steps_per_launch == 2 && !b->kernel2) return LBM_EINVAL;
  if (steps_per_launch != 1 && steps_per_launch != 2 && (steps_per_launch != b->kdepth || !b->kdepth))
    return LBM_EINVAL;
  b->fuse = steps_per_launch;
  return LBM_OK;
}

int32_t lbm_batch_fusion(const lbm_batch* b) { return b ? b->fuse : 0; }

int32_t lbm_batch_tile_width(const lbm_batch* b, int32_t run) {
  if (!b || run < 0 || run >= b->nruns) return -1;
  return b->bx_of_class.at(b->cls[run]);
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  destroy_graphs(b);
  delete b;
}

}  // extern "C"
