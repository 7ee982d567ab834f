// Host-side internals shared by the translation units of liblbm.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_device.hpp"

namespace lbm {

// Scalar coefficients of one run, in double (init) and float (step).
struct RunCoef {
  double dx, mu, alpha_rho, alpha_q, omega_rho, omega_q, ref;
  float neq_s[4] = {1.0f, 1.0f, 1.0f, 1.0f};  // split storage: power-of-two scale per set
};

template <int D>
inline NeqScale<D> neq_scale_of(const RunCoef& r) {
  NeqScale<D> sc;
  for (int i = 0; i < D + 1; ++i) {
    sc.s[i] = r.neq_s[i];
    sc.inv[i] = 1.0f / r.neq_s[i];  // exact: a power of two
  }
  return sc;
}

// Geometry of one state buffer.
struct Geometry {
  int dim;
  int32_t nx, ny, nz;
  int64_t cells;
  int64_t stride;       // elements between two planes (cells rounded up)
  size_t rest_elem;     // bytes per rest-plane element
  size_t move_elem;     // bytes per moving-plane element
  size_t rest_bytes;    // bytes of the rest-plane region (256-aligned)
  size_t buf_bytes;     // bytes of one full state buffer (256-aligned)
  int32_t zseg = 32;    // planes per block of the deepest 3D z-marching launch (Ops::zseg)
};

// Launchers of one (dimension, storage) instantiation.  Every launcher
// enqueues on `s` and returns the launch status.
struct Ops {
  hipError_t (*init)(const Geometry&, const RunCoef&, const double* u0, const double* rho0,
                     void* dst, hipStream_t s);
  hipError_t (*step)(const Geometry&, const RunCoef&, const void* src, void* dst, int bx, int by,
                     hipStream_t s);
  // two steps in one launch (2D only; nullptr where not available)
  hipError_t (*step2)(const Geometry&, const RunCoef&, const void* src, void* dst, hipStream_t s);
  hipError_t (*moments)(const Geometry&, const RunCoef&, const void* src, double* out64,
                        float* out32, hipStream_t s);
  hipError_t (*diag)(const Geometry&, const RunCoef&, const void* src, double* partials,
                     double* result, hipStream_t s);
  int64_t (*diag_blocks)(const Geometry&);
  // one step with the channel boundaries (2D population storages; nullptr otherwise)
  hipError_t (*step_walls)(const Geometry&, const RunCoef&, const void* src, void* dst, const WallArgs& w, int bx,
                           int by, hipStream_t s);
  // K = 3 .. max_fuse steps in one launch (2D population storages, 3D FP32; nullptr otherwise)
  hipError_t (*stepK)(const Geometry&, const RunCoef&, int K, const void* src, void* dst, hipStream_t s);
  int max_fuse;  // most steps per launch (1 .. kMaxFusion)
  // blocks of the 3D launch that advances `depth` steps (the z-marching
  // kernels take one block per column tile and z segment); INT64_MAX where
  // the grid does not depend on it (2D, and the one-step kernel)
  int64_t (*launch_blocks)(const Geometry&, int depth);
  // planes per block of the deepest 3D z-marching launch on a device with
  // `cus` compute units (nullptr where no such launch takes a segment length)
  int32_t (*zseg)(const Geometry&, int cus);
};

// Most time steps one launch may advance.
constexpr int kMaxFusion = 6;

// Fewest blocks with which a 3D z-marching launch is used where a
// cell-parallel launch can do the same work: those kernels take one block per
// column tile and z segment, so small grids leave most of the 256 compute
// units idle (64^3 FP32: 5.0 GLUPS with two steps per launch in 16 blocks,
// against 19.7 with the cell-parallel single step; moment-only single step
// at 64^3 / 128^3 / 192^3, z-marching in 8 / 64 / 216 blocks against
// cell-parallel: 5.3 / 36.1 / 101.8 against 61.3 / 87.6 / 96.4 GLUPS).
constexpr int64_t kMinZmarchBlocks3d = 128;

// Most blocks of the diagnostics launch (Ops::diag_blocks), hence most FP64
// partials its final pass reads.
constexpr int kDiagMaxBlocks = 2048;

// Ops for a dimension and an lbm_storage value; nullptr if unsupported.
const Ops* ops_for(int dim, int storage);

// Element sizes of a storage mode (rest planes, moving planes); false if unknown.
bool storage_elems(int storage, size_t* rest_elem, size_t* move_elem);

// Buffer geometry of one run (plane stride, region sizes) for a storage mode.
Geometry make_geometry(int dim, int storage, const int64_t n[3]);

// Planes per block of a 3D z-marching launch that fuses `stages` steps on
// 64 x `rows` column tiles, `per_cu` blocks per compute unit, on a device
// with `cus` compute units (lbm_kernels.hip).
int32_t zseg_for(const Geometry& g, int rows, int stages, int per_cu, int cus);

// Whether a storage mode stores deviations from the reference equilibrium.
bool storage_is_deviation(int storage);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Fused inference of the correction network (lbm_cnn.hip): y[3][h][w] and
// per-16x16-tile FP64 sums of y (4 doubles per tile) in part.
hipError_t net_infer_launch(const float* m, int h, int w, double rho_ref, float s_rho, float s_u,
                            const void* const* packed, const float* const* bias, float* y, double* part,
                            hipStream_t s);
// Tiles of the fused inference (0 if h or w is not a positive multiple of 16).
int64_t net_infer_tiles(int h, int w);

// A relaxation parameter omega in (0, 2) and 1 - omega as a pair of values of
// type R that sum to 1 exactly: the one of the two that is at least 1/2 is
// rounded, the other is its complement, which is exact (Sterbenz).  With a
// pair that missed 1 by an ulp, every relaxation would scale the moments by
// that ulp, a bias that grows with the number of steps.
template <typename R>
inline void omega_pair(double omega, R* w, R* r) {
  if (omega >= 0.5) {
    *w = static_cast<R>(omega);
    *r = static_cast<R>(1.0 - static_cast<double>(*w));
  } else {
    *r = static_cast<R>(1.0 - omega);
    *w = static_cast<R>(1.0 - static_cast<double>(*r));
  }
}

template <typename R>
inline CoefT<R> make_coef(const RunCoef& r, int D, bool deviation) {
  CoefT<R> k;
  k.c = static_cast<R>(1.0 / (2.0 * r.mu));
  k.a_rho = static_cast<R>(r.alpha_rho);
  k.a_q = static_cast<R>(r.alpha_q);
  k.d2a_rho = static_cast<R>(2.0 * D * r.alpha_rho);
  k.d2a_q = static_cast<R>(2.0 * D * r.alpha_q);
  omega_pair<R>(r.omega_rho, &k.w_rho, &k.r_rho);
  omega_pair<R>(r.omega_q, &k.w_q, &k.r_q);
  k.ref = static_cast<R>(deviation ? r.ref : 0.0);
  const double w_rho = static_cast<double>(k.w_rho), w_q = static_cast<double>(k.w_q);
  k.aw_rho = static_cast<R>(w_rho * r.alpha_rho);
  k.aw_q = static_cast<R>(w_q * r.alpha_q);
  k.d2aw_rho = static_cast<R>(2.0 * D * static_cast<double>(k.aw_rho));
  k.d2aw_q = static_cast<R>(2.0 * D * static_cast<double>(k.aw_q));
  k.cw_rho = static_cast<R>(w_rho / (2.0 * r.mu));
  k.cw_q = static_cast<R>(w_q / (2.0 * r.mu));
  return k;
}

template <typename TR, typename TM>
struct PlaneSet {
  TR* rest;  // [D+1][stride]
  TM* move;  // [D+1][2D][stride]
};

template <typename TR, typename TM>
__host__ __device__ inline PlaneSet<TR, TM> planes_of(void* base, size_t rest_bytes) {
  PlaneSet<TR, TM> p;
  p.rest = reinterpret_cast<TR*>(base);
  p.move = reinterpret_cast<TM*>(reinterpret_cast<char*>(base) + rest_bytes);
  return p;
}


}  // namespace lbm

// Host-side state of one run (the device memory belongs to the caller).
struct lbm_ctx {
  lbm_params p;
  double mu;
  double alpha_q;
  uint32_t flags;
  lbm::Geometry g;
  const lbm::Ops* ops;
  lbm::RunCoef coef;
  char* ws;
  size_t ws_bytes;
  char* cur;        // buffer holding the state at step `steps`
  char* nxt;        // the other buffer (also used as staging between steps)
  double* partials; // diagnostics per-block partials (also the closure's reduction scratch)
  int64_t part_doubles;  // capacity of `partials` in doubles
  double* result;   // diagnostics final slots
  double* closure_slots;  // lbm_closure_apply decision and report (8 doubles)
  double* static_scratch; // device address of the library's static diagnostics scratch on this device
  int64_t diag_blocks;
  hipStream_t stream;
  int64_t steps;
  int bx, by;       // step kernel block shape
  int fuse;         // time steps per launch: 1, 2 (two-step kernel) or 3..kMaxFusion (2D)
  int walls;        // 1: channel boundaries (lbm_set_walls) instead of periodic
  lbm::WallArgs wall;
  double* wall_profile;  // [2][ny] inlet velocity, in the workspace (2D)
};
