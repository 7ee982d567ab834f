// Host-side internals shared by the translation units of liblbm.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// Scalar coefficients of one run, in double (init) and float (step).
struct RunCoef {
  double dx, mu, alpha_rho, alpha_q, omega_rho, omega_q, ref;
};

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
};

// Launchers of one (dimension, storage) instantiation.  Every launcher
// enqueues on `s` and returns the launch status.
struct Ops {
  hipError_t (*init)(const Geometry&, const RunCoef&, const double* u0, const double* rho0,
                     void* dst, hipStream_t s);
  hipError_t (*step)(const Geometry&, const RunCoef&, const void* src, void* dst, int bx, int by,
                     hipStream_t s);
  hipError_t (*moments)(const Geometry&, const RunCoef&, const void* src, double* out64,
                        float* out32, hipStream_t s);
  hipError_t (*diag)(const Geometry&, const RunCoef&, const void* src, double* partials,
                     double* result, hipStream_t s);
  int64_t (*diag_blocks)(const Geometry&);
};

// Ops for a dimension and an lbm_storage value; nullptr if unsupported.
const Ops* ops_for(int dim, int storage);

// Element sizes of a storage mode (rest planes, moving planes); false if unknown.
bool storage_elems(int storage, size_t* rest_elem, size_t* move_elem);

// Whether a storage mode stores deviations from the reference equilibrium.
bool storage_is_deviation(int storage);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace lbm
