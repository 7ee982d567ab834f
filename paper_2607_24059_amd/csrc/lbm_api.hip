// C ABI of the single-run engine (see include/lbm.h for the contract).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "lbm.h"
#include "lbm_fused.hpp"
#include "lbm_internal.hpp"

using lbm::Geometry;
using lbm::Ops;
using lbm::RunCoef;



namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagSlots = 16;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

lbm_status check(const lbm_params* p, double* mu, double* alpha_q, uint32_t* flags) {
  if (!p) return LBM_EINVAL;
  if (p->dim != 2 && p->dim != 3) return LBM_EINVAL;
  size_t re, me;
  if (!lbm::storage_elems(p->storage, &re, &me)) return LBM_EINVAL;
  for (int a = 0; a < 3; ++a) {
    if (p->n[a] < 1 || p->n[a] > (int64_t(1) << 30)) return LBM_EINVAL;
  }
  if (p->dim == 2 && p->n[2] != 1) return LBM_EINVAL;
  const int64_t cells = p->n[0] * p->n[1] * p->n[2];
  if (cells > (int64_t(1) << 31) - 1) return LBM_EINVAL;
  if (p->dim == 3 && p->n[2] > 65535) return LBM_EINVAL;
  if (!(p->dx > 0.0) || !(p->dt > 0.0) || !isfinite(p->dx) || !isfinite(p->dt)) return LBM_EINVAL;
  if (!(p->nu >= 0.0) || !isfinite(p->nu)) return LBM_EINVAL;
  if (p->gamma != 1.0) return LBM_EINVAL;
  if (!(p->rho_ref > 0.0) || !isfinite(p->rho_ref)) return LBM_EINVAL;
  // omega in (0, 2): omega = 2 is inviscid (Section 3); Lemma 1 gives stability
  // of the checkerboard mode only for omega in [0, 2] and alpha in [0, 1/(2 dim)].
  if (!(p->omega_rho > 0.0 && p->omega_rho < 2.0)) return LBM_EUNSTABLE;
  if (!(p->omega_q > 0.0 && p->omega_q < 2.0)) return LBM_EUNSTABLE;
  // moment-only storage represents the relaxation scheme (omega = 1) only
  if (p->storage == LBM_F32_MOMENTS && (p->omega_rho != 1.0 || p->omega_q != 1.0)) return LBM_EINVAL;
  const double m = p->dx * p->dx / p->dt;
  const double aq = p->nu / (2.0 * m * (1.0 / p->omega_q - 0.5));
  const double amax = 1.0 / (2.0 * p->dim);
  if (!(p->alpha_rho >= 0.0 && p->alpha_rho <= amax)) return LBM_EUNSTABLE;
  if (!(aq >= 0.0 && aq <= amax)) return LBM_EUNSTABLE;
  uint32_t fl = 0;
  if (m * m * (p->alpha_rho + aq) < 1.0) fl |= LBM_WARN_LOWFREQ;
  if (mu) *mu = m;
  if (alpha_q) *alpha_q = aq;
  if (flags) *flags = fl;
  return LBM_OK;
}

Geometry geometry(const lbm_params* p) { return lbm::make_geometry(p->dim, p->storage, p->n); }

// staging (FP64 moments or initial fields) lives in the idle buffer
size_t staging_bytes(const Geometry& g) { return static_cast<size_t>(g.dim + 1) * g.cells * sizeof(double); }

// Storages whose state buffer is smaller than the FP64 staging (the
// moment-only storage: 12 B per cell in 2D against 24) get a staging region
// of their own after the other regions; the others stage in the idle buffer.
size_t extra_staging_bytes(const Geometry& g) {
  return staging_bytes(g) > g.buf_bytes ? align_up(staging_bytes(g)) : 0;
}

lbm_status dev(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

// compute units of the current device (256 if the query fails)
int device_cus() {
  int d = 0, cus = 0;
  if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

// Power-of-two scales of the split storage, one per set, from the run's
// parameters alone (so that any state loaded later, by lbm_load_state or
// lbm_set_equilibrium_device, is covered): s_i = 2^13 / M_i rounded down to a
// power of two, M_i the largest moving equilibrium deviation
// |alpha_i W_i| + |F_ij| / (2 mu) for a reference flow with W_q = 0.1 rho_ref
// (lattice Mach number 0.1) and |rho - rho_ref| = 0.01 rho_ref.  Non-equilibrium
// parts are a small fraction of M_i; they stay in FP16's normal range for
// flows from that Mach number down to about a hundredth of it, with 8x
// headroom below FP16's largest finite value at the reference.
void neq_scales(const lbm_params* p, double mu, double aq, float out[4]) {
  const double c = 1.0 / (2.0 * mu);
  const double w = 0.1 * p->rho_ref, dr = 0.01 * p->rho_ref;
  const double M[2] = {p->alpha_rho * dr + c * w, aq * w + c * (w * w / p->rho_ref + dr)};
  for (int i = 0; i < 4; ++i) {
    const double m = M[i == 0 ? 0 : 1];
    int e = 13 - static_cast<int>(ceil(log2(m)));
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    out[i] = (i <= p->dim) ? static_cast<float>(ldexp(1.0, e)) : 1.0f;
  }
}

// Doubles of the partials region: the diagnostics' per-block partials, and
// the closure's reductions (4-double partials of one 16 x 16 network tile or
// 256-cell guard block each, lbm_closure_apply / lbm_closure_correct).
int64_t partial_doubles(const Ops* o, const Geometry& g) {
  const int64_t diag = o->diag_blocks(g) * kDiagSlots;
  const int64_t closure = 4 * ((g.cells + 255) / 256 + 256);
  return diag > closure ? diag : closure;
}

// partials, then the diagnostics final slots, then 16 doubles of closure slots
size_t scratch_bytes(const Ops* o, const Geometry& g) {
  return align_up((static_cast<size_t>(partial_doubles(o, g)) + kDiagSlots + 16) * sizeof(double));
}

// inlet velocity profile of the channel boundaries: [2][ny] doubles (2D)
size_t profile_bytes(const lbm_params* p) {
  return p->dim == 2 ? align_up(2 * static_cast<size_t>(p->n[1]) * sizeof(double)) : 0;
}

// FP64 staging for initial fields and moments: the idle state buffer, or the
// region of its own (extra_staging_bytes) at the end of the workspace.
char* staging(lbm_ctx* c) {
  if (staging_bytes(c->g) <= c->g.buf_bytes) return c->nxt;
  return c->ws + 2 * c->g.buf_bytes + scratch_bytes(c->ops, c->g) + profile_bytes(&c->p);
}

// ---- scratch of the allocation-free diagnostics ------------------------------
// lbm_diagnostics_noalloc keeps the per-block partials and the final slots in
// this file-scope device array instead of the workspace: at most
// kDiagMaxBlocks partials of kDiagSlots doubles, then the final slots
// (262 KB).  Every GPU the library runs on holds its own copy until the
// process ends.  In host code the array's name is not a device address: its
// address on each device is looked up once, with that device current
// (static_scratch_of_current_device), and only that pointer is passed on.
constexpr int64_t kStaticDiagDoubles = (static_cast<int64_t>(lbm::kDiagMaxBlocks) + 1) * kDiagSlots;
static __device__ __align__(256) double scratch[kStaticDiagDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
hipError_t static_scratch_of_current_device(double** out) {
  int d = -1;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  if (d < 0 || d >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[d]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[d] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[d];
  return hipSuccess;
}

void default_block(const Geometry& g, int* bx, int* by) {
  int x = 256;
  while (x > 64 && x / 2 >= g.nx) x /= 2;
  *bx = x;
  *by = 256 / x;
}

}  // namespace

// Whether a context may run the K >= 3 kernels: the 2D tiles and the 3D
// three-step kernel address a plane (an x-y plane in 3D) with 32-bit byte
// offsets (fused_offsets_fit), so planes of more than 2^32 bytes take the
// two-step kernel.
static bool multi_step_fits(const lbm_ctx* c) {
  const int64_t plane = c->p.dim == 2 ? c->g.cells : static_cast<int64_t>(c->g.nx) * c->g.ny;
  return c->ops->stepK &&
         lbm::fused_offsets_fit(plane, c->g.move_elem > c->g.rest_elem ? c->g.move_elem : c->g.rest_elem);
}

// Whether a context may run its two-step kernel: the 3D moment-only one, too,
// addresses an x-y plane with 32-bit byte offsets.
static bool step2_fits(const lbm_ctx* c) {
  if (!c->ops->step2) return false;
  if (c->p.dim == 3 && c->p.storage == LBM_F32_MOMENTS)
    return lbm::fused_offsets_fit(static_cast<int64_t>(c->g.nx) * c->g.ny, sizeof(float));
  return true;
}

// Default steps per launch of the multi-step kernels, from sweeps at 4096^2:
// the FP32 storages peak at 6 (rest in registers on 32x28 tiles of 768
// threads: 192.6 GLUPS against 176.3 at 5 on 32x32, 191.5 at 7 and 177.8 at
// 8), the 16-bit storages with FP32 rest planes at 6 too (64x20 tiles: FP16 +
// FP32 rest 210.0 against 203.4 at 5), the all-16-bit and split storages at 5
// (BF16 214.5 against 210.7 at 6, split FP16 129.6 against 78.7), the
// moment-only storage at 4.
static int default_depth(int storage) {
  switch (storage) {
    case LBM_F32_MOMENTS: return 4;
    case LBM_F32: case LBM_F32_RAW: case LBM_F16_DEV_R32: case LBM_BF16_DEV_R32: return 6;
    default: return 5;
  }
}

// Steps per launch when a context is created.  2D: the multi-step kernels from
// 1024^2 cells on; smaller grids are launch-bound and keep the two-step
// kernel's small tiles.  3D: the deepest z-marching kernel whose launch has
// lbm::kMinZmarchBlocks3d blocks, else one step per launch.
static int default_fusion(const lbm_ctx* c) {
  const lbm::Ops* o = c->ops;
  if (c->p.dim == 3) {
    for (int d = std::min(3, o->max_fuse); d >= 2; --d) {
      const bool has = d >= 3 ? multi_step_fits(c) : step2_fits(c);
      if (has && o->launch_blocks(c->g, d) >= lbm::kMinZmarchBlocks3d) return d;
    }
    return 1;
  }
  if (multi_step_fits(c) && c->g.cells >= (int64_t(1) << 20)) return std::min(default_depth(c->p.storage), o->max_fuse);
  return o->step2 ? 2 : 1;
}

extern "C" {

lbm_status lbm_check_params(const lbm_params* p, double* mu, double* alpha_q, uint32_t* flags) {
  return check(p, mu, alpha_q, flags);
}

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (check(p, nullptr, nullptr, nullptr) != LBM_OK) return 0;
  const Geometry g = geometry(p);
  const Ops* o = lbm::ops_for(p->dim, p->storage);
  if (!o) return 0;
  return 2 * g.buf_bytes + scratch_bytes(o, g) + profile_bytes(p) + extra_staging_bytes(g);
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, const double* u0, const double* rho0,
                    void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out || !p || !u0 || !workspace) return LBM_EINVAL;
  *out = nullptr;
  double mu = 0, aq = 0;
  uint32_t flags = 0;
  lbm_status st = check(p, &mu, &aq, &flags);
  if (st != LBM_OK) return st;
  const size_t need = lbm_workspace_bytes(p);
  if (ws_bytes < need) return LBM_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return LBM_EINVAL;
  const Geometry g = geometry(p);
  const Ops* ops = lbm::ops_for(p->dim, p->storage);
  if (!ops) return LBM_EINVAL;

  lbm_ctx* c = new (std::nothrow) lbm_ctx;
  if (!c) return LBM_ENOMEM;
  c->p = *p;
  c->mu = mu;
  c->alpha_q = aq;
  c->flags = flags;
  c->g = g;
  c->ops = ops;
  if (p->dim == 3 && ops->zseg) c->g.zseg = ops->zseg(g, device_cus());
  c->coef = RunCoef{p->dx, mu, p->alpha_rho, aq, p->omega_rho, p->omega_q, p->rho_ref};
  if (p->storage == LBM_F16_NEQ) neq_scales(p, mu, aq, c->coef.neq_s);
  c->ws = static_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  c->cur = c->ws;
  c->nxt = c->ws + g.buf_bytes;
  c->partials = reinterpret_cast<double*>(c->ws + 2 * g.buf_bytes);
  c->diag_blocks = c->ops->diag_blocks(g);
  c->part_doubles = partial_doubles(c->ops, g);
  c->result = c->partials + c->part_doubles;
  c->closure_slots = c->result + kDiagSlots;
  c->walls = 0;
  c->wall = lbm::WallArgs{};
  c->wall_profile = p->dim == 2 ? reinterpret_cast<double*>(c->ws + 2 * g.buf_bytes + scratch_bytes(c->ops, g))
                                : nullptr;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->static_scratch = nullptr;
  default_block(g, &c->bx, &c->by);
  c->fuse = default_fusion(c);

  // stage u0 (and rho0) as FP64 in the idle buffer, then build the equilibrium
  double* su = reinterpret_cast<double*>(staging(c));
  double* sr = rho0 ? su + static_cast<size_t>(g.dim) * g.cells : nullptr;
  hipError_t e = hipMemcpyAsync(su, u0, static_cast<size_t>(g.dim) * g.cells * sizeof(double),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && rho0)
    e = hipMemcpyAsync(sr, rho0, static_cast<size_t>(g.cells) * sizeof(double), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = c->ops->init(g, c->coef, su, sr, c->cur, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->closure_slots, 0, 16 * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  // set-up of lbm_diagnostics_noalloc: the static scratch's address on this device
  if (e == hipSuccess) e = static_scratch_of_current_device(&c->static_scratch);
  if (e != hipSuccess) {
    delete c;
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  while (nsteps > 0) {
    // the longest launch that fits: fuse steps, then two, then one (all give
    // the same state bit for bit)
    const int k = c->walls ? 1 : nsteps >= c->fuse ? c->fuse : (c->fuse >= 2 && nsteps >= 2) ? 2 : 1;
    hipError_t e = c->walls ? c->ops->step_walls(c->g, c->coef, c->cur, c->nxt, c->wall, c->bx, c->by, c->stream)
                   : k >= 3 ? c->ops->stepK(c->g, c->coef, k, c->cur, c->nxt, c->stream)
                   : k == 2 ? c->ops->step2(c->g, c->coef, c->cur, c->nxt, c->stream)
                            : c->ops->step(c->g, c->coef, c->cur, c->nxt, c->bx, c->by, c->stream);
    if (e != hipSuccess) return LBM_EDEVICE;
    char* t = c->cur;
    c->cur = c->nxt;
    c->nxt = t;
    c->steps += k;
    nsteps -= k;
  }
  return LBM_OK;
}

lbm_status lbm_set_fusion(lbm_ctx* c, int32_t steps_per_launch) {
  if (!c || steps_per_launch < 1 || steps_per_launch > c->ops->max_fuse) return LBM_EINVAL;
  if (steps_per_launch >= 2 && (!step2_fits(c) || c->walls)) return LBM_EINVAL;
  if (steps_per_launch >= 3 && !multi_step_fits(c)) return LBM_EINVAL;
  c->fuse = steps_per_launch;
  return LBM_OK;
}

int32_t lbm_fusion(const lbm_ctx* c) { return c ? c->fuse : 0; }

lbm_status lbm_set_walls(lbm_ctx* c, const lbm_walls* w, const double* u_in) {
  if (!c) return LBM_EINVAL;
  if (!w) {
    c->walls = 0;
    return LBM_OK;
  }
  if (!c->ops->step_walls || !u_in || c->p.n[0] < 3 || c->p.n[1] < 3) return LBM_EINVAL;
  if (!isfinite(w->rho_out) || !(w->rho_out > 0.0) || !isfinite(w->u_bottom) || !isfinite(w->u_top))
    return LBM_EINVAL;
  const size_t bytes = 2 * static_cast<size_t>(c->p.n[1]) * sizeof(double);
  hipError_t e = hipMemcpyAsync(c->wall_profile, u_in, bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the host array may go away
  if (e != hipSuccess) return LBM_EDEVICE;
  c->wall = lbm::WallArgs{c->wall_profile, w->rho_out, w->u_bottom, w->u_top, c->p.dx, c->p.rho_ref,
                          w->correction ? 1 : 0};
  c->walls = 1;
  c->fuse = 1;
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, double* rho, double* q) {
  if (!c || !rho) return LBM_EINVAL;
  double* st = reinterpret_cast<double*>(staging(c));
  const size_t plane = static_cast<size_t>(c->g.cells) * sizeof(double);
  hipError_t e = c->ops->moments(c->g, c->coef, c->cur, st, nullptr, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(rho, st, plane, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && q)
    e = hipMemcpyAsync(q, st + c->g.cells, plane * c->g.dim, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return dev(e);
}

lbm_status lbm_moments_device(lbm_ctx* c, float* out) {
  if (!c || !out) return LBM_EINVAL;
  return dev(c->ops->moments(c->g, c->coef, c->cur, nullptr, out, c->stream));
}

}  // extern "C"

// Diagnostics with the partials and final slots in `partials` and `result`.
static lbm_status diagnostics_into(lbm_ctx* c, double* partials, double* result, lbm_diag* out) {
  double r[kDiagSlots];
  hipError_t e = c->ops->diag(c->g, c->coef, c->cur, partials, result, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(r, result, sizeof(r), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return LBM_EDEVICE;
  const double dv = pow(c->p.dx, c->p.dim);
  memset(out, 0, sizeof(*out));
  out->step = c->steps;
  out->time = static_cast<double>(c->steps) * c->p.dt;
  out->mass = dv * r[0];
  for (int j = 0; j < c->p.dim; ++j) out->mom[j] = dv * r[1 + j];
  out->kinetic = 0.5 * dv * r[4];
  out->enstrophy = 0.5 * dv * r[5];
  out->div_l2 = sqrt(dv * r[6]);
  out->max_u = sqrt(r[7]);
  out->rho_min = r[8];
  out->rho_max = r[9];
  out->nonfinite = static_cast<int64_t>(r[10]);
  out->flags = c->flags;
  return out->nonfinite > 0 ? LBM_ENONFINITE : LBM_OK;
}

extern "C" {

lbm_status lbm_diagnostics(lbm_ctx* c, lbm_diag* out) {
  if (!c || !out) return LBM_EINVAL;
  return diagnostics_into(c, c->partials, c->result, out);
}

// The kernels of lbm_diagnostics, with their scratch in the static array:
// every partial slot the final pass reads is written by the first launch of
// the same call, so nothing needs clearing; calls that overlap on one GPU
// share the array and race.
lbm_status lbm_diagnostics_noalloc(lbm_ctx* c, lbm_diag* out) {
  if (!c || !out) return LBM_EINVAL;
  if (!c->static_scratch) return LBM_EDEVICE;
  if (c->diag_blocks < 1 || c->diag_blocks > lbm::kDiagMaxBlocks) return LBM_EINVAL;
  double* partials = c->static_scratch;
  double* result = c->static_scratch + static_cast<int64_t>(lbm::kDiagMaxBlocks) * kDiagSlots;
  return diagnostics_into(c, partials, result, out);
}

// The snapshot holds every plane without its padding: the rest planes
// (D+1 x cells x rest element), the moving planes ((D+1) 2D x cells x moving
// element), then the step count, then (split storage only) the four FP32
// per-set scales the moving planes were written with.
static size_t compact_rest(const lbm_ctx* c) {
  return static_cast<size_t>(c->p.dim + 1) * c->g.cells * c->g.rest_elem;
}
static size_t compact_move(const lbm_ctx* c) {
  return static_cast<size_t>(c->p.dim + 1) * 2 * c->p.dim * c->g.cells * c->g.move_elem;
}

static size_t trailer_bytes(const lbm_ctx* c) {
  return sizeof(int64_t) + (c->p.storage == LBM_F16_NEQ ? sizeof(c->coef.neq_s) : 0);
}

size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  return compact_rest(c) + compact_move(c) + trailer_bytes(c);
}

static hipError_t copy_planes(lbm_ctx* c, char* host, bool to_host) {
  const Geometry& g = c->g;
  const int ns = c->p.dim + 1, nm = ns * 2 * c->p.dim;
  const size_t wr = static_cast<size_t>(g.cells) * g.rest_elem, pr = static_cast<size_t>(g.stride) * g.rest_elem;
  const size_t wm = static_cast<size_t>(g.cells) * g.move_elem, pm = static_cast<size_t>(g.stride) * g.move_elem;
  char* dev_rest = c->cur;
  char* dev_move = c->cur + g.rest_bytes;
  hipError_t e;
  if (to_host) {
    e = hipMemcpy2DAsync(host, wr, dev_rest, pr, wr, ns, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(host + ns * wr, wm, dev_move, pm, wm, nm, hipMemcpyDeviceToHost, c->stream);
  } else {
    e = hipMemcpy2DAsync(dev_rest, pr, host, wr, wr, ns, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(dev_move, pm, host + ns * wr, wm, wm, nm, hipMemcpyHostToDevice, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

lbm_status lbm_save_state(lbm_ctx* c, void* host, size_t bytes) {
  if (!c || !host) return LBM_EINVAL;
  if (bytes != lbm_state_bytes(c)) return LBM_ESTATE;
  if (copy_planes(c, static_cast<char*>(host), true) != hipSuccess) return LBM_EDEVICE;
  char* t = static_cast<char*>(host) + compact_rest(c) + compact_move(c);
  memcpy(t, &c->steps, sizeof(int64_t));
  if (c->p.storage == LBM_F16_NEQ) memcpy(t + sizeof(int64_t), c->coef.neq_s, sizeof(c->coef.neq_s));
  return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx* c, const void* host, size_t bytes) {
  if (!c || !host) return LBM_EINVAL;
  if (bytes != lbm_state_bytes(c)) return LBM_ESTATE;
  if (copy_planes(c, const_cast<char*>(static_cast<const char*>(host)), false) != hipSuccess) return LBM_EDEVICE;
  const char* t = static_cast<const char*>(host) + compact_rest(c) + compact_move(c);
  memcpy(&c->steps, t, sizeof(int64_t));
  if (c->p.storage == LBM_F16_NEQ) memcpy(c->coef.neq_s, t + sizeof(int64_t), sizeof(c->coef.neq_s));
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->steps : -1; }

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EUNSTABLE: return "parameters outside the stability region (omega in (0,2), alpha in [0,1/(2d)])";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite populations";
    case LBM_ESTATE: return "state blob size or layout mismatch";
  }
  return "unknown status";
}

lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16 != 0) return LBM_EINVAL;
  if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16) return LBM_EINVAL;
  return dev(lbm::launch_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream)));
}

}  // extern "C"
