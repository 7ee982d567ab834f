// Device-side building blocks of the vectorial lattice Boltzmann engine (gfx950).
//
// Units.  Every stored population is in the scaled units of the paper's moment
// definition (Section 2): the moments are W = sum_l f_l = (rho, dx q_x, dx q_y
// [, dx q_z]).  Dividing the equilibria of Section 2 through by the powers of dx
// they carry leaves a form that depends on W, mu = dx^2/dt and the alphas only:
//
//   F_{rho j} = W_j,      F_{i j} = W_i W_j / W_rho + delta_ij P(W_rho)
//   f^eq_{i,rest} = (1 - 2 D alpha_i) W_i
//   f^eq_{i,+-j}  = alpha_i W_i +- F_{ij} / (2 mu)
//
// (for example dx alpha q_x = alpha W_x and dx^2/(2 mu) q_x^2/rho = W_x^2/(2 mu W_rho)).
// The rest component of each momentum set carries the factor dx that makes
// the equilibria sum to W, the reading under which Lemma 1 holds.
//
// Deviation storage.  With a reference density rho_ref, the populations can be
// stored as g = f - fbar where fbar = f^eq(rho_ref, 0):
//   density set  fbar_rest = (1 - 2D alpha_rho) rho_ref, fbar_{+-j} = alpha_rho rho_ref
//   set q_i      fbar_{+-i} = +- rho_ref / (2 mu), every other entry 0.
// Since sum_l fbar_{rho,l} = rho_ref and sum_l fbar_{q_i,l} = 0, the sums of g
// are (W_rho - rho_ref, W_q), and for P(rho) = rho the deviation of the
// equilibrium, f^eq(W) - fbar, is the same formula with W_rho replaced by its
// deviation in every linear term and only 1/W_rho using rho_ref + deviation.
// So one collision routine serves both forms: rho_ref = 0 is the plain scheme.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ----------------------------------------------------------------------------
// storage element types
// ----------------------------------------------------------------------------
struct bf16 {
  uint16_t bits;
};

// FP16 bits of v (round to nearest even) and the float of FP16 bits: the
// hardware conversions written out, so that the compiler keeps each value in
// a 32-bit register of its own.  Left to itself it packs FP16 values into
// register halves and folds a conversion into the FMA before it (rounding the
// exact product-sum to FP16 once instead of the FP32 result); in the 3D
// three-step kernels that spilled 24-26 bytes per lane at 64 x 8 tiles (GLUPS
// at 256^3: FP16 + FP32 rest 57.4 -> 84.0, FP16 63.1 -> 83.7; 2D FP16 at
// 4096^2: 185 -> 212).
__device__ __forceinline__ uint16_t f16_bits(float v) {
  uint32_t b;
  __asm__("v_cvt_f16_f32_e32 %0, %1" : "=v"(b) : "v"(v));
  return static_cast<uint16_t>(b);
}
__device__ __forceinline__ float f16_value(uint16_t h) {
  float f;
  __asm__("v_cvt_f32_f16_e32 %0, %1" : "=v"(f) : "v"(static_cast<uint32_t>(h)));
  return f;
}

__device__ __forceinline__ float load_f32(const float* p) { return *p; }
__device__ __forceinline__ float load_f32(const _Float16* p) { return f16_value(*reinterpret_cast<const uint16_t*>(p)); }
__device__ __forceinline__ float load_f32(const bf16* p) {
  return __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
}

__device__ __forceinline__ void store_f32(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_f32(_Float16* p, float v) { *reinterpret_cast<uint16_t*>(p) = f16_bits(v); }
// BF16 bits of v, rounded to nearest even by the hardware conversion (one
// instruction on gfx950, against six for the same rounding in integer code)
__device__ __forceinline__ uint16_t bf16_bits(float v) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}
__device__ __forceinline__ void store_f32(bf16* p, float v) { p->bits = bf16_bits(v); }

// Moving planes of the equilibrium-split storage (LBM_F16_NEQ): FP16 bits of a
// scaled non-equilibrium part; a type of its own selects that storage's code.
struct neq16 {
  _Float16 v;
};
__device__ __forceinline__ float load_f32(const neq16* p) { return static_cast<float>(p->v); }
__device__ __forceinline__ void store_f32(neq16* p, float v) { p->v = static_cast<_Float16>(v); }
template <typename TM>
struct IsNeq {
  static constexpr bool value = false;
};
template <>
struct IsNeq<neq16> {
  static constexpr bool value = true;
};

// Moment-only storage (LBM_F32_MOMENTS, the relaxation scheme omega = 1 on
// every set): no moving planes at all; a tag type for the missing planes.
struct mom0 {};
template <typename TM>
struct IsMom {
  static constexpr bool value = false;
};
template <>
struct IsMom<mom0> {
  static constexpr bool value = true;
};
// Storages whose rest planes hold the moments W themselves.
template <typename TM>
struct StoresMoments {
  static constexpr bool value = IsNeq<TM>::value || IsMom<TM>::value;
};

// FP64 storage (the reference mode): loaded, updated and stored in FP64.
__device__ __forceinline__ double load_f64(const double* p) { return *p; }
template <typename T>
__device__ __forceinline__ double load_f64(const T* p) { return static_cast<double>(load_f32(p)); }

// Store an FP64 value: kept whole in FP64 storage, otherwise rounded to FP32
// first and then to the element type (the rounding of every FP32 path).
__device__ __forceinline__ void store_real(double* p, double v) { *p = v; }
template <typename T>
__device__ __forceinline__ void store_real(T* p, double v) { store_f32(p, static_cast<float>(v)); }

// Arithmetic type of the update for a storage element type.
template <typename T>
struct ComputeOf {
  using type = float;
};
template <>
struct ComputeOf<double> {
  using type = double;
};

template <typename R>
__device__ __forceinline__ R load_as(const double* p) { return static_cast<R>(*p); }
template <typename R, typename T>
__device__ __forceinline__ R load_as(const T* p) { return static_cast<R>(load_f32(p)); }

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Streaming stores for the step kernel: the next step reads these values from
// HBM anyway (the state is far larger than the caches), so they are written
// with the non-temporal hint and do not displace the neighbour lines that the
// shifted loads of adjacent tiles still need.
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(_Float16* p, float v) {
  __builtin_nontemporal_store(f16_bits(v), reinterpret_cast<uint16_t*>(p));
}
__device__ __forceinline__ void store_stream(bf16* p, float v) {
  __builtin_nontemporal_store(bf16_bits(v), reinterpret_cast<uint16_t*>(p));
}
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(neq16* p, float v) {
  __builtin_nontemporal_store(static_cast<_Float16>(v), reinterpret_cast<_Float16*>(p));
}

// ----------------------------------------------------------------------------
// lattice description: D2Q5 / D3Q7 per set, D+1 sets
//   velocity l: 0 = rest, 1 + 2j = +e_j, 2 + 2j = -e_j   (j = 0 is x)
//   set i:      0 = rho, 1 + j = q_j
// plane layout in HBM (SoA, x fastest):
//   rest planes  [set][cells]           element type TR
//   moving planes[set][2D][cells]       element type TM, velocity order 1..2D
// ----------------------------------------------------------------------------
template <int D>
struct Lattice {
  static constexpr int NS = D + 1;      // sets
  static constexpr int NV = 2 * D + 1;  // velocities per set
  static constexpr int NM = 2 * D;      // moving velocities per set
};

template <typename R>
struct CoefT {
  R c;         // 1 / (2 mu)
  R a_rho;     // alpha_rho
  R a_q;       // alpha_q
  R d2a_rho;   // 2 D alpha_rho
  R d2a_q;     // 2 D alpha_q
  R w_rho;     // omega_rho
  R w_q;       // omega_q
  R ref;       // rho_ref for deviation storage, 0 for plain storage
  // the relaxation's coefficients with omega folded in (collide)
  R r_rho, r_q;        // 1 - omega (exact in R: omega lies in (0, 2))
  R aw_rho, aw_q;      // omega alpha
  R d2aw_rho, d2aw_q;  // 2 D (omega alpha), from the rounded omega alpha
  R cw_rho, cw_q;      // omega / (2 mu)
};
using Coef = CoefT<float>;

// Equilibrium (or its deviation from fbar) of one cell in scaled units.
// W[0] is W_rho for plain storage or W_rho - rho_ref for deviations; W[1+j]
// is W_{q_j}; inv = 1 / W_rho (always the full density).
template <int D, typename R>
__device__ __forceinline__ void equilibrium(const R (&W)[D + 1], R inv, const CoefT<R>& k,
                                            R (&eq)[D + 1][2 * D + 1]) {
  const R wl = W[0];
  // density set: F_{rho j} = W_j.  The rest entry (1 - 2D alpha) W is formed
  // as W - (2D alpha) W: rounding the coefficient 1 - 2D alpha itself would
  // break the exact sum of the equilibria by up to half an ulp of W per step,
  // a bias that accumulates; the product (2D alpha) W is small, so its
  // rounding error is negligible.
  eq[0][0] = wl - k.d2a_rho * wl;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R base = k.a_rho * wl;
    const R flux = k.c * W[1 + j];
    eq[0][1 + 2 * j] = base + flux;
    eq[0][2 + 2 * j] = base - flux;
  }
  // momentum sets: F_{ij} = W_i W_j / W_rho + delta_ij P(W_rho), P(rho) = rho
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const R wi = W[1 + i];
    eq[1 + i][0] = wi - k.d2a_q * wi;
    const R base = k.a_q * wi;
    const R wi_inv = wi * inv;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R F = wi_inv * W[1 + j];
      if (i == j) F = F + wl;
      const R flux = k.c * F;
      eq[1 + i][1 + 2 * j] = base + flux;
      eq[1 + i][2 + 2 * j] = base - flux;
    }
  }
}

// Relax the populations of one cell in place: f* = f + omega (f^eq - f),
// equation (LBM_scheme).  g[i][l] holds plain values (ref = 0) or deviations;
// R is the arithmetic type (FP32, or FP64 for the FP64 storage).
// 1 / rho in the relaxation: the hardware reciprocal (1 ulp) in FP32, as in
// every kernel that relaxes a cell, and the correctly rounded quotient in FP64
__device__ __forceinline__ float recip_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip_r(double x) { return 1.0 / x; }

// Periodic index of v on a grid of n cells, for v within a tile border of the
// grid: two compares while v lies in [-n, 2n), the remainder otherwise (tiny
// grids, where a border wraps several times).
// XCD-major order of n tiles: with a one-dimensional grid, block (slot) q
// runs on XCD q mod 8, so XCD j takes the slots j, j + 8, ...; giving it the
// j-th of eight contiguous runs of tiles (the first n mod 8 runs one longer)
// makes the tiles that run together on one XCD neighbours, and their shared
// borders are read through its L2.  A bijection of [0, n) for every n.
__host__ __device__ __forceinline__ int64_t xcd_major(int64_t q, int64_t n) {
  const int64_t j = q % 8, per = n / 8, extra = n % 8;
  return j * per + (j < extra ? j : extra) + q / 8;
}

__device__ __forceinline__ int wrap_coord(int v, int n) {
  if (v >= -n && v < 2 * n) return v < 0 ? v + n : (v >= n ? v - n : v);
  return ((v % n) + n) % n;
}

// Relaxation of one cell, f* = f + omega (f^eq - f), evaluated as
// f* = (1 - omega) f + omega f^eq with omega folded into the equilibrium
// coefficients (omega alpha, omega / (2 mu)), so that each entry costs one FMA
// after omega f^eq (about 60 operations per cell in 2D against 79 for the
// separate difference and FMA).  The rest entry, omega (1 - 2 D alpha) W, is
// formed as omega W - (2 D omega alpha) W with 2 D omega alpha = 2 D times the
// rounded omega alpha: the coefficients of one set then sum to omega exactly
// in 2D (see equilibrium() for why a rounded 1 - 2 D alpha would bias the sums).
template <int D, typename R>
__device__ __forceinline__ void collide(R (&g)[D + 1][2 * D + 1], const CoefT<R>& k) {
  R W[D + 1];
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    R s = g[i][0];
#pragma unroll
    for (int l = 1; l < 2 * D + 1; ++l) s = s + g[i][l];
    W[i] = s;
  }
  const R inv = recip_r(W[0] + k.ref);
  const R wl = W[0];
  {  // density set: F_{rho j} = W_j
    const R base = k.aw_rho * wl;
    g[0][0] = fma_r(k.r_rho, g[0][0], fma_r(-k.d2aw_rho, wl, k.w_rho * wl));
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const R flux = k.cw_rho * W[1 + j];
      g[0][1 + 2 * j] = fma_r(k.r_rho, g[0][1 + 2 * j], base + flux);
      g[0][2 + 2 * j] = fma_r(k.r_rho, g[0][2 + 2 * j], base - flux);
    }
  }
  // momentum sets: F_{ij} = W_i W_j / W_rho + delta_ij P(W_rho), P(rho) = rho
  const R cinv = k.cw_q * inv;
  const R cwl = k.cw_q * wl;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const R wi = W[1 + i];
    const R base = k.aw_q * wi;
    g[1 + i][0] = fma_r(k.r_q, g[1 + i][0], fma_r(-k.d2aw_q, wi, k.w_q * wi));
    const R ci = cinv * wi;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const R flux = (i == j) ? fma_r(ci, W[1 + j], cwl) : ci * W[1 + j];
      g[1 + i][1 + 2 * j] = fma_r(k.r_q, g[1 + i][1 + 2 * j], base + flux);
      g[1 + i][2 + 2 * j] = fma_r(k.r_q, g[1 + i][2 + 2 * j], base - flux);
    }
  }
}


// Gather the post-relaxation values of the upwind neighbours of cell (x, y, z):
// the pull form of the transport phase, f_{+e_j}(t+dt, x) = f*_{+e_j}(t, x - dx e_j),
// on the periodic grid.  c is the cell's linear index.
// Linear indices of the upwind neighbour of cell c = (x, y, z) for each moving
// velocity (periodic wrap).
template <int D>
__device__ __forceinline__ void upwind_sources(int x, int y, int z, int nx, int ny, int nz, int64_t c,
                                               int64_t (&src)[2 * D]) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  src[0] = (x == 0) ? c + (nx - 1) : c - 1;                                   // +x from x-1
  src[1] = (x == nx - 1) ? c - (nx - 1) : c + 1;                              // -x from x+1
  src[2] = (y == 0) ? c + static_cast<int64_t>(ny - 1) * nx : c - nx;         // +y from y-1
  src[3] = (y == ny - 1) ? c - static_cast<int64_t>(ny - 1) * nx : c + nx;    // -y from y+1
  if constexpr (D == 3) {
    src[4] = (z == 0) ? c + static_cast<int64_t>(nz - 1) * plane : c - plane;      // +z
    src[5] = (z == nz - 1) ? c - static_cast<int64_t>(nz - 1) * plane : c + plane; // -z
  }
}

template <int D, typename TR, typename TM, typename R>
__device__ __forceinline__ void gather_cell(const TR* __restrict__ sr, const TM* __restrict__ sm, int x, int y,
                                            int z, int nx, int ny, int nz, int64_t stride, int64_t c,
                                            R (&g)[D + 1][2 * D + 1]) {
  int64_t src[2 * D];
  upwind_sources<D>(x, y, z, nx, ny, nz, c, src);
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    g[i][0] = load_as<R>(sr + i * stride + c);
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) g[i][1 + m] = load_as<R>(sm + (i * 2 * D + m) * stride + src[m]);
  }
}

// One lattice update of cell (x, y, z): gather, sum the moments, relax, and
// write the cell's own post-relaxation values.  Every stored value is read
// once and written once per step.  Used by the single-run and the batched
// kernels, so both produce bit-identical states.
template <int D, typename TR, typename TM, typename R = typename ComputeOf<TM>::type>
__device__ __forceinline__ void step_cell(const TR* __restrict__ sr, const TM* __restrict__ sm,
                                          TR* __restrict__ dr, TM* __restrict__ dm, int x, int y,
                                          int z, int nx, int ny, int nz, int64_t stride,
                                          const CoefT<R>& k) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const int64_t c = static_cast<int64_t>(z) * plane + static_cast<int64_t>(y) * nx + x;
  R g[D + 1][2 * D + 1];
  gather_cell<D, TR, TM, R>(sr, sm, x, y, z, nx, ny, nz, stride, c, g);
  collide<D, R>(g, k);
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    store_stream(dr + i * stride + c, g[i][0]);
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) store_stream(dm + (i * 2 * D + m) * stride + c, g[i][1 + m]);
  }
}

// ----------------------------------------------------------------------------
// Equilibrium-split storage (LBM_F16_NEQ)
//
// Per cell the moments W (FP32 planes in place of the rest planes; W_rho as a
// deviation from rho_ref) and, per set i and moving velocity, the
// non-equilibrium part n = f* - f^eq(W) of the stored post-relaxation
// population, in FP16 after multiplication by a power of two s_i per set.
// The rest entry's non-equilibrium part is minus the sum of the moving ones
// (f* and f^eq both sum to W), so W is conserved exactly by the storage and
// FP16 only ever rounds the small non-equilibrium parts.
// ----------------------------------------------------------------------------
template <int D>
struct NeqScale {
  float s[D + 1];    // stored value = n * s[i]
  float inv[D + 1];  // 1 / s[i]
};

// 1 / rho where equilibria are rebuilt from stored moments (the split and the
// moment-only storage): the hardware reciprocal (1 ulp), used by every such
// routine alike so that a cell's equilibrium rebuilt by a neighbour equals the
// one the cell computed itself, bit for bit, in every kernel.
__device__ __forceinline__ float recip_neq(float x) { return __builtin_amdgcn_rcpf(x); }

// The equilibrium (deviation) of set i, moving velocity 1 + m (axis m / 2,
// + for even m), at a cell with moments W; the arithmetic of equilibrium<D, float>.
template <int D, typename R>
__device__ __forceinline__ R eq_moving(const R (&W)[D + 1], R inv, const CoefT<R>& k, int i, int m) {
  const int j = m >> 1;
  R base, flux;
  if (i == 0) {
    base = k.a_rho * W[0];
    flux = k.c * W[1 + j];
  } else {
    const R wi = W[i];
    base = k.a_q * wi;
    R F = (wi * inv) * W[1 + j];
    if (i - 1 == j) F = F + W[0];
    flux = k.c * F;
  }
  return (m & 1) ? base - flux : base + flux;
}

// Pull-transported populations (deviations) of one cell from split storage.
// w_at(i, nb): W_i of the cell (nb < 0) or of its upwind neighbour for moving
// velocity nb; n_at(i, m, nb): stored (scaled) n of set i, velocity m there.
template <int D, typename WAt, typename NAt>
__device__ __forceinline__ void gather_neq(WAt w_at, NAt n_at, const Coef& k, const NeqScale<D>& sc,
                                           float (&g)[D + 1][2 * D + 1]) {
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    float s = n_at(i, 0, -1);
#pragma unroll
    for (int m = 1; m < 2 * D; ++m) s = s + n_at(i, m, -1);
    const float wl = w_at(i, -1);
    const float d2a = (i == 0) ? k.d2a_rho : k.d2a_q;
    g[i][0] = (wl - d2a * wl) - s * sc.inv[i];
  }
#pragma unroll
  for (int m = 0; m < 2 * D; ++m) {
    float Wn[D + 1];
#pragma unroll
    for (int i = 0; i < D + 1; ++i) Wn[i] = w_at(i, m);
    const float inv = recip_neq(Wn[0] + k.ref);
#pragma unroll
    for (int i = 0; i < D + 1; ++i) g[i][1 + m] = eq_moving<D>(Wn, inv, k, i, m) + n_at(i, m, m) * sc.inv[i];
  }
}

// Relaxation in split form: W = sum_l f_l (unchanged by the relaxation) and
// n* = f* - f^eq(W) = (1 - omega)(f - f^eq(W)) for the moving velocities;
// eq receives f^eq(W).
template <int D>
__device__ __forceinline__ void collide_neq(const float (&g)[D + 1][2 * D + 1], const Coef& k, float (&W)[D + 1],
                                            float (&n)[D + 1][2 * D], float (&eq)[D + 1][2 * D + 1]) {
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    float s = g[i][0];
#pragma unroll
    for (int l = 1; l < 2 * D + 1; ++l) s = s + g[i][l];
    W[i] = s;
  }
  const float inv = recip_neq(W[0] + k.ref);
  equilibrium<D, float>(W, inv, k, eq);
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    const float r = 1.0f - ((i == 0) ? k.w_rho : k.w_q);
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) n[i][m] = r * (g[i][1 + m] - eq[i][1 + m]);
  }
}

// One lattice update of cell (x, y, z) in split storage.
template <int D>
__device__ __forceinline__ void step_cell_neq(const float* __restrict__ sr, const neq16* __restrict__ sm,
                                              float* __restrict__ dr, neq16* __restrict__ dm, int x, int y, int z,
                                              int nx, int ny, int nz, int64_t stride, const Coef& k,
                                              const NeqScale<D>& sc) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const int64_t c = static_cast<int64_t>(z) * plane + static_cast<int64_t>(y) * nx + x;
  int64_t src[2 * D];
  upwind_sources<D>(x, y, z, nx, ny, nz, c, src);
  auto w_at = [&](int i, int nb) { return sr[i * stride + (nb < 0 ? c : src[nb])]; };
  auto n_at = [&](int i, int m, int nb) { return load_f32(sm + (i * 2 * D + m) * stride + (nb < 0 ? c : src[nb])); };
  float g[D + 1][2 * D + 1];
  gather_neq<D>(w_at, n_at, k, sc, g);
  float W[D + 1], n[D + 1][2 * D], eq[D + 1][2 * D + 1];
  collide_neq<D>(g, k, W, n, eq);
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    store_stream(dr + i * stride + c, W[i]);
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) store_stream(dm + (i * 2 * D + m) * stride + c, n[i][m] * sc.s[i]);
  }
}

// ----------------------------------------------------------------------------
// Moment-only storage: with omega = 1 on every set the post-relaxation
// populations are the equilibria of the cell's moments, so the state is W
// alone and a step is the stencil
//   W_i(t+1, x) = f^eq_{i,rest}(W(t, x)) + sum_moving f^eq_{i,l}(W(t, x - c_l))
// (the relaxation scheme of Section 2; in deviation form, since the reference
// equilibria of one set sum to the same constant in every cell).
// ----------------------------------------------------------------------------
// With inv_at(m) the 1 / rho of upwind neighbour m, as recip_neq(W_0 + ref)
// gives it (callers that keep it per cell pass it in; the value is the same).
template <int D, typename WAt, typename InvAt>
__device__ __forceinline__ void step_moments_inv(WAt w_at, InvAt inv_at, const Coef& k, float (&out)[D + 1]) {
  // Every moving entry of set i at an upwind neighbour is base + flux or
  // base - flux: the bases (a W_i of the neighbour) are summed once over the
  // 2D neighbours, and the fluxes c F_ij once per axis j as the difference of
  // the neighbours behind (x - e_j, entry + flux) and ahead (x + e_j, entry
  // - flux).  F_0j = W_{1+j}; F_ij = (W_i / rho) W_{1+j} (+ W_0 for the
  // pressure, i - 1 = j), with 1 / rho the hardware reciprocal of the split
  // storage's equilibria.
  float sum_w[D + 1], sum_f[D + 1];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    float Fb[D + 1], Fa[D + 1];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int m = 2 * j + side;
      float Wn[D + 1];
#pragma unroll
      for (int i = 0; i < D + 1; ++i) Wn[i] = w_at(i, m);
      const float inv = inv_at(m);
      float (&F)[D + 1] = side == 0 ? Fb : Fa;
      F[0] = Wn[1 + j];
#pragma unroll
      for (int i = 1; i < D + 1; ++i) {
        F[i] = (Wn[i] * inv) * Wn[1 + j];
        if (i - 1 == j) F[i] = F[i] + Wn[0];
      }
#pragma unroll
      for (int i = 0; i < D + 1; ++i) sum_w[i] = (m == 0) ? Wn[i] : sum_w[i] + Wn[i];
    }
#pragma unroll
    for (int i = 0; i < D + 1; ++i) sum_f[i] = (j == 0) ? Fb[i] - Fa[i] : sum_f[i] + (Fb[i] - Fa[i]);
  }
#pragma unroll
  for (int i = 0; i < D + 1; ++i) {
    const float w = w_at(i, -1);
    const float rest = w - ((i == 0) ? k.d2a_rho : k.d2a_q) * w;
    out[i] = (rest + ((i == 0) ? k.a_rho : k.a_q) * sum_w[i]) + k.c * sum_f[i];
  }
}

template <int D, typename WAt>
__device__ __forceinline__ void step_moments(WAt w_at, const Coef& k, float (&out)[D + 1]) {
  step_moments_inv<D>(w_at, [&](int m) { return recip_neq(w_at(0, m) + k.ref); }, k, out);
}

template <int D>
__device__ __forceinline__ void step_cell_mom(const float* __restrict__ sr, float* __restrict__ dr, int x, int y,
                                              int z, int nx, int ny, int nz, int64_t stride, const Coef& k) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  const int64_t c = static_cast<int64_t>(z) * plane + static_cast<int64_t>(y) * nx + x;
  int64_t src[2 * D];
  upwind_sources<D>(x, y, z, nx, ny, nz, c, src);
  float out[D + 1];
  step_moments<D>([&](int i, int nb) { return sr[i * stride + (nb < 0 ? c : src[nb])]; }, k, out);
#pragma unroll
  for (int i = 0; i < D + 1; ++i) store_stream(dr + i * stride + c, out[i]);
}

// ----------------------------------------------------------------------------
// Channel boundaries (2D, Section 5.2): inlet at x = 0 with a prescribed
// velocity profile, outlet at x = L with a prescribed density, walls at y = 0
// and y = L.  A population entering the domain comes from a ghost cell whose
// moments are second-order formulas in the interior moments; its value is the
// equilibrium of those moments (the non-equilibrium part of the first interior
// cell is added on the walls when `corr` is set).  Every moment here is that
// of the stored post-relaxation state, i.e. of the time level the step starts
// from (the relaxation does not change moments).
// ----------------------------------------------------------------------------
struct WallArgs {
  const double* u_in;  // [2][ny] inlet velocity (physical units), device memory
  double rho_out;      // outlet density target
  double u_bottom, u_top;
  double dx, rho_bar;
  int corr;
};

// moments (deviation form for W_rho) of the stored cell c
template <typename TR, typename TM, typename R>
__device__ __forceinline__ void cell_moments2(const TR* __restrict__ sr, const TM* __restrict__ sm, int64_t c,
                                              int64_t stride, R (&W)[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    R s = load_as<R>(sr + i * stride + c);
#pragma unroll
    for (int m = 0; m < 4; ++m) s = s + load_as<R>(sm + (i * 4 + m) * stride + c);
    W[i] = s;
  }
}

// Replace the entering populations of boundary cell (x, y) in the gathered g.
template <typename TR, typename TM, typename R>
__device__ __forceinline__ void wall_ghosts(const TR* __restrict__ sr, const TM* __restrict__ sm, int x, int y,
                                            int nx, int ny, int64_t stride, const CoefT<R>& k, const WallArgs& w,
                                            R (&g)[3][5]) {
  const int64_t c = static_cast<int64_t>(y) * nx + x;
  const R two = R(2);
  if (x == 0) {  // inlet: +x populations
    R a[3], b[3], Wg[3];
    cell_moments2<TR, TM, R>(sr, sm, c, stride, a);
    cell_moments2<TR, TM, R>(sr, sm, c + 1, stride, b);
    Wg[0] = two * a[0] - b[0];
    Wg[1] = static_cast<R>(2.0 * w.dx * w.rho_bar * w.u_in[y]) - a[1];
    Wg[2] = static_cast<R>(2.0 * w.dx * w.rho_bar * w.u_in[ny + y]) - a[2];
    const R inv = R(1) / (Wg[0] + k.ref);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i][1] = eq_moving<2, R>(Wg, inv, k, i, 0);
  }
  if (x == nx - 1) {  // outlet: -x populations
    R a[3], b[3], Wg[3];
    cell_moments2<TR, TM, R>(sr, sm, c, stride, a);
    cell_moments2<TR, TM, R>(sr, sm, c - 1, stride, b);
    Wg[0] = static_cast<R>(2.0 * (w.rho_out - static_cast<double>(k.ref))) - a[0];
    Wg[1] = two * a[1] - b[1];
    Wg[2] = two * a[2] - b[2];
    const R inv = R(1) / (Wg[0] + k.ref);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i][2] = eq_moving<2, R>(Wg, inv, k, i, 1);
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {  // lower wall: +y populations; upper wall: -y
    const bool on = side == 0 ? (y == 0) : (y == ny - 1);
    if (!on) continue;
    const int m = side == 0 ? 2 : 3;
    const int64_t inner = side == 0 ? c + nx : c - nx;
    R a[3], b[3], Wg[3];
    cell_moments2<TR, TM, R>(sr, sm, c, stride, a);
    cell_moments2<TR, TM, R>(sr, sm, inner, stride, b);
    Wg[0] = two * a[0] - b[0];
    Wg[1] = static_cast<R>(2.0 * w.dx * w.rho_bar * (side == 0 ? w.u_bottom : w.u_top)) - a[1];
    Wg[2] = -a[2];
    const R inv = R(1) / (Wg[0] + k.ref);
    const R inv_a = R(1) / (a[0] + k.ref);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R v = eq_moving<2, R>(Wg, inv, k, i, m);
      if (w.corr) v = v + (load_as<R>(sm + (i * 4 + m) * stride + c) - eq_moving<2, R>(a, inv_a, k, i, m));
      g[i][1 + m] = v;
    }
  }
}

}  // namespace lbm
