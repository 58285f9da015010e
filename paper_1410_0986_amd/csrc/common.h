// Shared device/host helpers of the hydot library: complex storage types,
// fast integer division, the matrix-free finite-volume operator, and wave64
// reductions.  Internal header; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/hydot.h"

namespace hydot {

constexpr int kBlock = 256;          // threads per block of the vector kernels
constexpr int kWaves = kBlock / 64;  // wave64 count per block

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};
using cd = cplx<double>;
using cf = cplx<float>;

__host__ __device__ inline cd cmk(double r, double i) { return cd{r, i}; }
__host__ __device__ inline cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd operator*(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__host__ __device__ inline cd conj(cd a) { return cd{a.re, -a.im}; }
__host__ __device__ inline double norm2(cd a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
__host__ __device__ inline cd cmulc(cd a, cd b) {
  return cd{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// ---------------------------------------------------------------- storage ops
// The Krylov kernels are written once for complex FP64 (cd) and complex FP32
// (cf) storage; arithmetic on vectors runs in the storage precision and every
// inner product accumulates in FP64.
template <typename S> struct Store;
template <> struct Store<cd> {
  using real = double;
  __device__ static inline cd zero() { return cd{0.0, 0.0}; }
  __device__ static inline cd from(cd a) { return a; }
  __device__ static inline cd to_cd(cd a) { return a; }
};
template <> struct Store<cf> {
  using real = float;
  __device__ static inline cf zero() { return cf{0.f, 0.f}; }
  __device__ static inline cf from(cd a) { return cf{(float)a.re, (float)a.im}; }
  __device__ static inline cd to_cd(cf a) { return cd{(double)a.re, (double)a.im}; }
};

// complex BF16 storage (re, im) of fields: written with round-to-nearest-even from
// FP32 and widened exactly on load
struct alignas(4) cbf {
  uint16_t re, im;
};
__device__ inline uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_value(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
template <> struct Store<cbf> {
  using real = float;
  __device__ static inline cbf from(cd a) { return cbf{bf16_bits((float)a.re), bf16_bits((float)a.im)}; }
  __device__ static inline cd to_cd(cbf a) { return cd{(double)bf16_value(a.re), (double)bf16_value(a.im)}; }
};

template <typename S>
__device__ inline S sub(S a, S b) { return S{a.re - b.re, a.im - b.im}; }
template <typename S>
__device__ inline S add(S a, S b) { return S{a.re + b.re, a.im + b.im}; }
// a - c*x with c complex (given in FP64, applied in storage precision)
template <typename S>
__device__ inline S axpy_neg(S a, cd c, S x) {
  using R = typename Store<S>::real;
  const R cr = (R)c.re, ci = (R)c.im;
  return S{a.re - (cr * x.re - ci * x.im), a.im - (cr * x.im + ci * x.re)};
}
// a - r*c*x with r real (storage precision) and c complex
template <typename S>
__device__ inline S axpy_neg_rc(S a, typename Store<S>::real r, cd c, S x) {
  using R = typename Store<S>::real;
  const R cr = (R)c.re * r, ci = (R)c.im * r;
  return S{a.re - (cr * x.re - ci * x.im), a.im - (cr * x.im + ci * x.re)};
}
template <typename S>
__device__ inline S scale(S a, double s) {
  using R = typename Store<S>::real;
  return S{(R)(a.re * s), (R)(a.im * s)};
}
// acc += conj(a) * b in FP64
template <typename S>
__device__ inline void dot_acc(cd& acc, S a, S b) {
  const double ar = a.re, ai = a.im, br = b.re, bi = b.im;
  acc.re += ar * br + ai * bi;
  acc.im += ar * bi - ai * br;
}
// acc += r * b in FP64 (r real)
template <typename S>
__device__ inline void rdot_acc(cd& acc, double r, S b) {
  acc.re += r * (double)b.re;
  acc.im += r * (double)b.im;
}
template <typename S>
__device__ inline double nrm2(S a) {
  const double r = a.re, i = a.im;
  return r * r + i * i;
}

// ------------------------------------------------------------ fast division
// Division by a runtime-invariant divisor with a multiply-high (round-up method
// of Granlund and Montgomery); valid for numerators below 2^31.
struct FastDiv {
  uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1ull);
  return f;
}
__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f) {
  const uint32_t hi = (uint32_t)(((uint64_t)n * (uint64_t)f.m) >> 32);
  return (hi + n) >> f.s;
}

// ------------------------------------------------------------- the operator
// Matrix-free finite-volume operator scaled by 1/(D h^3) (shift form of
// eq. multipleshifted):  A_hat x = Kt x + (sigma + sigma' rho) x  with
//   (Kt x)_n = (1/h^2) [ sum_{face nbrs m}(x_n - x_m) + 2 x_n per Dirichlet face ],
//   rho_n    = (number of Robin faces of n)/h.
struct GridP {
  int32_t nx, ny, nz;
  int32_t N;
  FastDiv dx, dxy;
  uint32_t robin;      // face mask (-x,+x,-y,+y,-z,+z)
  double inv_h2;       // 1/h^2
  double inv_h;        // 1/h
};

// Neighbour flags and boundary face counts of voxel n.
struct VoxelInfo {
  int32_t i, j, k;
  int32_t nrobin, ndir;
};
__host__ __device__ inline VoxelInfo voxel_info(const GridP& g, uint32_t n) {
  VoxelInfo v;
  const uint32_t kz = fdiv(n, g.dxy);
  const uint32_t rem = n - kz * (uint32_t)(g.nx * g.ny);
  const uint32_t jy = fdiv(rem, g.dx);
  v.i = (int32_t)(rem - jy * (uint32_t)g.nx);
  v.j = (int32_t)jy;
  v.k = (int32_t)kz;
  // exterior faces of the voxel as a mask (-x,+x,-y,+y,-z,+z), split by the Robin mask
  const uint32_t m = (uint32_t)(v.i == 0) | (uint32_t)(v.i == g.nx - 1) << 1 | (uint32_t)(v.j == 0) << 2 |
                     (uint32_t)(v.j == g.ny - 1) << 3 | (uint32_t)(v.k == 0) << 4 | (uint32_t)(v.k == g.nz - 1) << 5;
  v.nrobin = __builtin_popcount(m & g.robin);
  v.ndir = __builtin_popcount(m & ~g.robin & 0x3fu);
  return v;
}

// (A_hat x)_n for a system with shift sig (complex), absolute Robin shift sigp and an
// extra real diagonal term at this voxel (the absorption perturbation, 0 without one).
template <typename S>
__device__ inline S apply_op(const GridP& g, const S* __restrict__ x, uint32_t n,
                             const VoxelInfo& vi, cd sig, double sigp, double extra = 0.0) {
  using R = typename Store<S>::real;
  const S xc = x[n];
  R ar = 0, ai = 0;   // sum over neighbours of (x_n - x_m)
  int nn = 0;
  const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
  if (vi.i > 0) { const S m = x[n - sx]; ar -= m.re; ai -= m.im; ++nn; }
  if (vi.i < g.nx - 1) { const S m = x[n + sx]; ar -= m.re; ai -= m.im; ++nn; }
  if (vi.j > 0) { const S m = x[n - sy]; ar -= m.re; ai -= m.im; ++nn; }
  if (vi.j < g.ny - 1) { const S m = x[n + sy]; ar -= m.re; ai -= m.im; ++nn; }
  if (vi.k > 0) { const S m = x[n - sz]; ar -= m.re; ai -= m.im; ++nn; }
  if (vi.k < g.nz - 1) { const S m = x[n + sz]; ar -= m.re; ai -= m.im; ++nn; }
  const R diag_k = (R)(nn + 2 * vi.ndir);
  const R ih2 = (R)g.inv_h2;
  // diagonal shift: sigma + sigp * rho
  const R dr = (R)(sig.re + sigp * (double)vi.nrobin * g.inv_h + extra);
  const R di = (R)sig.im;
  S y;
  y.re = ih2 * (diag_k * xc.re + ar) + (dr * xc.re - di * xc.im);
  y.im = ih2 * (diag_k * xc.im + ai) + (dr * xc.im + di * xc.re);
  return y;
}

// ------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Error bookkeeping shared by the translation units of the library.
void set_error(const std::string& msg);
hydot_status fail(hydot_status st, const std::string& msg);
hydot_status hip_check(hipError_t e, const char* what);

}  // namespace hydot

#define HYDOT_HIP(call)                                          \
  do {                                                           \
    hipError_t _e = (call);                                      \
    if (_e != hipSuccess) return ::hydot::hip_check(_e, #call);  \
  } while (0)
