// Real shift-invariant Lanczos on K_hat (Alg. 1 step 1).  K_hat = Kt + mean(sigma') R
// (or Kt without the mean shift) is real symmetric and the right-hand sides are unit
// injections, so the basis is real: it is stored as real FP32 for the mixed path and
// real FP64 for the FP64 path (a quarter and a half of the complex FP64 bytes).
// Full reorthogonalisation (two classical Gram-Schmidt passes per step).  The kernels
// write per-chunk FP64 partial sums in the layout of the Arnoldi kernels with k = 0,
// so k_reduce in its Lanczos mode records the tridiagonal T_bar and the scales.
#pragma once

#include "krylov_kernels.h"

namespace hydot {

template <typename T>
struct LzCtx {
  GridP g;
  int nchunks, vdim, ndots;
  double sigp;          // Robin shift of K_hat (absolute)
  double tau;           // absorption-perturbation weight in K_hat (its mean over wavelengths)
  const T* mu;          // [N] perturbation shape, or null
  const SysParam* prm;  // injection voxel
  const SysState* st;
  T* V;                 // [nr][vdim][N]
  T* W;                 // [nr][N]
  cd* part;             // [nr][nchunks][ndots]
  const cd* small;      // per-system coefficients written by k_reduce
  Small sl;
  int mkmax;
};

// (K_hat x)_n, real: the stencil of apply_op with sigma = 0 and an extra real diagonal term
template <typename T>
__device__ inline double lz_apply(const GridP& g, const T* __restrict__ x, uint32_t n, const VoxelInfo& vi,
                                  double sigp, double extra) {
  const double xc = (double)x[n];
  double a = 0.0;
  int nn = 0;
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  if (vi.i > 0) { a -= (double)x[n - 1]; ++nn; }
  if (vi.i < g.nx - 1) { a -= (double)x[n + 1]; ++nn; }
  if (vi.j > 0) { a -= (double)x[n - sy]; ++nn; }
  if (vi.j < g.ny - 1) { a -= (double)x[n + sy]; ++nn; }
  if (vi.k > 0) { a -= (double)x[n - sz]; ++nn; }
  if (vi.k < g.nz - 1) { a -= (double)x[n + sz]; ++nn; }
  return g.inv_h2 * ((double)(nn + 2 * vi.ndir) * xc + a) + (sigp * (double)vi.nrobin * g.inv_h + extra) * xc;
}

// per-wave FP64 sums of slots [0, ns) to LDS, then per-block partials to part
template <int NS>
struct LzRed {
  double s[kWaves][NS];
};

template <int NS>
__device__ inline void lz_put(LzRed<NS>& r, int slot, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) r.s[threadIdx.x >> 6][slot] = v;
}

template <int NS>
__device__ inline void lz_flush(const LzRed<NS>& r, int nslots, int norm_slot, cd* out, int norm_out) {
  for (int s = threadIdx.x; s < nslots; s += kBlock) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) a += r.s[w][s];
    out[s == norm_slot ? norm_out : s] = cd{a, 0.0};
  }
}

// V_0 = e_voxel with unit scale
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_v0(LzCtx<T> c, cd* small) {
  const int sys = blockIdx.y;
  const Chunk<cd> ch(c.g);
  T* v0 = c.V + (size_t)sys * c.vdim * c.g.N;
  const uint32_t vox = (uint32_t)c.prm[sys].voxel;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) v0[ch.n[q]] = ch.n[q] == vox ? (T)1 : (T)0;
  if (blockIdx.x == 0 && threadIdx.x == 0) small[(size_t)sys * c.sl.total + c.sl.vs] = cd{1.0, 0.0};
}

// step j, first pass: W = K_hat v_j, partials V_l . W for l <= j
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_dots(LzCtx<T> c, int j) {
  __shared__ LzRed<kMaxMK + 2> red;
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle) return;
  const Chunk<cd> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const T* Vs = c.V + (size_t)sys * c.vdim * N;
  T* wv = c.W + (size_t)sys * N;
  const double sj = c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re;
  T w[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    w[q] = (T)0;
    if (!ch.ok[q]) continue;
    const VoxelInfo vi = voxel_info(c.g, ch.n[q]);
    const double extra = c.mu ? c.tau * (double)c.mu[ch.n[q]] : 0.0;
    w[q] = (T)(sj * lz_apply<T>(c.g, Vs + (size_t)j * N, ch.n[q], vi, c.sigp, extra));
    wv[ch.n[q]] = w[q];
  }
  for (int l = 0; l <= j; ++l) {
    const T* Vl = Vs + (size_t)l * N;
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) a += (double)(Vl[ch.n[q]] * w[q]);
    lz_put(red, l, a);
  }
  __syncthreads();
  lz_flush(red, j + 1, -1, c.part + part_base(sys, c.nchunks, blockIdx.x, c.ndots), 0);
}

// step j, first projection (w' = W - sum coefA_l V_l, stored as V_{j+1}) and second-pass
// partials V_l . w' plus |w'|^2
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_update(LzCtx<T> c, int j) {
  __shared__ LzRed<kMaxMK + 2> red;
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle) return;
  const Chunk<cd> ch(c.g);
  const size_t N = (size_t)c.g.N;
  T* Vs = c.V + (size_t)sys * c.vdim * N;
  const T* wv = c.W + (size_t)sys * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  T w[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) w[q] = ch.ok[q] ? wv[ch.n[q]] : (T)0;
  for (int l = 0; l <= j; ++l) {
    const T* Vl = Vs + (size_t)l * N;
    const T hl = (T)coef[l].re;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) w[q] -= hl * Vl[ch.n[q]];
  }
  T* vn = Vs + (size_t)(j + 1) * N;
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) {
      vn[ch.n[q]] = w[q];
      nrm += (double)w[q] * (double)w[q];
    }
  for (int l = 0; l <= j; ++l) {
    const T* Vl = Vs + (size_t)l * N;
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) a += (double)(Vl[ch.n[q]] * w[q]);
    lz_put(red, l, a);
  }
  lz_put(red, j + 1, nrm);
  __syncthreads();
  lz_flush(red, j + 2, j + 1, c.part + part_base(sys, c.nchunks, blockIdx.x, c.ndots), slot_norm(0, c.mkmax));
}

// step j, second projection and normalisation of V_{j+1} in place
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lz_finish(LzCtx<T> c, int j) {
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle || !c.st[sys].reorth) return;
  const Chunk<cd> ch(c.g);
  const size_t N = (size_t)c.g.N;
  T* Vs = c.V + (size_t)sys * c.vdim * N;
  T* vn = Vs + (size_t)(j + 1) * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefB;
  const T inv_eta = (T)coef[c.mkmax + 1].re;
  T w[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) w[q] = ch.ok[q] ? vn[ch.n[q]] : (T)0;
  for (int l = 0; l <= j; ++l) {
    const T* Vl = Vs + (size_t)l * N;
    const T hl = (T)coef[l].re;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) w[q] -= hl * Vl[ch.n[q]];
  }
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) vn[ch.n[q]] = w[q] * inv_eta;
}

}  // namespace hydot
