// Device kernels of the batched augmented-GMRES field solver (Alg. 1, Sec. 3.1).
//
// Every kernel covers a batch of systems: grid.y = system, grid.x = voxel chunk
// of kChunk voxels.  Blocks of systems whose flag is clear exit at once, so one
// launch per Krylov step serves every unconverged system.  Inner products are
// written as per-chunk FP64 partial sums and reduced, in a fixed order, by
// k_reduce (one wave per system), which also runs the small per-system FP64
// algebra (Givens rotations, k x k triangular solves).
#pragma once

#include "common.h"
#include "krylov_index.h"

namespace hydot {

constexpr int kVPT = 8;                    // voxels per thread
constexpr int kChunk = kBlock * kVPT;      // voxels per block
static_assert(kChunk == kChunkVoxels, "chunk size shared with the index arithmetic");

// Per-system constants (host-built).  Internal order of a batch is rhs-major so
// the wavelengths of one right-hand side, which share U and C, are adjacent.
struct SysParam {
  cd sig;            // sigma_j = (mu_a + i omega/nu)/D
  double sigp_abs;   // sigma'_j (Robin shift in the operator)
  double sigp_rel;   // sigma'_j - mean sigma' (Robin shift relative to K_hat = K + mean R)
  double out_scale;  // 1/(D_j h^3): phi = x * out_scale
  double tau_abs;    // absorption-perturbation weight in the operator (0 without one)
  double tau_rel;    // tau_abs minus the part included in K_hat
  int32_t rhs;       // index of the right-hand side in the U/C buffers
  int32_t voxel;     // injection voxel
  int32_t lam;       // wavelength index
  int32_t gsys;      // lambda*n_rhs + r in the output
};

struct SysState {
  int32_t in_sweep;     // still iterating (outer FP64 refinement)
  int32_t in_inner;     // inner solve of this sweep not finished
  int32_t in_cycle;     // stepping inside the current restart cycle
  int32_t cyc_ran;      // the current cycle was started (needs its update)
  int32_t nsteps;       // Arnoldi steps taken in the current cycle
  int32_t total_iters;  // Arnoldi steps over all cycles
  int32_t converged;    // FP64 residual met the tolerance
  int32_t sweeps;       // outer sweeps started
  int32_t stalls;       // sweeps that failed to reduce the outer residual
  int32_t reorth;       // the second Gram-Schmidt pass of the current step is applied
  double rnorm_outer;   // ||b - A x|| (FP64) at the start of the sweep
  double target_in;     // absolute target of the inner residual (inner rhs has norm 1)
  double beta;          // ||deflated residual|| at cycle start
  double resid_est;     // |gamma_{j+1}|
  double inner_rnorm;   // inner residual at the last cycle start
  double prev_outer;    // outer residual of the previous sweep
};

template <typename S>
struct Ctx {
  using R = typename Store<S>::real;
  GridP g;
  int k;            // deflation dimension (0: none)
  int mkmax;        // slot stride of the basis dots
  int nchunks;
  const SysParam* prm;
  SysState* st;
  S* V;             // [nb][vdim][N]
  int vdim;
  S* W;             // [nb][N] work vector
  S* Din;           // [nb][N] inner correction
  S* Rin;           // [nb][N] inner right-hand side
  cd* X;            // [nb][N] FP64 iterate
  cd* Rout;         // [nb][N] FP64 residual
  const R* mu;      // [N] absorption-perturbation shape, or null
  const R* C;       // [n_rhs][k][N]
  const R* U;       // [n_rhs][k][N]
  cd* part;         // [nb][nchunks][ndots]
  int ndots;
  cd* small;        // [nb][sl.total]
  Small sl;
  int* counter;     // [2 + 3 kMaxMK]: in_sweep count, in_inner count, systems stepping at step j,
                    // systems re-orthogonalising at step j, right-hand sides stepping at step j
  S* Z = nullptr;   // [nb][N] preconditioned vector P^{-1} V_j (right preconditioning), or null
};

__device__ inline void wave_store(cd v, int slot, cd* lds) {
  const double re = wave_sum(v.re), im = wave_sum(v.im);
  if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * kMaxDots + slot] = cd{re, im};
}

// after __syncthreads(): sum the wave partials of slots [lo, hi) into out
__device__ inline void block_flush(const cd* lds, int lo, int hi, cd* out) {
  for (int s = lo + (int)threadIdx.x; s < hi; s += kBlock) {
    cd a{0.0, 0.0};
#pragma unroll
    for (int w = 0; w < kWaves; ++w) a = a + lds[w * kMaxDots + s];
    out[s] = a;
  }
}

template <typename S>
struct Chunk {
  uint32_t n[kVPT];
  bool ok[kVPT];
  __device__ Chunk(const GridP& g) {
    const uint32_t base = blockIdx.x * kChunk + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kVPT; ++q) {
      n[q] = base + q * kBlock;
      ok[q] = n[q] < (uint32_t)g.N;
    }
  }
};

// Deflation dots f_i = C'_i^H w with C'_i = C_i + (sigma + xs) U_i formed per voxel (xs the
// voxel's relative real shift), basis dots V_l^H w for l < nv, and optionally ||w||^2,
// written as this chunk's partial sums.
template <typename S>
__device__ inline void chunk_dots(const Ctx<S>& c, int sys, const Chunk<S>& ch, const S* w,
                                  const double* xs, const S* Vsys, int nv, bool with_norm,
                                  cd* lds) {
  const size_t N = (size_t)c.g.N;
  if (c.k > 0) {
    const int r = c.prm[sys].rhs;
    const cd sig = c.prm[sys].sig;
    for (int i = 0; i < c.k; ++i) {
      const auto* Ci = c.C + ((size_t)r * c.k + i) * N;
      const auto* Ui = c.U + ((size_t)r * c.k + i) * N;
      cd a{0, 0};
#pragma unroll
      for (int q = 0; q < kVPT; ++q) {
        if (!ch.ok[q]) continue;
        const double cv = (double)Ci[ch.n[q]], uv = (double)Ui[ch.n[q]];
        const double ar = cv + (sig.re + xs[q]) * uv, ai = -sig.im * uv;   // conj(C'_i) at this voxel
        const double wr = (double)w[q].re, wi = (double)w[q].im;
        a.re += ar * wr - ai * wi;
        a.im += ar * wi + ai * wr;
      }
      wave_store(a, slot_defl(i, 0), lds);
    }
  }
  for (int l = 0; l < nv; ++l) {
    const S* Vl = Vsys + (size_t)l * N;
    cd a{0, 0};
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) dot_acc(a, Vl[ch.n[q]], w[q]);
    wave_store(a, slot_v(c.k, l), lds);
  }
  if (with_norm) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) a += nrm2(w[q]);
    wave_store(cd{a, 0.0}, slot_norm(c.k, c.mkmax), lds);
  }
  __syncthreads();
  cd* out = c.part + part_base(sys, c.nchunks, blockIdx.x, c.ndots);
  for (int i = threadIdx.x; i < c.k; i += kBlock) {
    cd a{0.0, 0.0};
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) a = a + lds[wv * kMaxDots + slot_defl(i, 0)];
    out[slot_defl(i, 0)] = a;
  }
  block_flush(lds, slot_v(c.k, 0), slot_v(c.k, nv), out);
  if (with_norm) block_flush(lds, slot_norm(c.k, c.mkmax), slot_norm(c.k, c.mkmax) + 1, out);
}

// w <- w - C' g - sum_l V_l h_l, where C' g = C g + (sigma + xs) U g per voxel and
// (optionally) acc_u += U g.  coef = [g (k), h (nv)] in FP64.
template <typename S>
__device__ inline void chunk_project(const Ctx<S>& c, int sys, const Chunk<S>& ch, S* w,
                                     const double* xs, const S* Vsys, int nv, const cd* coef,
                                     S* ug) {
  using R = typename Store<S>::real;
  const size_t N = (size_t)c.g.N;
  if (c.k > 0) {
    const int r = c.prm[sys].rhs;
    const cd sig = c.prm[sys].sig;
    S a[kVPT], b[kVPT];
#pragma unroll
    for (int q = 0; q < kVPT; ++q) {
      a[q] = Store<S>::zero();
      b[q] = Store<S>::zero();
    }
    for (int i = 0; i < c.k; ++i) {
      const R* Ci = c.C + ((size_t)r * c.k + i) * N;
      const R* Ui = c.U + ((size_t)r * c.k + i) * N;
      const cd gi = coef[i];
      const R gr = (R)gi.re, gim = (R)gi.im;
#pragma unroll
      for (int q = 0; q < kVPT; ++q) {
        if (!ch.ok[q]) continue;
        const R cv = Ci[ch.n[q]], uv = Ui[ch.n[q]];
        a[q].re += cv * gr;
        a[q].im += cv * gim;
        b[q].re += uv * gr;
        b[q].im += uv * gim;
      }
    }
#pragma unroll
    for (int q = 0; q < kVPT; ++q) {
      const cd shift{sig.re + xs[q], sig.im};
      // w -= a + shift * b
      w[q] = sub(w[q], a[q]);
      w[q] = axpy_neg(w[q], shift, b[q]);
      if (ug) ug[q] = add(ug[q], b[q]);
    }
  }
  for (int l = 0; l < nv; ++l) {
    const S* Vl = Vsys + (size_t)l * N;
    const cd hl = coef[c.k + l];
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) w[q] = axpy_neg(w[q], hl, Vl[ch.n[q]]);
  }
}

// relative real shift of each voxel of the chunk: sigma'_rel rho + tau_rel mu
template <typename S>
__device__ inline void load_xs(const Ctx<S>& c, const SysParam& p, const Chunk<S>& ch, double* xs) {
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    if (!ch.ok[q]) { xs[q] = 0.0; continue; }
    const VoxelInfo vi = voxel_info(c.g, ch.n[q]);
    xs[q] = p.sigp_rel * (double)vi.nrobin * c.g.inv_h + (c.mu ? p.tau_rel * (double)c.mu[ch.n[q]] : 0.0);
  }
}

// ------------------------------------------------------------------ kernels

// V_0 = e_voxel (unit scale) for the Lanczos (shift-invariant Krylov) runs.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_unit_v0(Ctx<S> c) {
  const int sys = blockIdx.y;
  const Chunk<S> ch(c.g);
  S* v0 = c.V + (size_t)sys * c.vdim * c.g.N;
  const uint32_t vox = (uint32_t)c.prm[sys].voxel;
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    if (!ch.ok[q]) continue;
    S z = Store<S>::zero();
    if (ch.n[q] == vox) z.re = 1;
    v0[ch.n[q]] = z;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c.small[(size_t)sys * c.sl.total + c.sl.vs] = cd{1.0, 0.0};
}

// X = 0 (no initial guess)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_zero_x(Ctx<S> c) {
  const int sys = blockIdx.y;
  const Chunk<S> ch(c.g);
  cd* x = c.X + (size_t)sys * c.g.N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) x[ch.n[q]] = cd{0.0, 0.0};
}

// X = V_L[rhs][0..nl) y0 (multi-shift initial guess, Alg. 1 step 5); VL holds
// the real shift-invariant basis as complex vectors with zero imaginary part.
template <typename S, typename VT>
__global__ __launch_bounds__(kBlock) void k_combine_x0(Ctx<S> c, const VT* VL, int vldim, int nl) {
  const int sys = blockIdx.y;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const cd* y0 = c.small + (size_t)sys * c.sl.total + c.sl.y0;
  const VT* Vb = VL + (size_t)c.prm[sys].rhs * vldim * N;
  cd acc[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) acc[q] = cd{0.0, 0.0};
  for (int l = 0; l < nl; ++l) {
    const cd yl = y0[l];
    const VT* Vl = Vb + (size_t)l * N;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) {
        const double v = (double)Vl[ch.n[q]];
        acc[q].re += v * yl.re;
        acc[q].im += v * yl.im;
      }
  }
  cd* x = c.X + (size_t)sys * N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) x[ch.n[q]] = acc[q];
}

// Rout = e_voxel - A_hat X in FP64, partial ||Rout||^2.  force: ignore flags.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_outer_resid(Ctx<S> c, int force) {
  __shared__ cd lds[kWaves * kMaxDots];
  const int sys = blockIdx.y;
  if (!force && !c.st[sys].in_sweep) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const SysParam p = c.prm[sys];
  const cd* x = c.X + (size_t)sys * N;
  cd* r = c.Rout + (size_t)sys * N;
  double a = 0.0;
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    if (!ch.ok[q]) continue;
    const VoxelInfo vi = voxel_info(c.g, ch.n[q]);
    cd ax = apply_op<cd>(c.g, x, ch.n[q], vi, p.sig, p.sigp_abs, c.mu ? p.tau_abs * (double)c.mu[ch.n[q]] : 0.0);
    cd rr{-ax.re, -ax.im};
    if (ch.n[q] == (uint32_t)p.voxel) rr.re += 1.0;
    r[ch.n[q]] = rr;
    a += norm2(rr);
  }
  wave_store(cd{a, 0.0}, 0, lds);
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += lds[w * kMaxDots].re;
    c.part[part_base(sys, c.nchunks, blockIdx.x, c.ndots) + slot_norm(c.k, c.mkmax)] = cd{t, 0.0};
  }
}

// Rin = Rout / ||Rout|| in the inner precision; Din = 0.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_rhs_in(Ctx<S> c) {
  const int sys = blockIdx.y;
  if (!c.st[sys].in_sweep) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const double inv = 1.0 / c.st[sys].rnorm_outer;
  const cd* r = c.Rout + (size_t)sys * N;
  S* ri = c.Rin + (size_t)sys * N;
  S* d = c.Din + (size_t)sys * N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) {
      ri[ch.n[q]] = Store<S>::from(inv * r[ch.n[q]]);
      d[ch.n[q]] = Store<S>::zero();
    }
}

// W = Rin - A_hat Din (inner precision); deflation dots and ||W||^2.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_inner_resid(Ctx<S> c) {
  __shared__ cd lds[kWaves * kMaxDots];
  const int sys = blockIdx.y;
  if (!c.st[sys].in_inner) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const SysParam p = c.prm[sys];
  const S* d = c.Din + (size_t)sys * N;
  const S* ri = c.Rin + (size_t)sys * N;
  S* wv = c.W + (size_t)sys * N;
  S w[kVPT];
  double xs[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    xs[q] = 0.0;
    w[q] = Store<S>::zero();
    if (!ch.ok[q]) continue;
    const VoxelInfo vi = voxel_info(c.g, ch.n[q]);
    const double mu = c.mu ? (double)c.mu[ch.n[q]] : 0.0;
    xs[q] = p.sigp_rel * (double)vi.nrobin * c.g.inv_h + p.tau_rel * mu;
    const S ad = apply_op<S>(c.g, d, ch.n[q], vi, p.sig, p.sigp_abs, p.tau_abs * mu);
    w[q] = sub(ri[ch.n[q]], ad);
    wv[ch.n[q]] = w[q];
  }
  chunk_dots<S>(c, sys, ch, w, xs, nullptr, 0, true, lds);
}

// Initial deflation (Alg. 1 step 9): Din += U g, W -= C' g, V_0 = W; ||V_0||^2.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_defl_start(Ctx<S> c) {
  __shared__ cd lds[kWaves * kMaxDots];
  const int sys = blockIdx.y;
  if (!c.st[sys].cyc_ran) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  S* wv = c.W + (size_t)sys * N;
  S* d = c.Din + (size_t)sys * N;
  S* v0 = c.V + (size_t)sys * c.vdim * N;
  S w[kVPT], ug[kVPT];
  double xs[kVPT];
  load_xs<S>(c, c.prm[sys], ch, xs);
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    w[q] = ch.ok[q] ? wv[ch.n[q]] : Store<S>::zero();
    ug[q] = Store<S>::zero();
  }
  chunk_project<S>(c, sys, ch, w, xs, nullptr, 0, coef, ug);
  double a = 0.0;
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    if (!ch.ok[q]) continue;
    v0[ch.n[q]] = w[q];
    if (c.k > 0) d[ch.n[q]] = add(d[ch.n[q]], ug[q]);
    a += nrm2(w[q]);
  }
  wave_store(cd{a, 0.0}, 0, lds);
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int wq = 0; wq < kWaves; ++wq) t += lds[wq * kMaxDots].re;
    c.part[part_base(sys, c.nchunks, blockIdx.x, c.ndots) + slot_norm(c.k, c.mkmax)] = cd{t, 0.0};
  }
}


// Arnoldi step j, first pass: W = A_hat V_j; dots against C', V_0..V_j.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_step_dots(Ctx<S> c, int j) {
  __shared__ cd lds[kWaves * kMaxDots];
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const SysParam p = c.prm[sys];
  const S* Vsys = c.V + (size_t)sys * c.vdim * N;
  const S* vj = Vsys + (size_t)j * N;
  S* wv = c.W + (size_t)sys * N;
  const double sj = c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re;   // v_j = sj * stored V_j
  S w[kVPT];
  double xs[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) {
    xs[q] = 0.0;
    w[q] = Store<S>::zero();
    if (!ch.ok[q]) continue;
    const VoxelInfo vi = voxel_info(c.g, ch.n[q]);
    const double mu = c.mu ? (double)c.mu[ch.n[q]] : 0.0;
    xs[q] = p.sigp_rel * (double)vi.nrobin * c.g.inv_h + p.tau_rel * mu;
    w[q] = scale(apply_op<S>(c.g, vj, ch.n[q], vi, p.sig, p.sigp_abs, p.tau_abs * mu), sj);
    wv[ch.n[q]] = w[q];
  }
  chunk_dots<S>(c, sys, ch, w, xs, Vsys, j + 1, false, lds);
}

// Arnoldi step j, first projection and second-pass dots (CGS2); w' is stored as V_{j+1}.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_step_update(Ctx<S> c, int j) {
  __shared__ cd lds[kWaves * kMaxDots];
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const S* Vsys = c.V + (size_t)sys * c.vdim * N;
  const S* wv = c.W + (size_t)sys * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  S w[kVPT];
  double xs[kVPT];
  load_xs<S>(c, c.prm[sys], ch, xs);
#pragma unroll
  for (int q = 0; q < kVPT; ++q) w[q] = ch.ok[q] ? wv[ch.n[q]] : Store<S>::zero();
  chunk_project<S>(c, sys, ch, w, xs, Vsys, j + 1, coef, nullptr);
  S* vn = c.V + ((size_t)sys * c.vdim + j + 1) * N;   // w' becomes V_{j+1} (scaled or re-orthogonalised later)
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) vn[ch.n[q]] = w[q];
  chunk_dots<S>(c, sys, ch, w, xs, Vsys, j + 1, true, lds);
}

// Arnoldi step j, second projection and normalisation, for the systems whose
// second Gram-Schmidt pass is applied: V_{j+1} = (w' - C'g2 - V h2)/eta in place.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_step_finish(Ctx<S> c, int j) {
  const int sys = blockIdx.y;
  if (!c.st[sys].in_cycle || !c.st[sys].reorth) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  S* Vsys = c.V + (size_t)sys * c.vdim * N;
  S* vn = Vsys + (size_t)(j + 1) * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefB;
  const double inv_eta = coef[c.k + c.mkmax + 1].re;
  S w[kVPT];
  double xs[kVPT];
  load_xs<S>(c, c.prm[sys], ch, xs);
#pragma unroll
  for (int q = 0; q < kVPT; ++q) w[q] = ch.ok[q] ? vn[ch.n[q]] : Store<S>::zero();
  chunk_project<S>(c, sys, ch, w, xs, Vsys, j + 1, coef, nullptr);
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) vn[ch.n[q]] = scale(w[q], inv_eta);
}

// End of cycle (Alg. 1 step 11): Din += U z + V y2.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_cycle_update(Ctx<S> c) {
  using R = typename Store<S>::real;
  const int sys = blockIdx.y;
  if (!c.st[sys].cyc_ran) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const int ns = c.st[sys].nsteps;
  const S* Vsys = c.V + (size_t)sys * c.vdim * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  S* d = c.Din + (size_t)sys * N;
  S acc[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) acc[q] = ch.ok[q] ? d[ch.n[q]] : Store<S>::zero();
  if (c.k > 0) {
    const int r = c.prm[sys].rhs;
    for (int i = 0; i < c.k; ++i) {
      const R* Ui = c.U + ((size_t)r * c.k + i) * N;
      const cd zi = coef[i];
      const cd mz{-zi.re, -zi.im};
#pragma unroll
      for (int q = 0; q < kVPT; ++q)
        if (ch.ok[q]) {
          const R u = Ui[ch.n[q]];
          S us;
          us.re = u;
          us.im = 0;
          acc[q] = axpy_neg(acc[q], mz, us);
        }
    }
  }
  if (c.Z != nullptr) {
    // right preconditioning: the basis part of the update is P^{-1} (V y2), formed beforehand
    const S* z = c.Z + (size_t)sys * N;
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) acc[q] = add(acc[q], z[ch.n[q]]);
  } else {
    for (int l = 0; l < ns; ++l) {
      const S* Vl = Vsys + (size_t)l * N;
      const cd yl = coef[c.k + l];
      const cd my{-yl.re, -yl.im};
#pragma unroll
      for (int q = 0; q < kVPT; ++q)
        if (ch.ok[q]) acc[q] = axpy_neg(acc[q], my, Vl[ch.n[q]]);
    }
  }
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) d[ch.n[q]] = acc[q];
}

// X += ||Rout|| * Din (FP64 refinement update)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_outer_update(Ctx<S> c) {
  const int sys = blockIdx.y;
  if (!c.st[sys].in_sweep) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const double s = c.st[sys].rnorm_outer;
  cd* x = c.X + (size_t)sys * N;
  const S* d = c.Din + (size_t)sys * N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) {
      const cd dd = Store<S>::to_cd(d[ch.n[q]]);
      x[ch.n[q]] = x[ch.n[q]] + s * dd;
    }
}

// phi[gsys] = X * out_scale in the output precision
template <typename S, typename O>
__global__ __launch_bounds__(kBlock) void k_output(Ctx<S> c, O* phi) {
  const int sys = blockIdx.y;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const SysParam p = c.prm[sys];
  const cd* x = c.X + (size_t)sys * N;
  O* out = phi + (size_t)p.gsys * N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) out[ch.n[q]] = Store<O>::from(p.out_scale * x[ch.n[q]]);
}

constexpr int kCounters = 2 + 3 * kMaxMK;

__global__ void k_zero_counters(int* counter) {
  for (int i = threadIdx.x; i < kCounters; i += blockDim.x) counter[i] = 0;
}

// ----------------------------------------------------------- reduce phases
enum Phase : int {
  PH_OUTER = 0,
  PH_START_A = 1,
  PH_START_B = 2,
  PH_STEP_A = 3,
  PH_STEP_B = 4,
  PH_CYCLE_END = 5,
  PH_FINAL = 6
};

struct ReduceArgs {
  double tol;          // outer relative tolerance
  double inner_floor;  // lowest inner relative target (mixed precision)
  int max_iter;
  int max_sweeps;
  int mk;              // Arnoldi steps per cycle
  int lanczos;         // 1: plain Arnoldi/Lanczos recording, no Givens, no stopping test
  double cgs_tau;      // > 0: skip the second Gram-Schmidt pass when its projection is below
                       // cgs_tau * ||w'|| (the basis is then orthogonal to working precision)
  double* final_res;   // PH_FINAL: per-system residual norms (device)
  int count_rhs;       // PH_STEP_A: also count the distinct right-hand sides stepping (measurement)
};

// g = G^-1 f with G = L L^H (lower L, column-major k x k)
__device__ inline void gsolve(int k, const cd* L, const cd* f, cd* g) {
  for (int i = 0; i < k; ++i) {
    cd s = f[i];
    for (int q = 0; q < i; ++q) s = s - L[i + k * q] * g[q];
    const double d = L[i + k * i].re;
    g[i] = cd{s.re / d, s.im / d};
  }
  for (int i = k - 1; i >= 0; --i) {
    cd s = g[i];
    for (int q = i + 1; q < k; ++q) s = s - conj(L[q + k * i]) * g[q];
    const double d = L[i + k * i].re;
    g[i] = cd{s.re / d, s.im / d};
  }
}

// The deflation partials hold f_i = C'_i^H w in slot_defl(i, 0).
template <typename S>
__global__ __launch_bounds__(64) void k_reduce(Ctx<S> c, ReduceArgs ra, int phase, int j) {
  __shared__ cd sum[kMaxDots];
  __shared__ cd tmp[2 * kMaxK + kMaxMK + 4];
  const int sys = blockIdx.x;
  SysState* st = c.st + sys;
  const SysParam p = c.prm[sys];
  // which systems take part in this phase
  bool act;
  switch (phase) {
    case PH_OUTER: act = st->in_sweep != 0; break;
    case PH_START_A: act = st->in_sweep != 0; break;
    case PH_START_B: act = st->cyc_ran != 0; break;
    case PH_STEP_A:
    case PH_STEP_B: act = st->in_cycle != 0; break;
    case PH_CYCLE_END: act = st->cyc_ran != 0; break;
    default: act = true; break;
  }
  if (!act) return;
  if (phase == PH_STEP_A && ra.count_rhs) {
    // count this system if it is the first stepping system of its right-hand side (the
    // systems of one right-hand side are contiguous in a batch)
    const int lane = threadIdx.x, r = p.rhs;
    bool earlier = false;
    for (int s0 = sys - 1; s0 >= 0; s0 -= 64) {
      const int s = s0 - lane;
      const bool same = s >= 0 && c.prm[s].rhs == r;
      if (__any(same && c.st[s].in_cycle)) {
        earlier = true;
        break;
      }
      if (!__all(same)) break;
    }
    if (lane == 0 && !earlier) atomicAdd(&c.counter[2 + 2 * kMaxMK + j], 1);
  }
  cd* sm = c.small + (size_t)sys * c.sl.total;
  const cd* part = c.part + part_base(sys, c.nchunks, 0, c.ndots);
  const int k = c.k;
  // slots needed by the phase
  int lo = 0, hi = 0;
  bool need_norm = false, need_defl = false;
  switch (phase) {
    case PH_OUTER: case PH_START_B: case PH_FINAL: need_norm = true; break;
    case PH_START_A: need_norm = true; need_defl = true; break;
    case PH_STEP_A: need_defl = true; lo = slot_v(k, 0); hi = slot_v(k, j + 1); break;
    case PH_STEP_B: need_norm = true; need_defl = true; lo = slot_v(k, 0); hi = slot_v(k, j + 1); break;
    default: break;
  }
  const int sn = slot_norm(k, c.mkmax);
  for (int s = threadIdx.x; s < c.ndots; s += 64) {
    const bool want = (need_defl && s < 3 * k && s % 3 == 0) || (s >= lo && s < hi) ||
                      (need_norm && s == sn);
    cd a{0.0, 0.0};
    if (want) {
      // eight interleaved partial sums, so that the chunk loads overlap (fixed order)
      cd q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = cd{0.0, 0.0};
      int ck = 0;
      for (; ck + 8 <= c.nchunks; ck += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = q[u] + part[part_base(0, c.nchunks, ck + u, c.ndots) + s];
      for (; ck < c.nchunks; ++ck) q[0] = q[0] + part[part_base(0, c.nchunks, ck, c.ndots) + s];
      a = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    }
    sum[s] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;

  cd* f = tmp;            // k
  cd* g = tmp + kMaxK;    // k
  auto make_f = [&]() {   // f = C'^H w
    for (int i = 0; i < k; ++i) f[i] = sum[slot_defl(i, 0)];
  };
  const cd* Lc = sm + c.sl.Lc;

  switch (phase) {
    case PH_OUTER: {
      const double rn = sqrt(sum[sn].re);
      st->rnorm_outer = rn;
      st->cyc_ran = 0;
      st->in_cycle = 0;
      st->in_inner = 0;
      if (rn <= ra.tol) {
        st->converged = 1;
        st->in_sweep = 0;
      } else if (st->total_iters >= ra.max_iter || st->sweeps >= ra.max_sweeps || st->stalls >= 3) {
        st->in_sweep = 0;
      } else {
        if (st->sweeps > 0 && rn > 0.5 * st->prev_outer) st->stalls += 1;
        st->in_sweep = 1;
        st->in_inner = 1;
        double t = 0.5 * ra.tol / rn;
        if (t < ra.inner_floor) t = ra.inner_floor;
        st->target_in = t;
        st->prev_outer = rn;
        st->sweeps += 1;
        atomicAdd(&c.counter[0], 1);
      }
      break;
    }
    case PH_START_A: {
      if (!st->in_inner) {   // inner solve of this sweep already finished
        st->cyc_ran = 0;
        st->in_cycle = 0;
        break;
      }
      const double rn = sqrt(sum[sn].re);
      st->inner_rnorm = rn;
      if (rn <= st->target_in || st->total_iters >= ra.max_iter) {
        st->in_inner = 0;
        st->cyc_ran = 0;
        st->in_cycle = 0;
        break;
      }
      st->cyc_ran = 1;
      if (k > 0) {
        make_f();
        gsolve(k, Lc, f, g);
        for (int i = 0; i < k; ++i) sm[c.sl.coefA + i] = g[i];
      }
      break;
    }
    case PH_START_B: {
      const double beta = sqrt(sum[sn].re);
      st->beta = beta;
      st->nsteps = 0;
      cd* gam = sm + c.sl.gam;
      for (int i = 0; i <= ra.mk; ++i) gam[i] = cd{0.0, 0.0};
      gam[0] = cd{beta, 0.0};
      if (beta > 0.0 && beta > 1e-300) {
        st->in_cycle = 1;
        st->resid_est = beta;
        sm[c.sl.vs] = cd{1.0 / beta, 0.0};   // V_0 stays unnormalised: v_0 = V_0 / beta
      } else {
        st->in_cycle = 0;
        st->resid_est = 0.0;
      }
      break;
    }
    case PH_STEP_A: {
      atomicAdd(&c.counter[2 + j], 1);
      cd* coef = sm + c.sl.coefA;
      if (k > 0) {
        make_f();
        for (int i = 0; i < k; ++i) sm[small_Fp(c.sl, k, i, j)] = f[i];
        gsolve(k, Lc, f, g);
        for (int i = 0; i < k; ++i) coef[i] = g[i];
      }
      const cd* vs = sm + c.sl.vs;
      for (int l = 0; l <= j; ++l) {
        const double sl = vs[l].re;
        const cd h = sl * sum[slot_v(k, l)];   // v_l^H w from the stored V_l
        coef[k + l] = sl * h;                  // multiplier of the stored V_l
        sm[small_H(c.sl, c.mkmax, l, j)] = h;
      }
      // FP32 copy for the complex FP32 update kernels (read as block-uniform scalars there)
      cf* c32 = reinterpret_cast<cf*>(sm + c.sl.cA32);
      for (int i = 0; i < k + j + 1; ++i) c32[i] = cf{(float)coef[i].re, (float)coef[i].im};
      break;
    }
    case PH_STEP_B: {
      cd* coef = sm + c.sl.coefB;
      cd* vs = sm + c.sl.vs;
      // second-pass coefficients (f2 -> g2, h2) and the norm of their projection
      double proj = 0.0;
      if (k > 0) {
        make_f();
        gsolve(k, Lc, f, g);
        for (int i = 0; i < k; ++i) proj += (conj(f[i]) * g[i]).re;
      }
      cd* h2 = tmp + 2 * kMaxK;
      for (int l = 0; l <= j; ++l) {
        h2[l] = vs[l].re * sum[slot_v(k, l)];
        proj += norm2(h2[l]);
      }
      const double w2 = sum[sn].re;   // ||w'||^2 after the first pass
      double eta;
      if (ra.cgs_tau > 0.0 && proj <= ra.cgs_tau * ra.cgs_tau * w2) {
        // w' is orthogonal to working precision: keep it unnormalised as V_{j+1}
        st->reorth = 0;
        eta = w2 > 0.0 ? sqrt(w2) : 0.0;
        vs[j + 1] = cd{eta > 1e-300 ? 1.0 / eta : 0.0, 0.0};
      } else {
        st->reorth = 1;
        atomicAdd(&c.counter[2 + kMaxMK + j], 1);
        if (k > 0) {
          for (int i = 0; i < k; ++i) {
            sm[small_Fp(c.sl, k, i, j)] = sm[small_Fp(c.sl, k, i, j)] + f[i];
            coef[i] = g[i];
          }
        }
        for (int l = 0; l <= j; ++l) {
          coef[k + l] = vs[l].re * h2[l];
          sm[small_H(c.sl, c.mkmax, l, j)] = sm[small_H(c.sl, c.mkmax, l, j)] + h2[l];
        }
        const double e2 = w2 - proj;
        eta = e2 > 0.0 ? sqrt(e2) : 0.0;
        vs[j + 1] = cd{1.0, 0.0};       // the second pass writes V_{j+1} normalised
      }
      sm[small_H(c.sl, c.mkmax, j + 1, j)] = cd{eta, 0.0};
      const bool breakdown = !(eta > 1e-300);
      coef[k + c.mkmax + 1] = cd{breakdown ? 0.0 : 1.0 / eta, 0.0};
      st->total_iters += 1;
      st->nsteps = j + 1;
      if (ra.lanczos) {
        // the last step still writes V_{n+1}: C = V_{n+1} Q needs it
        if (breakdown) st->in_cycle = 0;
        break;
      }
      // apply the previous rotations to column j, then a new one
      double* cs = (double*)(sm + c.sl.cs);   // stored in the .re slots (stride 2)
      cd* snv = sm + c.sl.sn;
      cd* gam = sm + c.sl.gam;
      for (int i = 0; i < j; ++i) {
        const double ci = cs[2 * i];
        const cd si = snv[i];
        const cd h1 = sm[small_H(c.sl, c.mkmax, i, j)], h2 = sm[small_H(c.sl, c.mkmax, i + 1, j)];
        sm[small_H(c.sl, c.mkmax, i, j)] = ci * h1 + si * h2;
        sm[small_H(c.sl, c.mkmax, i + 1, j)] = ci * h2 - conj(si) * h1;
      }
      {
        const cd a = sm[small_H(c.sl, c.mkmax, j, j)], b = sm[small_H(c.sl, c.mkmax, j + 1, j)];
        const double aa = sqrt(norm2(a)), bb = sqrt(norm2(b));
        const double rr = sqrt(aa * aa + bb * bb);
        double cj;
        cd sj;
        if (aa == 0.0) {
          cj = 0.0;
          sj = cd{1.0, 0.0};
        } else {
          cj = aa / rr;
          const cd ph{a.re / aa, a.im / aa};
          sj = (1.0 / rr) * (ph * conj(b));
        }
        cs[2 * j] = cj;
        snv[j] = sj;
        sm[small_H(c.sl, c.mkmax, j, j)] = cj * a + sj * b;
        sm[small_H(c.sl, c.mkmax, j + 1, j)] = cd{0.0, 0.0};
        const cd g0 = gam[j];
        gam[j] = cj * g0;
        gam[j + 1] = cd{0.0, 0.0} - conj(sj) * g0;
      }
      const double est = sqrt(norm2(gam[j + 1]));
      st->resid_est = est;
      if (est <= st->target_in || j + 1 >= ra.mk || st->total_iters >= ra.max_iter || breakdown)
        st->in_cycle = 0;
      break;
    }
    case PH_CYCLE_END: {
      const int ns = st->nsteps;
      const cd* gam = sm + c.sl.gam;
      cd* y = tmp + 2 * kMaxK;   // ns
      for (int i = ns - 1; i >= 0; --i) {
        cd s = gam[i];
        for (int q = i + 1; q < ns; ++q) s = s - sm[small_H(c.sl, c.mkmax, i, q)] * y[q];
        const cd d = sm[small_H(c.sl, c.mkmax, i, i)];
        const double dn = norm2(d);
        y[i] = dn > 0.0 ? (1.0 / dn) * (s * conj(d)) : cd{0.0, 0.0};
      }
      cd* coef = sm + c.sl.coefA;
      if (k > 0) {
        for (int i = 0; i < k; ++i) {
          cd s{0.0, 0.0};
          for (int q = 0; q < ns; ++q) s = s + sm[small_Fp(c.sl, k, i, q)] * y[q];
          f[i] = s;
        }
        gsolve(k, Lc, f, g);
        for (int i = 0; i < k; ++i) coef[i] = cd{-g[i].re, -g[i].im};
      }
      const cd* vs = sm + c.sl.vs;
      for (int q = 0; q < ns; ++q) coef[k + q] = vs[q].re * y[q];
      if (st->resid_est <= st->target_in || st->total_iters >= ra.max_iter || ns == 0) st->in_inner = 0;
      if (st->in_inner) atomicAdd(&c.counter[1], 1);
      break;
    }
    case PH_FINAL: {
      ra.final_res[sys] = sqrt(sum[sn].re);
      break;
    }
    default: break;
  }
}

}  // namespace hydot
