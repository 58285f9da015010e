// Separable right preconditioner for the shifted systems of Algorithm 1, a GPU-friendly
// replacement for the incomplete LU factorisation of the mean-shifted matrix that the
// paper uses (Sec. 6.1).
//
// On the box the mean-shifted stiffness K_hat = K~ + sigma*' rho is a Kronecker sum of three
// real symmetric tridiagonal matrices, T_x (+) T_y (+) T_z (each axis: path Laplacian / h^2
// with the Dirichlet end terms, plus sigma*' / h on its Robin ends), so
//   P_j = K_hat + sigma_j I = (Q_z (x) Q_y (x) Q_x) (Lz (+) Ly (+) Lx + sigma_j) (Q_z (x) Q_y (x) Q_x)^T
// is inverted exactly by three 1-D eigenvector transforms, a diagonal scaling and the
// three inverse transforms.  What it leaves out of A_j is (sigma'_j - sigma*') rho and the
// heterogeneous absorption tau_j mu, so A_j P_j^{-1} = I + (a boundary and an anomaly term)
// and GMRES needs a few iterations.  sigma_j is the system's own shift, or one shift for all
// systems (the mean over the wavelengths: a single preconditioner, as the paper's ILU).
//
// Each transform is one kernel over lines of the grid along one axis: a block loads a tile
// of lines into LDS (coalesced along x), multiplies by the n x n eigenvector matrix with a
// 4 x 4 register tile per thread (FP32, the matrix read through the cache), and stores the
// tile back, in place or into another array.  The z pass does the forward transform, the
// scaling and the inverse transform in one kernel.
#pragma once

#include "krylov_kernels.h"

namespace hydot {

constexpr int kPrecTile = 4096;   // complex values per LDS tile (32 KB)
constexpr int kPrecMaxN = 256;    // longest grid axis handled

struct PrecAxis {
  const float* Qf;   // [n][n4]: Qf[i * n4 + a] = component i of eigenvector a (zero padded)
  const float* Qi;   // [n][n4]: Qi[a * n4 + i] = component i of eigenvector a
  const float* lam;  // [n] eigenvalues
  int n, n4;
};

struct PrecP {
  PrecAxis ax[3];
  int nx, ny, nz;
};

// Which vectors a launch transforms: system sys reads in + sys * in_stride and writes
// out + sys * out_stride; systems are skipped unless their state passes `pred`
// (0: every system, 1: stepping in the current cycle, 2: the current cycle ran).
struct PrecIO {
  const cf* in;
  cf* out;
  size_t in_stride, out_stride;
  const SysState* st;
  int pred;
  const SysParam* prm;   // per-system shift sigma_j (used when !fixed)
  cd sig_fixed;
  int fixed;
};

__device__ inline bool prec_active(const PrecIO& io, int sys) {
  if (io.pred == 0 || io.st == nullptr) return true;
  return io.pred == 1 ? io.st[sys].in_cycle != 0 : io.st[sys].cyc_ran != 0;
}

// first element and element stride of line l along AXIS
template <int AXIS>
__device__ inline void line_geom(const PrecP& pp, int l, size_t& base, size_t& stride) {
  if (AXIS == 0) {
    base = (size_t)l * pp.nx;
    stride = 1;
  } else if (AXIS == 1) {
    const int i = l % pp.nx, k = l / pp.nx;
    base = (size_t)i + (size_t)pp.nx * pp.ny * k;
    stride = (size_t)pp.nx;
  } else {
    base = (size_t)l;
    stride = (size_t)pp.nx * pp.ny;
  }
}

template <int AXIS>
__device__ inline int line_count(const PrecP& pp) {
  return AXIS == 0 ? pp.ny * pp.nz : AXIS == 1 ? pp.nx * pp.nz : pp.nx * pp.ny;
}

// tile element e <-> (i along the line, lt line in the tile): x lines are contiguous, so the
// x pass walks i fastest; the y and z passes walk neighbouring lines (neighbouring x) fastest
template <int AXIS>
__device__ inline void tile_elem(int e, int n, int tw, int& i, int& lt) {
  if (AXIS == 0) {
    lt = e / n;
    i = e - lt * n;
  } else {
    i = e / tw;
    lt = e - i * tw;
  }
}

// acc[r][c] = sum_i Q[i * n4 + a0 + r] * tile[i * tw + l0 + c]
__device__ inline void prec_gemm(const float* __restrict__ Q, const cf* tile, int n, int n4, int tw, int a0, int l0,
                                 cf (&acc)[4][4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = cf{0.f, 0.f};
  for (int i = 0; i < n; ++i) {
    const float4 q = *reinterpret_cast<const float4*>(Q + (size_t)i * n4 + a0);
    const cf* x = tile + i * tw + l0;
    const float qa[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cf xv = x[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[r][c].re += qa[r] * xv.re;
        acc[r][c].im += qa[r] * xv.im;
      }
    }
  }
}

// MODE 0: forward transform (Q^T) along AXIS; 1: inverse (Q); 2 (z only): forward, scale by
// 1 / (lx + ly + lz + sigma), inverse.
template <int AXIS, int MODE>
__global__ __launch_bounds__(256) void k_prec_axis(PrecP pp, PrecIO io) {
  __shared__ cf tile[kPrecTile];
  const int sys = blockIdx.y;
  if (!prec_active(io, sys)) return;
  const PrecAxis ax = pp.ax[AXIS];
  const int n = ax.n, n4 = ax.n4;
  const int tw = (kPrecTile / n4) & ~3;
  const int nlines = line_count<AXIS>(pp);
  const int lbeg = blockIdx.x * tw;
  if (lbeg >= nlines) return;
  const int lines = min(tw, nlines - lbeg);
  const cf* in = io.in + (size_t)sys * io.in_stride;
  cf* out = io.out + (size_t)sys * io.out_stride;
  const int t = threadIdx.x;
  for (int e = t; e < n * tw; e += 256) {
    int i, lt;
    tile_elem<AXIS>(e, n, tw, i, lt);
    cf v{0.f, 0.f};
    if (lt < lines) {
      size_t base, stride;
      line_geom<AXIS>(pp, lbeg + lt, base, stride);
      v = in[base + (size_t)i * stride];
    }
    tile[i * tw + lt] = v;
  }
  __syncthreads();
  const int ngr = n4 / 4;                    // output rows in groups of 4
  const int nthr = ngr * (tw / 4);           // <= 256 by the choice of tw
  const int ag = t % ngr, lg = t / ngr;
  const int a0 = 4 * ag, l0 = 4 * lg;
  cf acc[4][4];
  if (t < nthr) prec_gemm(MODE == 1 ? ax.Qi : ax.Qf, tile, n, n4, tw, a0, l0, acc);
  __syncthreads();
  if (MODE == 2) {
    if (t < nthr) {
      const cd sg = io.fixed ? io.sig_fixed : io.prm[sys].sig;
      const PrecAxis axx = pp.ax[0], axy = pp.ax[1];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int l = lbeg + l0 + c;
        const int li = l < nlines ? l : 0;
        const float lxy = axx.lam[li % pp.nx] + axy.lam[li / pp.nx];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = a0 + r;
          const float dre = (a < n ? ax.lam[a] : 0.f) + lxy + (float)sg.re, dim = (float)sg.im;
          const float inv = 1.f / (dre * dre + dim * dim);
          const cf v = acc[r][c];
          // v / (dre + i dim)
          const cf s{(v.re * dre + v.im * dim) * inv, (v.im * dre - v.re * dim) * inv};
          if (a < n) tile[a * tw + l0 + c] = s;
        }
      }
    }
    __syncthreads();
    if (t < nthr) prec_gemm(ax.Qi, tile, n, n4, tw, a0, l0, acc);
    __syncthreads();
  }
  if (t < nthr) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (a0 + r < n)
#pragma unroll
        for (int c = 0; c < 4; ++c) tile[(a0 + r) * tw + l0 + c] = acc[r][c];
  }
  __syncthreads();
  for (int e = t; e < n * tw; e += 256) {
    int i, lt;
    tile_elem<AXIS>(e, n, tw, i, lt);
    if (lt < lines) {
      size_t base, stride;
      line_geom<AXIS>(pp, lbeg + lt, base, stride);
      out[base + (size_t)i * stride] = tile[i * tw + lt];
    }
  }
}

// P^{-1} applied to one vector per system (io.in -> io.out; the passes after the first run in
// place on io.out).  Five launches on `stream`.
inline void prec_apply(const PrecP& pp, PrecIO io, int nb, hipStream_t stream) {
  auto tiles = [&](int axis, int nlines) {
    const int tw = (kPrecTile / pp.ax[axis].n4) & ~3;
    return dim3((unsigned)((nlines + tw - 1) / tw), (unsigned)nb);
  };
  const int lx = pp.ny * pp.nz, ly = pp.nx * pp.nz, lz = pp.nx * pp.ny;
  hipLaunchKernelGGL((k_prec_axis<0, 0>), tiles(0, lx), dim3(256), 0, stream, pp, io);
  PrecIO ip = io;
  ip.in = io.out;
  ip.in_stride = io.out_stride;
  hipLaunchKernelGGL((k_prec_axis<1, 0>), tiles(1, ly), dim3(256), 0, stream, pp, ip);
  hipLaunchKernelGGL((k_prec_axis<2, 2>), tiles(2, lz), dim3(256), 0, stream, pp, ip);
  hipLaunchKernelGGL((k_prec_axis<1, 1>), tiles(1, ly), dim3(256), 0, stream, pp, ip);
  hipLaunchKernelGGL((k_prec_axis<0, 1>), tiles(0, lx), dim3(256), 0, stream, pp, ip);
}

// Z = sum_l y_l V_l over the cycle's basis (coefficients of Alg. 1 step 11), for the systems
// whose cycle ran; with the preconditioner the update is Din += U z + P^{-1} Z.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_cycle_vy(Ctx<S> c, S* Z) {
  const int sys = blockIdx.y;
  if (!c.st[sys].cyc_ran) return;
  const Chunk<S> ch(c.g);
  const size_t N = (size_t)c.g.N;
  const int ns = c.st[sys].nsteps;
  const S* Vsys = c.V + (size_t)sys * c.vdim * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  S acc[kVPT];
#pragma unroll
  for (int q = 0; q < kVPT; ++q) acc[q] = Store<S>::zero();
  for (int l = 0; l < ns; ++l) {
    const S* Vl = Vsys + (size_t)l * N;
    const cd yl = coef[c.k + l];
    const cd my{-yl.re, -yl.im};
#pragma unroll
    for (int q = 0; q < kVPT; ++q)
      if (ch.ok[q]) acc[q] = axpy_neg(acc[q], my, Vl[ch.n[q]]);
  }
  S* z = Z + (size_t)sys * N;
#pragma unroll
  for (int q = 0; q < kVPT; ++q)
    if (ch.ok[q]) z[ch.n[q]] = acc[q];
}

// Host: eigen-decompositions of the three axis operators of K_hat = K~ + sigp_star rho
// (built on first use and cached in the operator for that sigp_star); fills pp.
hydot_status prec_prepare(const hydot_operator* op, double sigp_star, PrecP& pp);

}  // namespace hydot
