// Register-resident Arnoldi step kernels for complex FP32 storage (the batched
// mixed path).  A block walks its chunk in sub-tiles of kTSub voxels, one voxel
// per thread: the thread reads V_0..V_j, C and U of its voxel once from HBM into
// registers, applies the operator or the projection there, and writes one
// product per inner product into an LDS tile; the tile is then summed row by
// row (4-8 threads per row, FP64), so every lane stays busy and no per-product
// wave reduction is needed (the chunk-accumulating instances instead keep
// per-thread FP32 sums over the chunk and reduce once).  One HBM read of the
// basis per kernel replaces the double read of the generic CGS2 update.
//
// Grid: one dimension of nb * nchunks blocks, ordered in groups of grp systems
// (the wavelengths of one right-hand side when the batch holds whole
// right-hand sides): block b -> group b / (grp * nchunks), chunk
// (b / grp) % nchunks, system group * grp + b % grp, with the chunk position
// optionally permuted so that each XCD takes a slab of z-planes (tile_idx).
#pragma once

#include "krylov_kernels.h"

namespace hydot {

constexpr int kTSub = 128;                  // voxels per sub-tile = threads per block
constexpr int kTK = 10;                     // largest deflation dimension handled here (3k+1 <= 32 rows)
constexpr int kTNV = 32;                    // largest basis count handled here
constexpr int kTRows = 32;                  // rows of the product tile
static_assert(kChunk % kTSub == 0, "chunk must hold whole sub-tiles");
static_assert(16 + kTK + 1 <= kTRows, "single-round tile must hold 16 basis rows, k deflation rows and the norm");
static_assert(3 * kTK + 1 <= kTRows && kTNV <= kTRows, "product tile too small");

// Products of one sub-tile, one row per inner product, then reduced row-wise:
// thread t owns row t/TPR and sums its columns t%TPR, t%TPR+TPR, ... (FP64), keeping a
// running sum over the sub-tiles of the chunk.  With P > 1 the products of P
// neighbouring lanes are first summed across lanes (DPP, FP32) and one lane of
// each group writes the sum, so the tile has kTSub/P columns: a smaller tile
// lets more blocks share a CU's LDS.
template <int P>
struct ProdTile {
  static constexpr int cols = kTSub / P;
  static constexpr int pitch = cols + 4;
  cf p[kTRows * pitch];
};

// x + (x of lane t^1) and x + (x of lane t^2) within each quad of lanes
__device__ inline float dpp_add_xor1(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ inline float dpp_add_xor2(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, false));
}

// product v of this lane for tile row `row`; every lane of the block must call this
template <int P>
__device__ inline void put_product(ProdTile<P>& pt, int row, cf v) {
  const int t = threadIdx.x;
  if constexpr (P >= 2) {
    v.re = dpp_add_xor1(v.re);
    v.im = dpp_add_xor1(v.im);
  }
  if constexpr (P >= 4) {
    v.re = dpp_add_xor2(v.re);
    v.im = dpp_add_xor2(v.im);
  }
  if constexpr (P == 1) {
    pt.p[row * ProdTile<P>::pitch + t] = v;
  } else {
    if ((t & (P - 1)) == 0) pt.p[row * ProdTile<P>::pitch + t / P] = v;
  }
}

template <int TPR, int P>
__device__ inline void row_reduce(const ProdTile<P>& pt, int nrows, cd& acc) {
  const int t = threadIdx.x, row = t / TPR, seg = t % TPR;
  if (row >= nrows) return;
  const cf* r = pt.p + row * ProdTile<P>::pitch;
  double re = 0.0, im = 0.0;
#pragma unroll 8
  for (int i = 0; i < ProdTile<P>::cols / TPR; ++i) {
    const cf x = r[seg + TPR * i];
    re += (double)x.re;
    im += (double)x.im;
  }
  acc.re += re;
  acc.im += im;
}

// this block's (system, chunk): see tile_map
__device__ inline TileIdx tile_idx(int nchunks, int grp, int flags) {
  return tile_map(blockIdx.x, gridDim.x, nchunks, grp, flags);
}

// finish the TPR-thread row sums and store them as the chunk's partial sums;
// rows map to partial slots through slot0 (+row), the norm row to its own slot
template <int TPR>
__device__ inline void row_flush(const Ctx<cf>& c, int sys, int chunk, int nrows, int slot0, int norm_row, cd acc) {
#pragma unroll
  for (int off = 1; off < TPR; off <<= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  const int t = threadIdx.x, row = t / TPR;
  if ((t % TPR) != 0 || row >= nrows) return;
  c.part[part_base(sys, c.nchunks, chunk, c.ndots) + flush_rows_slot(row, slot0, norm_row, c.k, c.mkmax)] = acc;
}

template <int TPR>
__device__ inline void row_flush_v(const Ctx<cf>& c, int sys, int chunk, int nrows, cd acc) {
#pragma unroll
  for (int off = 1; off < TPR; off <<= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  const int t = threadIdx.x, row = t / TPR;
  if ((t % TPR) != 0 || row >= nrows) return;
  c.part[part_base(sys, c.nchunks, chunk, c.ndots) + flush_v_slot(row, c.k)] = acc;
}

// Single-round form (at most 16 basis vectors): rows [0, nv) V dots, [nv, nv+k)
// f = C'^H w, row nv+k the norm; all in one tile, flushed to their slots.
template <int TPR>
__device__ inline void row_flush_all(const Ctx<cf>& c, int sys, int chunk, int nv, int nrows, cd acc) {
#pragma unroll
  for (int off = 1; off < TPR; off <<= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  const int t = threadIdx.x, row = t / TPR;
  if ((t % TPR) != 0 || row >= nrows) return;
  c.part[part_base(sys, c.nchunks, chunk, c.ndots) + flush_all_slot(row, nv, c.k, c.mkmax)] = acc;
}

// Buffer-resource access (raw buffer loads): one 32-bit voxel byte offset in a VGPR
// serves every vector of a system, the vector's byte offset rides in an SGPR, and an
// offset past the end of the resource reads zero.  Each system's basis (and each
// right-hand side's C, U) must stay below 2 GiB; the host checks this.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kOutside = 0x80000000u;   // voxel offset beyond every resource
__device__ inline Rsrc make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline cf ld_cf(Rsrc r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
// non-temporal (streaming) form, for data read once per launch
__device__ inline cf ld_cf_nt(Rsrc r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 2));
}
__device__ inline float ld_f(Rsrc r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}

struct SysBuf {
  Rsrc V, C, U, W, M;   // M: absorption-perturbation shape (no records without one)
  Rsrc S;               // stencil source of the dots kernel: the basis, or P^{-1} V_j when preconditioned
  uint32_t sv, sc;      // bytes between basis vectors, between C (U) vectors
  bool pert, precond;
};
__device__ inline SysBuf sys_buf(const Ctx<cf>& c, int sys, int rhs) {
  const uint32_t N = (uint32_t)c.g.N;
  SysBuf b;
  b.sv = N * 8u;
  b.sc = N * 4u;
  b.V = make_rsrc(c.V + (size_t)sys * c.vdim * N, (uint32_t)c.vdim * b.sv);
  b.C = make_rsrc(c.C + (size_t)rhs * c.k * N, (uint32_t)c.k * b.sc);
  b.U = make_rsrc(c.U + (size_t)rhs * c.k * N, (uint32_t)c.k * b.sc);
  b.W = make_rsrc(c.W + (size_t)sys * N, b.sv);
  b.pert = c.mu != nullptr;
  b.M = make_rsrc(c.mu, b.pert ? N * 4u : 0u);
  b.precond = c.Z != nullptr;
  b.S = b.precond ? make_rsrc(c.Z + (size_t)sys * N, b.sv) : b.V;
  return b;
}
// The buffers of a system without an absorption perturbation or a preconditioner: the basis,
// C and U only (the other resources alias the basis and are never read).
__device__ inline SysBuf sys_buf_plain(const Ctx<cf>& c, int sys, int rhs) {
  const uint32_t N = (uint32_t)c.g.N;
  SysBuf b;
  b.sv = N * 8u;
  b.sc = N * 4u;
  b.V = make_rsrc(c.V + (size_t)sys * c.vdim * N, (uint32_t)c.vdim * b.sv);
  b.C = make_rsrc(c.C + (size_t)rhs * c.k * N, (uint32_t)c.k * b.sc);
  b.U = make_rsrc(c.U + (size_t)rhs * c.k * N, (uint32_t)c.k * b.sc);
  b.W = b.V;
  b.M = b.V;
  b.S = b.V;
  b.pert = false;
  b.precond = false;
  return b;
}
// shape value of voxel byte offset vo4 (0 without a perturbation)
__device__ inline float mu_at(const SysBuf& b, uint32_t vo4) { return b.pert ? ld_f(b.M, vo4, 0u) : 0.f; }
// per-voxel shift of C'_j: sigma + sigma'_rel rho + tau_rel mu
__device__ inline cd voxel_shift(const SysParam& p, double rho, float mu) {
  return cd{p.sig.re + p.sigp_rel * rho + p.tau_rel * (double)mu, p.sig.im};
}

template <int NV>
__device__ inline void load_basis(const SysBuf& b, uint32_t vo8, int nv, cf* vr) {
#pragma unroll
  for (int l = 0; l < NV; ++l) vr[l] = l < nv ? ld_cf(b.V, vo8, (uint32_t)l * b.sv) : cf{0.f, 0.f};
}

// Exactly NV basis vectors, V_0..V_{NV-2} streamed (read once per launch) and V_{NV-1} = V_j
// cached (it is also the stencil operand, whose neighbours other threads read).
template <int NV>
__device__ inline void load_basis_stream(const SysBuf& b, uint32_t vo8, cf* vr) {
#pragma unroll
  for (int l = 0; l < NV; ++l)
    vr[l] = l + 1 < NV ? ld_cf_nt(b.V, vo8, (uint32_t)l * b.sv) : ld_cf(b.V, vo8, (uint32_t)l * b.sv);
}
// non-temporal store of one complex FP32 value
__device__ inline void st_cf_nt(cf* p, cf v) {
  __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), reinterpret_cast<unsigned long long*>(p));
}

// C and U of one voxel into registers: KM slots, the first k live (all KM when EXACT)
template <int KM, bool EXACT>
__device__ inline void load_cu_k(const SysBuf& b, int k, uint32_t vo4, float* cr, float* ur) {
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    const bool on = EXACT || i < k;
    cr[i] = on ? ld_f(b.C, vo4, (uint32_t)i * b.sc) : 0.f;
    ur[i] = on ? ld_f(b.U, vo4, (uint32_t)i * b.sc) : 0.f;
  }
}
__device__ inline void load_cu(const SysBuf& b, int k, uint32_t vo4, float* cr, float* ur) {
  load_cu_k<kTK, false>(b, k, vo4, cr, ur);
}

// w - C'g - sum_l h_l V_l for one voxel, from registers
template <int NV>
__device__ inline cf project_voxel(cf w, const cf* vr, const float* cr, const float* ur, const cf* g,
                                   const cf* h, int k, int nv, cd shift) {
  if (k > 0) {
    float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
    for (int i = 0; i < kTK; ++i) {
      if (i < k) {
        ar += cr[i] * g[i].re;
        ai += cr[i] * g[i].im;
        br += ur[i] * g[i].re;
        bi += ur[i] * g[i].im;
      }
    }
    const float sr = (float)shift.re, si = (float)shift.im;
    w.re -= ar + (sr * br - si * bi);
    w.im -= ai + (sr * bi + si * br);
  }
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    if (l < nv) {
      const cf v = vr[l], hl = h[l];
      w.re -= hl.re * v.re - hl.im * v.im;
      w.im -= hl.re * v.im + hl.im * v.re;
    }
  }
  return w;
}

// Stencil operands of voxel n of x, gathered into registers ahead of use: the
// centre and the six face neighbours (zero where the neighbour is outside).
struct StencilRegs {
  cf xc, m[6];
};
__device__ inline void gather_stencil(const GridP& g, Rsrc r, uint32_t so, uint32_t n, bool ok, const VoxelInfo& vi,
                                      StencilRegs& sr, bool load_centre = true) {
  // missing neighbours read past the resource (zero); the caller may supply the centre
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)g.nx * (uint32_t)g.ny;
  if (load_centre) sr.xc = ld_cf(r, ok ? n * 8u : kOutside, so);
  sr.m[0] = ld_cf(r, ok && vi.i > 0 ? (n - 1) * 8u : kOutside, so);
  sr.m[1] = ld_cf(r, ok && vi.i < g.nx - 1 ? (n + 1) * 8u : kOutside, so);
  sr.m[2] = ld_cf(r, ok && vi.j > 0 ? (n - sy) * 8u : kOutside, so);
  sr.m[3] = ld_cf(r, ok && vi.j < g.ny - 1 ? (n + sy) * 8u : kOutside, so);
  sr.m[4] = ld_cf(r, ok && vi.k > 0 ? (n - sz) * 8u : kOutside, so);
  sr.m[5] = ld_cf(r, ok && vi.k < g.nz - 1 ? (n + sz) * 8u : kOutside, so);
}
// Chunk-accumulating form: voxels are numbered consecutively across the lanes of a wave, so the
// x - 1 and x + 1 neighbours of lanes 1..63 and 0..62 are the adjacent lanes' centres and come
// by wave-wide DPP shifts once the centre is in a register (stencil_x_from_lanes).  Only lane 0
// and lane 63 load theirs, and only when the neighbour is inside the grid (never for x rows of
// 64 voxels); the y and z neighbours are loaded as in gather_stencil.
// y_lo_lds / y_hi_lds: the y - 1 / y + 1 neighbour is another thread's centre in the same
// sub-tile and comes from LDS (stencil_y_from_tile) instead.
__device__ inline void gather_stencil_yz(const GridP& g, Rsrc r, uint32_t so, uint32_t n, bool ok,
                                         const VoxelInfo& vi, StencilRegs& sr, bool load_centre,
                                         bool y_lo_lds = false, bool y_hi_lds = false) {
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)g.nx * (uint32_t)g.ny;
  const int lane = threadIdx.x & 63;
  if (load_centre) sr.xc = ld_cf(r, ok ? n * 8u : kOutside, so);
  // lanes other than 0 and 63 take these from the adjacent lanes (an offset past the resource
  // reads zero, so every lane issues the load and no branch is needed)
  sr.m[0] = ld_cf(r, lane == 0 && ok && vi.i > 0 ? (n - 1) * 8u : kOutside, so);
  sr.m[1] = ld_cf(r, lane == 63 && ok && vi.i < g.nx - 1 ? (n + 1) * 8u : kOutside, so);
  sr.m[2] = cf{0.f, 0.f};
  sr.m[3] = cf{0.f, 0.f};
  if (!y_lo_lds) sr.m[2] = ld_cf(r, ok && vi.j > 0 ? (n - sy) * 8u : kOutside, so);
  if (!y_hi_lds) sr.m[3] = ld_cf(r, ok && vi.j < g.ny - 1 ? (n + sy) * 8u : kOutside, so);
  sr.m[4] = ld_cf(r, ok && vi.k > 0 ? (n - sz) * 8u : kOutside, so);
  sr.m[5] = ld_cf(r, ok && vi.k < g.nz - 1 ? (n + sz) * 8u : kOutside, so);
}
// value of lane - 1 (0 in lane 0) and of lane + 1 (0 in lane 63): DPP wave_shr:1 / wave_shl:1
__device__ inline float lane_prev(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, true));
}
__device__ inline float lane_next(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, true));
}
// x neighbours of the inner lanes from the centres; called by every lane of the wave
__device__ inline void stencil_x_from_lanes(const GridP& g, const VoxelInfo& vi, StencilRegs& sr) {
  const int lane = threadIdx.x & 63;
  const cf prev{lane_prev(sr.xc.re), lane_prev(sr.xc.im)};
  const cf next{lane_next(sr.xc.re), lane_next(sr.xc.im)};
  // component selects (a select between two structs may be lowered through scratch memory)
  const bool kp = lane == 0, hp = vi.i > 0, kn = lane == 63, hn = vi.i < g.nx - 1;
  sr.m[0].re = kp ? sr.m[0].re : (hp ? prev.re : 0.f);
  sr.m[0].im = kp ? sr.m[0].im : (hp ? prev.im : 0.f);
  sr.m[1].re = kn ? sr.m[1].re : (hn ? next.re : 0.f);
  sr.m[1].im = kn ? sr.m[1].im : (hn ? next.im : 0.f);
}

// y neighbours from other threads' centres (x rows of at most one sub-tile): every thread
// publishes its centre in the sub-tile's LDS row; three rows rotate, so that the previous
// sub-tile's row is still intact while this one is read and one barrier per sub-tile suffices.
// y - 1 comes from this row (t >= nx) or the previous one (later sub-tiles), y + 1 from this
// row when it lies in the sub-tile; the rest was loaded (gather_stencil_yz).  Called by every
// thread of the block.
__device__ inline void stencil_y_from_tile(const GridP& g, const VoxelInfo& vi, StencilRegs& sr, cf* cur,
                                           const cf* prev, bool has_prev, int t) {
  cur[t] = sr.xc;
  __syncthreads();
  const cf z{0.f, 0.f};
  if (t >= g.nx) sr.m[2] = vi.j > 0 ? cur[t - g.nx] : z;
  else if (has_prev) sr.m[2] = vi.j > 0 ? prev[t - g.nx + kTSub] : z;
  if (t + g.nx < kTSub) sr.m[3] = vi.j < g.ny - 1 ? cur[t + g.nx] : z;
}

// (A_hat x)_n from gathered operands: the same arithmetic as apply_op.
// K's diagonal at a voxel: one per interior neighbour, two per Dirichlet face; the exterior faces
// are the Robin plus the Dirichlet ones, so nn + 2 ndir = 6 - nrobin + ndir.
__device__ inline float diag_k_of(const VoxelInfo& vi) { return (float)(6 - vi.nrobin + vi.ndir); }

__device__ inline cf stencil_apply(const GridP& g, const StencilRegs& sr, const VoxelInfo& vi, cd sig,
                                   double sigp, double extra) {
  float ar = 0.f, ai = 0.f;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    ar -= sr.m[f].re;
    ai -= sr.m[f].im;
  }
  const float diag_k = diag_k_of(vi);
  const float ih2 = (float)g.inv_h2;
  const float dr = (float)(sig.re + sigp * (double)vi.nrobin * g.inv_h + extra);
  const float di = (float)sig.im;
  const cf xc = sr.xc;
  return cf{ih2 * (diag_k * xc.re + ar) + (dr * xc.re - di * xc.im),
            ih2 * (diag_k * xc.im + ai) + (dr * xc.im + di * xc.re)};
}

// FP32 forms for the chunk-accumulating kernels: the system's shifts converted once per block,
// the per-voxel diagonal and C' shift formed in FP32 (the products are FP32 anyway).
struct SysF {
  float sig_re, sig_im, sigp_abs_h, sigp_rel_h, tau_abs, tau_rel;
};
__device__ inline SysF sys_f(const GridP& g, const SysParam& p) {
  return SysF{(float)p.sig.re, (float)p.sig.im, (float)(p.sigp_abs * g.inv_h), (float)(p.sigp_rel * g.inv_h),
              (float)p.tau_abs, (float)p.tau_rel};
}
// s (A_hat x)_n with the stencil constants pre-multiplied by the basis scale s (ScaledOp), so the
// stored basis vector V_j gives v_j = s V_j's image directly.
struct ScaledOp {
  float ih2, sig_re, sig_im, sigp_abs_h, tau_abs;
};
__device__ inline ScaledOp scaled_op(const GridP& g, const SysF& q, float s) {
  return ScaledOp{(float)g.inv_h2 * s, q.sig_re * s, q.sig_im * s, q.sigp_abs_h * s, q.tau_abs * s};
}
__device__ inline cf stencil_apply_f(const StencilRegs& sr, const VoxelInfo& vi, const ScaledOp& o, float mu) {
  float ar = 0.f, ai = 0.f;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    ar -= sr.m[f].re;
    ai -= sr.m[f].im;
  }
  const float diag_k = diag_k_of(vi);
  const float dr = o.sig_re + o.sigp_abs_h * (float)vi.nrobin + o.tau_abs * mu;
  const float di = o.sig_im;
  const cf xc = sr.xc;
  return cf{o.ih2 * (diag_k * xc.re + ar) + (dr * xc.re - di * xc.im),
            o.ih2 * (diag_k * xc.im + ai) + (dr * xc.im + di * xc.re)};
}
// w - C'g - sum_l h_l V_l with the per-voxel C' shift (sr, si) in FP32 (KM slots of C, U and g,
// the first k live; all KM when EXACT)
template <int NV, int KM = kTK, bool EXACT = false>
__device__ inline cf project_voxel_f(cf w, const cf* vr, const float* cr, const float* ur, const cf* g,
                                     const cf* h, int k, float sr, float si) {
  if (k > 0) {
    float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      if (EXACT || i < k) {
        ar += cr[i] * g[i].re;
        ai += cr[i] * g[i].im;
        br += ur[i] * g[i].re;
        bi += ur[i] * g[i].im;
      }
    }
    w.re -= ar + (sr * br - si * bi);
    w.im -= ai + (sr * bi + si * br);
  }
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    const cf v = vr[l], hl = h[l];
    w.re -= hl.re * v.re - hl.im * v.im;
    w.im -= hl.re * v.im + hl.im * v.re;
  }
  return w;
}

// Product rows of one voxel: round 0 -> conj(V_l) w for l < nv; round 1 ->
// conj(C'_i) w (row i) with C'_i = C_i + (sigma + sigma'_rel rho) U_i formed per
// voxel, so f = C'^H w arrives directly (k rows instead of C^T w, U^T w,
// (rho U)^T w), and |w|^2 (row k) if with_norm.
template <int NV, int P>
__device__ inline void write_products(ProdTile<P>& pt, int round, const cf* vr, const float* cr, const float* ur,
                                      cd shift, cf w, int k, int nv, bool with_norm, int row0 = 0) {
  if (round == 0) {
#pragma unroll
    for (int l = 0; l < NV; ++l)
      if (l < nv) {
        const cf v = vr[l];
        put_product<P>(pt, l, cf{v.re * w.re + v.im * w.im, v.re * w.im - v.im * w.re});
      }
  } else {
    const float sr = (float)shift.re, si = -(float)shift.im;   // conj(shift)
#pragma unroll
    for (int i = 0; i < kTK; ++i)
      if (i < k) {
        const float ar = cr[i] + sr * ur[i], ai = si * ur[i];
        put_product<P>(pt, row0 + i, cf{ar * w.re - ai * w.im, ar * w.im + ai * w.re});
      }
    if (with_norm) put_product<P>(pt, row0 + k, cf{w.re * w.re + w.im * w.im, 0.f});
  }
}

// Shared body of the dots (kind 0) and update (kind 1) kernels.
template <int NV, int KIND, int P>
__device__ inline void tiled_step(const Ctx<cf>& c, int j, TileIdx ti) {
  __shared__ ProdTile<P> pt;
  const int sys = ti.sys;
  const size_t N = (size_t)c.g.N;
  // NV <= 16: instance for exactly NV = j + 1 basis vectors (no per-vector guards);
  // NV = 32: any 17..32 vectors
  const int k = c.k, nv = NV <= 16 ? NV : j + 1, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  const cf* Vsys = c.V + (size_t)sys * c.vdim * N;
  cf* wv = c.W + (size_t)sys * N;
  cf g[kTK], h[NV];
  if (KIND == 1) {
    const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
#pragma unroll
    for (int i = 0; i < kTK; ++i) g[i] = i < k ? Store<cf>::from(coef[i]) : cf{0.f, 0.f};
#pragma unroll
    for (int l = 0; l < NV; ++l) h[l] = l < nv ? Store<cf>::from(coef[k + l]) : cf{0.f, 0.f};
  }
  const bool with_norm = KIND == 1;
  const int drows = k + (with_norm ? 1 : 0);
  cd accv{0.0, 0.0}, accd{0.0, 0.0};
  // Register double buffer (instances with at most 16 basis vectors): the next
  // sub-tile's loads are issued before this sub-tile's barriers and row sums,
  // which wait on LDS only, so HBM traffic overlaps the reduction.
  constexpr bool kPre = NV <= 16;
  constexpr int nsub = kChunk / kTSub;
  cf vr[NV];
  float cr[kTK], ur[kTK];
  cf wpre{0.f, 0.f};
  const SysBuf bf = sys_buf(c, sys, p.rhs);
  cf* vnext = c.V + ((size_t)sys * c.vdim + j + 1) * N;   // the update stores w' as V_{j+1}
  const float sj = KIND == 0 ? (float)c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re : 1.f;
  StencilRegs sreg;
  VoxelInfo vinf;
  {
    const uint32_t n0 = ti.chunk * kChunk + t;
    const bool ok0 = n0 < (uint32_t)c.g.N;
    load_basis<NV>(bf, ok0 ? n0 * 8u : kOutside, nv, vr);
    load_cu(bf, k, ok0 ? n0 * 4u : kOutside, cr, ur);
    vinf = voxel_info(c.g, ok0 ? n0 : 0u);
    if (KIND == 0) gather_stencil(c.g, bf.S, bf.precond ? 0u : (uint32_t)j * bf.sv, n0, ok0, vinf, sreg);
    if (KIND == 1) wpre = ld_cf(bf.W, ok0 ? n0 * 8u : kOutside, 0u);
  }
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t n = ti.chunk * kChunk + sub * kTSub + t;
    const bool ok = n < (uint32_t)c.g.N;
    if (!kPre && sub > 0) {
      load_basis<NV>(bf, ok ? n * 8u : kOutside, nv, vr);
      load_cu(bf, k, ok ? n * 4u : kOutside, cr, ur);
      vinf = voxel_info(c.g, ok ? n : 0u);
      if (KIND == 0) gather_stencil(c.g, bf.S, bf.precond ? 0u : (uint32_t)j * bf.sv, n, ok, vinf, sreg);
      if (KIND == 1) wpre = ld_cf(bf.W, ok ? n * 8u : kOutside, 0u);
    }
    double rho = 0.0;
    float muv = 0.f;
    cf w{0.f, 0.f};
    if (ok) {
      const VoxelInfo vi = vinf;
      rho = (double)vi.nrobin * c.g.inv_h;
      muv = mu_at(bf, n * 4u);
      if (KIND == 0) {
        w = stencil_apply(c.g, sreg, vi, p.sig, p.sigp_abs, p.tau_abs * (double)muv);
        w.re *= sj;   // v_j = sj * stored V_j
        w.im *= sj;
      } else {
        w = project_voxel<NV>(wpre, vr, cr, ur, g, h, k, nv, voxel_shift(p, rho, muv));
      }
      if (KIND == 0) wv[n] = w;
      else vnext[n] = w;
    }
    const cd shift = voxel_shift(p, rho, muv);
    if constexpr (NV <= 16) {
      // one round: V rows, then the deflation rows and the norm row below them
      write_products<NV, P>(pt, 0, vr, cr, ur, shift, w, k, nv, with_norm);
      if (drows > 0) write_products<NV, P>(pt, 1, vr, cr, ur, shift, w, k, nv, with_norm, nv);
      if (kPre && sub + 1 < nsub) {
        const uint32_t nn = n + kTSub;
        const bool okn = nn < (uint32_t)c.g.N;
        load_basis<NV>(bf, okn ? nn * 8u : kOutside, nv, vr);
        load_cu(bf, k, okn ? nn * 4u : kOutside, cr, ur);
        vinf = voxel_info(c.g, okn ? nn : 0u);
        if (KIND == 0) gather_stencil(c.g, bf.S, bf.precond ? 0u : (uint32_t)j * bf.sv, nn, okn, vinf, sreg);
        if (KIND == 1) wpre = ld_cf(bf.W, okn ? nn * 8u : kOutside, 0u);
      }
      __syncthreads();
      row_reduce<4, P>(pt, nv + drows, accv);
      __syncthreads();
    } else {
      write_products<NV, P>(pt, 0, vr, cr, ur, shift, w, k, nv, with_norm);
      __syncthreads();
      row_reduce<4, P>(pt, nv, accv);
      __syncthreads();
      if (drows > 0) {
        write_products<NV, P>(pt, 1, vr, cr, ur, shift, w, k, nv, with_norm);
        __syncthreads();
        row_reduce<8, P>(pt, drows, accd);
        __syncthreads();
      }
    }
  }
  if constexpr (NV <= 16) {
    row_flush_all<4>(c, sys, ti.chunk, nv, nv + drows, accv);
  } else {
    row_flush_v<4>(c, sys, ti.chunk, nv, accv);
    if (drows > 0) row_flush<8>(c, sys, ti.chunk, drows, 0, with_norm ? k : -1, accd);
  }
}

// Products of VX voxels per thread, summed in registers before the lane pre-sum:
// rows [0, nv) conj(V_l) w, rows nv + i conj(C'_i) w, row nv + k |w|^2 (with_norm).
template <int NV, int P, int VX>
__device__ inline void write_products_x(ProdTile<P>& pt, const cf (*vr)[NV], const float (*cr)[kTK],
                                        const float (*ur)[kTK], const cd* shift, const cf* w, int k, int nv,
                                        bool with_norm) {
#pragma unroll
  for (int l = 0; l < NV; ++l)
    if (l < nv) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int x = 0; x < VX; ++x) {
        const cf v = vr[x][l];
        re += v.re * w[x].re + v.im * w[x].im;
        im += v.re * w[x].im - v.im * w[x].re;
      }
      put_product<P>(pt, l, cf{re, im});
    }
#pragma unroll
  for (int i = 0; i < kTK; ++i)
    if (i < k) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int x = 0; x < VX; ++x) {
        const float ar = cr[x][i] + (float)shift[x].re * ur[x][i], ai = -(float)shift[x].im * ur[x][i];
        re += ar * w[x].re - ai * w[x].im;
        im += ar * w[x].im + ai * w[x].re;
      }
      put_product<P>(pt, nv + i, cf{re, im});
    }
  if (with_norm) {
    float a = 0.f;
#pragma unroll
    for (int x = 0; x < VX; ++x) a += w[x].re * w[x].re + w[x].im * w[x].im;
    put_product<P>(pt, nv + k, cf{a, 0.f});
  }
}

// Single-round body of the dots (kind 0) and update (kind 1) kernels for exactly NV <= 16
// basis vectors, VX voxels per thread per sub-tile (sub-tile = VX * kTSub voxels, the
// thread's voxels kTSub apart so each load stays coalesced).  The next sub-tile's
// loads are issued before this sub-tile's barriers and row sums.
template <int NV, int KIND, int P, int VX>
__device__ inline void tiled_step_x(const Ctx<cf>& c, int j, TileIdx ti) {
  static_assert(NV <= 16, "single-round instances hold at most 16 basis vectors");
  __shared__ ProdTile<P> pt;
  const int sys = ti.sys;
  const size_t N = (size_t)c.g.N;
  const int k = c.k, nv = NV, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  cf* wv = c.W + (size_t)sys * N;
  cf g[kTK], h[NV];
  if (KIND == 1) {
    const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
#pragma unroll
    for (int i = 0; i < kTK; ++i) g[i] = i < k ? Store<cf>::from(coef[i]) : cf{0.f, 0.f};
#pragma unroll
    for (int l = 0; l < NV; ++l) h[l] = Store<cf>::from(coef[k + l]);
  }
  const bool with_norm = KIND == 1;
  const int nrows = nv + k + (with_norm ? 1 : 0);
  constexpr int kSub = kTSub * VX, nsub = kChunk / kSub;
  static_assert(kChunk % kSub == 0, "chunk must hold whole sub-tiles");
  const SysBuf bf = sys_buf(c, sys, p.rhs);
  cf* vnext = c.V + ((size_t)sys * c.vdim + j + 1) * N;   // the update stores w' as V_{j+1}
  // Without a preconditioner the update recomputes w = s_j A V_j from the stencil of V_j (the
  // same arithmetic as the dots kernel, so the same value) instead of reading it back: the dots
  // kernel then writes no W, and a step moves two vectors per system less.  With one, the
  // stencil source P^{-1} V_j is not in the basis, and W is stored and read as before.
  const bool stencil = KIND == 0 || !bf.precond;
  const float sj = stencil ? (float)c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re : 1.f;
  cf vr[VX][NV];
  float cr[VX][kTK], ur[VX][kTK];
  cf wpre[VX];
  StencilRegs sreg[VX];
  VoxelInfo vinf[VX];
  float muv[VX];
  auto fetch = [&](uint32_t base) {
#pragma unroll
    for (int x = 0; x < VX; ++x) {
      const uint32_t n = base + x * kTSub + t;
      const bool ok = n < (uint32_t)c.g.N;
      load_basis<NV>(bf, ok ? n * 8u : kOutside, nv, vr[x]);
      load_cu(bf, k, ok ? n * 4u : kOutside, cr[x], ur[x]);
      vinf[x] = voxel_info(c.g, ok ? n : 0u);
      muv[x] = mu_at(bf, ok ? n * 4u : kOutside);
      if (stencil) {
        // without a preconditioner the stencil centre is V_j, already loaded as the last basis vector
        gather_stencil(c.g, bf.S, bf.precond ? 0u : (uint32_t)j * bf.sv, n, ok, vinf[x], sreg[x], bf.precond);
        if (!bf.precond) sreg[x].xc = vr[x][NV - 1];
      } else {
        wpre[x] = ld_cf(bf.W, ok ? n * 8u : kOutside, 0u);
      }
    }
  };
  cd acc{0.0, 0.0};
  fetch(ti.chunk * kChunk);
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t base = ti.chunk * kChunk + sub * kSub;
    cf w[VX];
    cd shift[VX];
#pragma unroll
    for (int x = 0; x < VX; ++x) {
      const uint32_t n = base + x * kTSub + t;
      const bool ok = n < (uint32_t)c.g.N;
      const double rho = ok ? (double)vinf[x].nrobin * c.g.inv_h : 0.0;
      shift[x] = voxel_shift(p, rho, muv[x]);
      w[x] = cf{0.f, 0.f};
      if (ok) {
        if (stencil) {
          w[x] = stencil_apply(c.g, sreg[x], vinf[x], p.sig, p.sigp_abs, p.tau_abs * (double)muv[x]);
          w[x].re *= sj;   // v_j = sj * stored V_j
          w[x].im *= sj;
        }
        if (KIND == 0) {
          if (bf.precond) wv[n] = w[x];
        } else {
          w[x] = project_voxel<NV>(stencil ? w[x] : wpre[x], vr[x], cr[x], ur[x], g, h, k, nv, shift[x]);
          vnext[n] = w[x];
        }
      }
    }
    write_products_x<NV, P, VX>(pt, vr, cr, ur, shift, w, k, nv, with_norm);
    if (sub + 1 < nsub) fetch(base + kSub);
    __syncthreads();
    row_reduce<4, P>(pt, nrows, acc);
    __syncthreads();
  }
  row_flush_all<4>(c, sys, ti.chunk, nv, nrows, acc);
}

// Chunk-accumulating form of tiled_step_x (VX = 1): each thread keeps its running FP32 sums
// of the inner-product terms of its 16 voxels in registers (4 FMA per row and voxel) and the
// block reduces them once per chunk (4-lane DPP pre-sum, LDS tile, FP64 row sums), instead of
// once per sub-tile.  The per-sub-tile reduction costs about as many VALU operations as the
// products themselves, and these kernels are bound by VALU issue, not by HBM.  Each row sums
// 64 terms in FP32 before FP64 (16 voxels times the pre-sum); the first-pass coefficients only
// set the orthogonalisation, whose loss the second-pass test measures.
// KX > 0: an instance for exactly k = KX deflation vectors (no per-slot guards or selects);
// KX = 0: any k <= kTK.
template <int NV, int KIND, int KX, bool PL = false>
__device__ inline void tiled_step_acc(const Ctx<cf>& c, int j, TileIdx ti) {
  static_assert(NV <= 16, "chunk-accumulating instances hold at most 16 basis vectors");
  static_assert(KX >= 0 && KX <= kTK, "exact deflation dimension out of range");
  constexpr bool EX = KX > 0;
  constexpr int KM = EX ? KX : kTK;
  __shared__ ProdTile<4> pt;
  // Stencil centres of four consecutive sub-tiles (rotating): the previous, the current and the
  // next one are read, the fourth is being overwritten, so one barrier per sub-tile suffices.
  __shared__ cf xs[4][kTSub];
  const int sys = ti.sys;
  const size_t N = (size_t)c.g.N;
  const int k = EX ? KX : c.k, nv = NV, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  cf* wv = c.W + (size_t)sys * N;
  cf g[KM], h[NV];
  if (KIND == 1) {
    // the FP32 copy of this step's coefficients: block-uniform loads kept in scalar registers
    const cf* coef = reinterpret_cast<const cf*>(c.small + (size_t)sys * c.sl.total + c.sl.cA32);
#pragma unroll
    for (int i = 0; i < KM; ++i) g[i] = EX || i < k ? coef[i] : cf{0.f, 0.f};
#pragma unroll
    for (int l = 0; l < NV; ++l) h[l] = coef[k + l];
  }
  const bool with_norm = KIND == 1;
  const int nrows = nv + k + (with_norm ? 1 : 0);
  constexpr int nsub = kChunk / kTSub;
  // PL: no absorption perturbation and no preconditioner (known at compile time)
  const SysBuf bf = PL ? sys_buf_plain(c, sys, p.rhs) : sys_buf(c, sys, p.rhs);
  cf* vnext = c.V + ((size_t)sys * c.vdim + j + 1) * N;
  const bool stencil = KIND == 0 || !bf.precond;
  // x rows of at most one sub-tile (the host routes longer rows to the other instances): every
  // face neighbour but the z ones is the centre of a voxel in this, the previous or the next
  // sub-tile, so the centres go through LDS (each loaded once, one sub-tile ahead) and only the z
  // neighbours are loaded
  const bool ytile = stencil;
  const bool vj_centre = ytile && !bf.precond;   // V_j's register value is the stencil centre
  const uint32_t so = bf.precond ? 0u : (uint32_t)j * bf.sv;   // stencil source: V_j or P^{-1} V_j
  const uint32_t Nu = (uint32_t)c.g.N, sz = (uint32_t)c.g.nx * (uint32_t)c.g.ny;
  const float sj = stencil ? (float)c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re : 1.f;
  const SysF q = sys_f(c.g, p);
  const ScaledOp qs = scaled_op(c.g, q, sj);   // v_j = sj * stored V_j
  cf vr[NV];
  float cr[KM], ur[KM];
  cf wpre{0.f, 0.f};
  cf c_ahead{0.f, 0.f};   // centre of the sub-tile after the one last fetched (published next)
  StencilRegs sreg;
  VoxelInfo vinf;
  float muv;
  auto fetch = [&](uint32_t n, bool first) {   // first: the chunk's first sub-tile
    const bool ok = n < Nu;
    if (vj_centre) {
      // V_0..V_{NV-2} streamed; V_j comes with the centres
#pragma unroll
      for (int l = 0; l + 1 < NV; ++l) vr[l] = ld_cf_nt(bf.V, ok ? n * 8u : kOutside, (uint32_t)l * bf.sv);
    } else {
      load_basis_stream<NV>(bf, ok ? n * 8u : kOutside, vr);
    }
    load_cu_k<KM, EX>(bf, k, ok ? n * 4u : kOutside, cr, ur);
    vinf = voxel_info(c.g, ok ? n : 0u);
    muv = mu_at(bf, ok ? n * 4u : kOutside);
    if (ytile) {
      sreg.m[4] = ld_cf(bf.S, ok && vinf.k > 0 ? (n - sz) * 8u : kOutside, so);
      sreg.m[5] = ld_cf(bf.S, ok && vinf.k < c.g.nz - 1 ? (n + sz) * 8u : kOutside, so);
      const uint32_t na = n + kTSub;   // centre of the sub-tile after the one being fetched
      c_ahead = ld_cf(bf.S, na < Nu ? na * 8u : kOutside, so);
    } else {
      wpre = ld_cf(bf.W, ok ? n * 8u : kOutside, 0u);
    }
    (void)first;
  };
  cf av[NV], ac[KM], au[KM], an{0.f, 0.f};
#pragma unroll
  for (int l = 0; l < NV; ++l) av[l] = cf{0.f, 0.f};
#pragma unroll
  for (int i = 0; i < KM; ++i) ac[i] = au[i] = cf{0.f, 0.f};
  const uint32_t n0 = (uint32_t)ti.chunk * kChunk;
  if (ytile) {
    // the centres of the sub-tile before the chunk and of its first sub-tile
    const uint32_t nm = n0 + (uint32_t)t - kTSub, nc = n0 + (uint32_t)t;
    xs[3][t] = ld_cf(bf.S, n0 >= (uint32_t)kTSub && nm < Nu ? nm * 8u : kOutside, so);
    xs[0][t] = ld_cf(bf.S, nc < Nu ? nc * 8u : kOutside, so);
  }
  fetch(n0 + t, true);
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t n = n0 + sub * kTSub + t;
    const bool ok = n < Nu;
    if (ytile) {
      xs[(sub + 1) & 3][t] = c_ahead;   // the next sub-tile's centres
      __syncthreads();
      // rows of the previous, current and next sub-tile (indices into xs, no LDS pointers)
      const int bp = (sub + 3) & 3, bc = sub & 3, bn = (sub + 1) & 3;
      const int nxg = c.g.nx, lane = t & 63;
      sreg.xc = xs[bc][t];
      if (vj_centre) vr[NV - 1] = sreg.xc;
      // neighbour positions in the ring (row, index), then value selects (selects between LDS
      // and register objects would go through generic pointers)
      const int ym = t - nxg, yp = t + nxg;
      const cf vym = xs[ym >= 0 ? bc : bp][ym >= 0 ? ym : ym + kTSub];
      const cf vyp = xs[yp < kTSub ? bc : bn][yp < kTSub ? yp : yp - kTSub];
      const bool hy0 = vinf.j > 0, hy1 = vinf.j < c.g.ny - 1;
      sreg.m[2] = cf{hy0 ? vym.re : 0.f, hy0 ? vym.im : 0.f};
      sreg.m[3] = cf{hy1 ? vyp.re : 0.f, hy1 ? vyp.im : 0.f};
      // x neighbours of the wave's edge lanes (the inner lanes take theirs by DPP below)
      if (lane == 0) {
        const cf v = xs[t > 0 ? bc : bp][t > 0 ? t - 1 : kTSub - 1];
        const bool hx = vinf.i > 0;
        sreg.m[0] = cf{hx ? v.re : 0.f, hx ? v.im : 0.f};
      }
      if (lane == 63) {
        const cf v = xs[t + 1 < kTSub ? bc : bn][t + 1 < kTSub ? t + 1 : 0];
        const bool hx = vinf.i < nxg - 1;
        sreg.m[1] = cf{hx ? v.re : 0.f, hx ? v.im : 0.f};
      }
    }
    if (stencil) stencil_x_from_lanes(c.g, vinf, sreg);   // every lane (no divergence yet)
    if (ok) {
      // C' shift of this voxel: sigma + sigma'_rel rho + tau_rel mu
      const float shr = q.sig_re + q.sigp_rel_h * (float)vinf.nrobin + q.tau_rel * muv, shi = q.sig_im;
      cf w{0.f, 0.f};
      if (stencil) w = stencil_apply_f(sreg, vinf, qs, muv);
      if (KIND == 0) {
        if (bf.precond) wv[n] = w;
      } else {
        w = project_voxel_f<NV, KM, EX>(stencil ? w : wpre, vr, cr, ur, g, h, k, shr, shi);
        st_cf_nt(vnext + n, w);
      }
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        const cf v = vr[l];
        av[l].re += v.re * w.re + v.im * w.im;
        av[l].im += v.re * w.im - v.im * w.re;
      }
      // conj(C'_i) w = (C_i + Re(shift) U_i) w - i Im(shift) U_i w with C, U real and Im(shift)
      // uniform: two real-times-complex sums per row here, the imaginary shift applied once per
      // chunk below
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (EX || i < k) {
          const float a = __builtin_fmaf(shr, ur[i], cr[i]);
          ac[i].re = __builtin_fmaf(a, w.re, ac[i].re);
          ac[i].im = __builtin_fmaf(a, w.im, ac[i].im);
          au[i].re = __builtin_fmaf(ur[i], w.re, au[i].re);
          au[i].im = __builtin_fmaf(ur[i], w.im, au[i].im);
        }
      if (with_norm) an.re += w.re * w.re + w.im * w.im;
    }
    if (sub + 1 < nsub) fetch(n + kTSub, false);
  }
  // one block reduction per chunk: rows [0, nv) V, [nv, nv + k) C', nv + k the norm
#pragma unroll
  for (int l = 0; l < NV; ++l) put_product<4>(pt, l, av[l]);
  const float shi = q.sig_im;
#pragma unroll
  for (int i = 0; i < KM; ++i)
    if (EX || i < k) put_product<4>(pt, nv + i, cf{ac[i].re + shi * au[i].im, ac[i].im - shi * au[i].re});
  if (with_norm) put_product<4>(pt, nv + k, an);
  __syncthreads();
  cd acc{0.0, 0.0};
  row_reduce<4, 4>(pt, nrows, acc);
  row_flush_all<4>(c, sys, ti.chunk, nv, nrows, acc);
}

// Two systems per block (pairs of wavelengths of one right-hand side at one chunk): the form of
// tiled_step_acc for plain systems (no absorption perturbation, no preconditioner) in which each
// thread handles its voxel for both systems, so C and U, which the wavelengths of a right-hand
// side share, are loaded once for the two.  The arithmetic of each system is that of
// tiled_step_acc's plain instances (same operations in the same order, same block reduction), so
// the results are identical to theirs.  A system that is not stepping is skipped (block-uniform
// branches).
template <int NV, int KIND, int KX>
__device__ inline void tiled_step_acc2(const Ctx<cf>& c, int j, int sys0, int chunk) {
  static_assert(NV >= 1 && NV <= 16, "chunk-accumulating instances hold 1 to 16 basis vectors");
  static_assert(KX >= 0 && KX <= kTK, "exact deflation dimension out of range");
  constexpr bool EX = KX > 0;
  constexpr int KM = EX ? KX : kTK;
  __shared__ ProdTile<4> pt;
  __shared__ cf xs[2][4][kTSub];
  const size_t N = (size_t)c.g.N;
  const int k = EX ? KX : c.k, nv = NV, t = threadIdx.x;
  const bool act[2] = {c.st[sys0].in_cycle != 0, c.st[sys0 + 1].in_cycle != 0};
  const int rhs = c.prm[sys0].rhs;   // shared by the pair
  const SysBuf bf = sys_buf_plain(c, sys0, rhs);   // C and U; the basis resources per system below
  Rsrc rv[2];
  cf* vnext[2];
  float sjs[2];
  SysF q[2];
  ScaledOp qs[2];
  cf g[2][KM], h[2][NV];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int sys = sys0 + s;
    const SysParam p = c.prm[sys];
    rv[s] = make_rsrc(c.V + (size_t)sys * c.vdim * N, (uint32_t)c.vdim * bf.sv);
    vnext[s] = c.V + ((size_t)sys * c.vdim + j + 1) * N;
    sjs[s] = (float)c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re;
    q[s] = sys_f(c.g, p);
    qs[s] = scaled_op(c.g, q[s], sjs[s]);
    if (KIND == 1) {
      const cf* coef = reinterpret_cast<const cf*>(c.small + (size_t)sys * c.sl.total + c.sl.cA32);
#pragma unroll
      for (int i = 0; i < KM; ++i) g[s][i] = EX || i < k ? coef[i] : cf{0.f, 0.f};
#pragma unroll
      for (int l = 0; l < NV; ++l) h[s][l] = coef[k + l];
    }
  }
  const bool with_norm = KIND == 1;
  const int nrows = nv + k + (with_norm ? 1 : 0);
  constexpr int nsub = kChunk / kTSub;
  const uint32_t so = (uint32_t)j * bf.sv;   // V_j within a system's basis
  const uint32_t Nu = (uint32_t)c.g.N, sz = (uint32_t)c.g.nx * (uint32_t)c.g.ny;
  cf vr[2][NV];
  float cr[KM], ur[KM];
  cf c_ahead[2];
  StencilRegs sreg[2];
  VoxelInfo vinf;
  auto fetch = [&](uint32_t n) {
    const bool ok = n < Nu;
    load_cu_k<KM, EX>(bf, k, ok ? n * 4u : kOutside, cr, ur);
    vinf = voxel_info(c.g, ok ? n : 0u);
    const uint32_t na = n + kTSub;   // centre of the sub-tile after the one being fetched
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (act[s]) {
#pragma unroll
        for (int l = 0; l + 1 < NV; ++l) vr[s][l] = ld_cf_nt(rv[s], ok ? n * 8u : kOutside, (uint32_t)l * bf.sv);
        sreg[s].m[4] = ld_cf(rv[s], ok && vinf.k > 0 ? (n - sz) * 8u : kOutside, so);
        sreg[s].m[5] = ld_cf(rv[s], ok && vinf.k < c.g.nz - 1 ? (n + sz) * 8u : kOutside, so);
        c_ahead[s] = ld_cf(rv[s], na < Nu ? na * 8u : kOutside, so);
      }
    }
  };
  cf av[2][NV], ac[2][KM], au[2][KM], an[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    an[s] = cf{0.f, 0.f};
#pragma unroll
    for (int l = 0; l < NV; ++l) av[s][l] = cf{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < KM; ++i) ac[s][i] = au[s][i] = cf{0.f, 0.f};
  }
  const uint32_t n0 = (uint32_t)chunk * kChunk;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const uint32_t nm = n0 + (uint32_t)t - kTSub, nc = n0 + (uint32_t)t;
    xs[s][3][t] = act[s] ? ld_cf(rv[s], n0 >= (uint32_t)kTSub && nm < Nu ? nm * 8u : kOutside, so) : cf{0.f, 0.f};
    xs[s][0][t] = act[s] ? ld_cf(rv[s], nc < Nu ? nc * 8u : kOutside, so) : cf{0.f, 0.f};
    c_ahead[s] = cf{0.f, 0.f};
  }
  fetch(n0 + t);
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t n = n0 + sub * kTSub + t;
    const bool ok = n < Nu;
#pragma unroll
    for (int s = 0; s < 2; ++s) xs[s][(sub + 1) & 3][t] = c_ahead[s];
    __syncthreads();
    const int bp = (sub + 3) & 3, bc = sub & 3, bn = (sub + 1) & 3;
    const int nxg = c.g.nx, lane = t & 63;
    const int ym = t - nxg, yp = t + nxg;
    const bool hy0 = vinf.j > 0, hy1 = vinf.j < c.g.ny - 1;
    const bool hx0 = vinf.i > 0, hx1 = vinf.i < nxg - 1;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      sreg[s].xc = xs[s][bc][t];
      vr[s][NV - 1] = sreg[s].xc;
      const cf vym = xs[s][ym >= 0 ? bc : bp][ym >= 0 ? ym : ym + kTSub];
      const cf vyp = xs[s][yp < kTSub ? bc : bn][yp < kTSub ? yp : yp - kTSub];
      sreg[s].m[2] = cf{hy0 ? vym.re : 0.f, hy0 ? vym.im : 0.f};
      sreg[s].m[3] = cf{hy1 ? vyp.re : 0.f, hy1 ? vyp.im : 0.f};
      if (lane == 0) {
        const cf v = xs[s][t > 0 ? bc : bp][t > 0 ? t - 1 : kTSub - 1];
        sreg[s].m[0] = cf{hx0 ? v.re : 0.f, hx0 ? v.im : 0.f};
      }
      if (lane == 63) {
        const cf v = xs[s][t + 1 < kTSub ? bc : bn][t + 1 < kTSub ? t + 1 : 0];
        sreg[s].m[1] = cf{hx1 ? v.re : 0.f, hx1 ? v.im : 0.f};
      }
      stencil_x_from_lanes(c.g, vinf, sreg[s]);   // every lane (no divergence yet)
    }
    if (ok) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (!act[s]) continue;
        const float shr = q[s].sig_re + q[s].sigp_rel_h * (float)vinf.nrobin, shi = q[s].sig_im;
        cf w = stencil_apply_f(sreg[s], vinf, qs[s], 0.f);
        if (KIND == 1) {
          w = project_voxel_f<NV, KM, EX>(w, vr[s], cr, ur, g[s], h[s], k, shr, shi);
          st_cf_nt(vnext[s] + n, w);
        }
#pragma unroll
        for (int l = 0; l < NV; ++l) {
          const cf v = vr[s][l];
          av[s][l].re += v.re * w.re + v.im * w.im;
          av[s][l].im += v.re * w.im - v.im * w.re;
        }
#pragma unroll
        for (int i = 0; i < KM; ++i)
          if (EX || i < k) {
            const float a = __builtin_fmaf(shr, ur[i], cr[i]);
            ac[s][i].re = __builtin_fmaf(a, w.re, ac[s][i].re);
            ac[s][i].im = __builtin_fmaf(a, w.im, ac[s][i].im);
            au[s][i].re = __builtin_fmaf(ur[i], w.re, au[s][i].re);
            au[s][i].im = __builtin_fmaf(ur[i], w.im, au[s][i].im);
          }
        if (with_norm) an[s].re += w.re * w.re + w.im * w.im;
      }
    }
    if (sub + 1 < nsub) fetch(n + kTSub);
  }
  // one block reduction per chunk and system, the product tile reused
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!act[s]) continue;
    if (s == 1) __syncthreads();   // the first system's rows have been read
#pragma unroll
    for (int l = 0; l < NV; ++l) put_product<4>(pt, l, av[s][l]);
    const float shi = q[s].sig_im;
#pragma unroll
    for (int i = 0; i < KM; ++i)
      if (EX || i < k) put_product<4>(pt, nv + i, cf{ac[s][i].re + shi * au[s][i].im, ac[s][i].im - shi * au[s][i].re});
    if (with_norm) put_product<4>(pt, nv + k, an[s]);
    __syncthreads();
    cd acc{0.0, 0.0};
    row_reduce<4, 4>(pt, nrows, acc);
    row_flush_all<4>(c, sys0 + s, chunk, nv, nrows, acc);
  }
}

// The two-system step kernels: block b takes the pair (2i, 2i + 1) of tile_map's index i over
// nb / 2 pairs in groups of grp pairs (half the wavelengths of one right-hand side, or 1).
template <int NV, int KIND, int KX>
__global__ __launch_bounds__(kTSub) void k_step_pair_t(Ctx<cf> c, int j, int grp, int flags) {
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  const int sys0 = 2 * ti.sys;
  if (!c.st[sys0].in_cycle && !c.st[sys0 + 1].in_cycle) return;
  tiled_step_acc2<NV, KIND, KX>(c, j, sys0, ti.chunk);
}

// w = A_hat V_j and first-pass inner products (tiled form of k_step_dots); w is stored as W
// only where the update cannot recompute it (preconditioner, more than 16 basis vectors).
// flags: block order (tile_idx).  VX voxels per thread per sub-tile (NV <= 16).
// PL: the system has no absorption perturbation and no preconditioner (chunk-accumulating form).
template <int NV, int P, int VX, int KX = 0, bool PL = false>
__global__ __launch_bounds__(kTSub) void k_step_dots_t(Ctx<cf> c, int j, int grp, int flags) {
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  if (!c.st[ti.sys].in_cycle) return;
  if constexpr (P == 16) {
    if constexpr (NV <= 16) tiled_step_acc<NV, 0, KX, PL>(c, j, ti);
  } else if constexpr (NV <= 16) {
    tiled_step_x<NV, 0, P, VX>(c, j, ti);
  } else {
    tiled_step<NV, 0, P>(c, j, ti);
  }
}

// First projection (w' stored as V_{j+1}) + second-pass inner products (tiled form of k_step_update).
template <int NV, int P, int VX, int KX = 0, bool PL = false>
__global__ __launch_bounds__(kTSub) void k_step_update_t(Ctx<cf> c, int j, int grp, int flags) {
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  if (!c.st[ti.sys].in_cycle) return;
  if constexpr (P == 16) {
    if constexpr (NV <= 16) tiled_step_acc<NV, 1, KX, PL>(c, j, ti);
  } else if constexpr (NV <= 16) {
    tiled_step_x<NV, 1, P, VX>(c, j, ti);
  } else {
    tiled_step<NV, 1, P>(c, j, ti);
  }
}

// Second projection and normalisation in place of V_{j+1}, for the systems whose
// second Gram-Schmidt pass is applied (tiled form of k_step_finish).
template <int NV>
__global__ __launch_bounds__(kTSub) void k_step_finish_t(Ctx<cf> c, int j, int grp, int flags) {
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  const int sys = ti.sys;
  if (!c.st[sys].in_cycle || !c.st[sys].reorth) return;
  const size_t N = (size_t)c.g.N;
  const int k = c.k, nv = j + 1, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  cf* Vsys = c.V + (size_t)sys * c.vdim * N;
  cf* vn = Vsys + (size_t)(j + 1) * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefB;
  const float inv_eta = (float)coef[k + c.mkmax + 1].re;
  const SysBuf bf = sys_buf(c, sys, p.rhs);
  cf g[kTK], h[NV];
#pragma unroll
  for (int i = 0; i < kTK; ++i) g[i] = i < k ? Store<cf>::from(coef[i]) : cf{0.f, 0.f};
#pragma unroll
  for (int l = 0; l < NV; ++l) h[l] = l < nv ? Store<cf>::from(coef[k + l]) : cf{0.f, 0.f};
  for (int sub = 0; sub < kChunk / kTSub; ++sub) {
    const uint32_t n = ti.chunk * kChunk + sub * kTSub + t;
    if (n >= (uint32_t)c.g.N) break;
    cf vr[NV];
    float cr[kTK], ur[kTK];
    load_basis<NV>(bf, n * 8u, nv, vr);
    load_cu(bf, k, n * 4u, cr, ur);
    const double rho = (double)voxel_info(c.g, n).nrobin * c.g.inv_h;
    cf w = project_voxel<NV>(vn[n], vr, cr, ur, g, h, k, nv, voxel_shift(p, rho, mu_at(bf, n * 4u)));
    vn[n] = cf{w.re * inv_eta, w.im * inv_eta};
  }
}

// Cycle start, first half (tiled form of k_inner_resid): W = Rin - A_hat Din, then
// f = C'^H W (k rows, C' formed per voxel) and |W|^2 as chunk partials.
template <int P>
__global__ __launch_bounds__(kTSub) void k_inner_resid_t(Ctx<cf> c, int grp, int flags) {
  __shared__ ProdTile<P> pt;
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  const int sys = ti.sys;
  if (!c.st[sys].in_inner) return;
  const size_t N = (size_t)c.g.N;
  const int k = c.k, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  const SysBuf bf = sys_buf(c, sys, p.rhs);
  const Rsrc rD = make_rsrc(c.Din + (size_t)sys * N, bf.sv), rR = make_rsrc(c.Rin + (size_t)sys * N, bf.sv);
  cf* wv = c.W + (size_t)sys * N;
  constexpr int nsub = kChunk / kTSub;
  float cr[kTK], ur[kTK];
  StencilRegs sreg;
  VoxelInfo vinf;
  cf rin;
  float muv = 0.f;
  auto fetch = [&](uint32_t n, bool ok) {
    load_cu(bf, k, ok ? n * 4u : kOutside, cr, ur);
    vinf = voxel_info(c.g, ok ? n : 0u);
    muv = mu_at(bf, ok ? n * 4u : kOutside);
    gather_stencil_yz(c.g, rD, 0u, n, ok, vinf, sreg, true);
    rin = ld_cf(rR, ok ? n * 8u : kOutside, 0u);
  };
  cd acc{0.0, 0.0};
  {
    const uint32_t n0 = ti.chunk * kChunk + t;
    fetch(n0, n0 < (uint32_t)c.g.N);
  }
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t n = ti.chunk * kChunk + sub * kTSub + t;
    const bool ok = n < (uint32_t)c.g.N;
    const double rho = ok ? (double)vinf.nrobin * c.g.inv_h : 0.0;
    stencil_x_from_lanes(c.g, vinf, sreg);   // every lane (no divergence yet)
    cf w{0.f, 0.f};
    if (ok) {
      const cf ad = stencil_apply(c.g, sreg, vinf, p.sig, p.sigp_abs, p.tau_abs * (double)muv);
      w = cf{rin.re - ad.re, rin.im - ad.im};
      wv[n] = w;
    }
    const cd shift = voxel_shift(p, rho, muv);
    write_products<1, P>(pt, 1, nullptr, cr, ur, shift, w, k, 0, true, 0);
    if (sub + 1 < nsub) {
      const uint32_t nn = n + kTSub;
      fetch(nn, nn < (uint32_t)c.g.N);
    }
    __syncthreads();
    row_reduce<4, P>(pt, k + 1, acc);
    __syncthreads();
  }
  row_flush_all<4>(c, sys, ti.chunk, 0, k + 1, acc);
}

// Cycle start, first half in the chunk-accumulating form of the step kernels (x rows of at most
// one sub-tile): W = Rin - A_hat Din with the stencil centres of Din through the four-sub-tile LDS
// ring (each loaded once, one sub-tile ahead; only the z neighbours are loaded besides), FP32
// running sums of conj(C'_i) W and |W|^2 per thread over its 16 voxels and one block reduction
// per chunk into the rows of k_inner_resid_t (rows [0, k) C', row k the norm).  KX, PL as the
// step kernels.
template <int KX, bool PL>
__global__ __launch_bounds__(kTSub) void k_inner_resid_acc(Ctx<cf> c, int grp, int flags) {
  static_assert(KX >= 0 && KX <= kTK, "exact deflation dimension out of range");
  constexpr bool EX = KX > 0;
  constexpr int KM = EX ? KX : kTK;
  __shared__ ProdTile<4> pt;
  __shared__ cf xs[4][kTSub];
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  const int sys = ti.sys;
  if (!c.st[sys].in_inner) return;
  const size_t N = (size_t)c.g.N;
  const int k = EX ? KX : c.k, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  const SysBuf bf = PL ? sys_buf_plain(c, sys, p.rhs) : sys_buf(c, sys, p.rhs);
  const Rsrc rD = make_rsrc(c.Din + (size_t)sys * N, bf.sv), rR = make_rsrc(c.Rin + (size_t)sys * N, bf.sv);
  cf* wv = c.W + (size_t)sys * N;
  const uint32_t Nu = (uint32_t)c.g.N, sz = (uint32_t)c.g.nx * (uint32_t)c.g.ny;
  const SysF q = sys_f(c.g, p);
  const ScaledOp qs = scaled_op(c.g, q, 1.f);
  float cr[KM], ur[KM];
  cf rin{0.f, 0.f}, c_ahead{0.f, 0.f};
  StencilRegs sreg;
  VoxelInfo vinf;
  float muv;
  auto fetch = [&](uint32_t n) {
    const bool ok = n < Nu;
    load_cu_k<KM, EX>(bf, k, ok ? n * 4u : kOutside, cr, ur);
    vinf = voxel_info(c.g, ok ? n : 0u);
    muv = mu_at(bf, ok ? n * 4u : kOutside);
    sreg.m[4] = ld_cf(rD, ok && vinf.k > 0 ? (n - sz) * 8u : kOutside, 0u);
    sreg.m[5] = ld_cf(rD, ok && vinf.k < c.g.nz - 1 ? (n + sz) * 8u : kOutside, 0u);
    const uint32_t na = n + kTSub;   // centre of the sub-tile after the one being fetched
    c_ahead = ld_cf(rD, na < Nu ? na * 8u : kOutside, 0u);
    rin = ld_cf(rR, ok ? n * 8u : kOutside, 0u);
  };
  cf ac[KM], au[KM], an{0.f, 0.f};
#pragma unroll
  for (int i = 0; i < KM; ++i) ac[i] = au[i] = cf{0.f, 0.f};
  const uint32_t n0 = (uint32_t)ti.chunk * kChunk;
  {
    const uint32_t nm = n0 + (uint32_t)t - kTSub, nc = n0 + (uint32_t)t;
    xs[3][t] = ld_cf(rD, n0 >= (uint32_t)kTSub && nm < Nu ? nm * 8u : kOutside, 0u);
    xs[0][t] = ld_cf(rD, nc < Nu ? nc * 8u : kOutside, 0u);
  }
  fetch(n0 + t);
  constexpr int nsub = kChunk / kTSub;
  for (int sub = 0; sub < nsub; ++sub) {
    const uint32_t n = n0 + sub * kTSub + t;
    const bool ok = n < Nu;
    xs[(sub + 1) & 3][t] = c_ahead;
    __syncthreads();
    const int bp = (sub + 3) & 3, bc = sub & 3, bn = (sub + 1) & 3;
    const int nxg = c.g.nx, lane = t & 63;
    sreg.xc = xs[bc][t];
    const int ym = t - nxg, yp = t + nxg;
    const cf vym = xs[ym >= 0 ? bc : bp][ym >= 0 ? ym : ym + kTSub];
    const cf vyp = xs[yp < kTSub ? bc : bn][yp < kTSub ? yp : yp - kTSub];
    const bool hy0 = vinf.j > 0, hy1 = vinf.j < c.g.ny - 1;
    sreg.m[2] = cf{hy0 ? vym.re : 0.f, hy0 ? vym.im : 0.f};
    sreg.m[3] = cf{hy1 ? vyp.re : 0.f, hy1 ? vyp.im : 0.f};
    if (lane == 0) {
      const cf v = xs[t > 0 ? bc : bp][t > 0 ? t - 1 : kTSub - 1];
      const bool hx = vinf.i > 0;
      sreg.m[0] = cf{hx ? v.re : 0.f, hx ? v.im : 0.f};
    }
    if (lane == 63) {
      const cf v = xs[t + 1 < kTSub ? bc : bn][t + 1 < kTSub ? t + 1 : 0];
      const bool hx = vinf.i < nxg - 1;
      sreg.m[1] = cf{hx ? v.re : 0.f, hx ? v.im : 0.f};
    }
    stencil_x_from_lanes(c.g, vinf, sreg);   // every lane (no divergence yet)
    if (ok) {
      const float shr = q.sig_re + q.sigp_rel_h * (float)vinf.nrobin + q.tau_rel * muv;
      const cf ad = stencil_apply_f(sreg, vinf, qs, muv);
      const cf w{rin.re - ad.re, rin.im - ad.im};
      wv[n] = w;
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (EX || i < k) {
          const float a = __builtin_fmaf(shr, ur[i], cr[i]);
          ac[i].re = __builtin_fmaf(a, w.re, ac[i].re);
          ac[i].im = __builtin_fmaf(a, w.im, ac[i].im);
          au[i].re = __builtin_fmaf(ur[i], w.re, au[i].re);
          au[i].im = __builtin_fmaf(ur[i], w.im, au[i].im);
        }
      an.re += w.re * w.re + w.im * w.im;
    }
    if (sub + 1 < nsub) fetch(n + kTSub);
  }
  const float shi = q.sig_im;
#pragma unroll
  for (int i = 0; i < KM; ++i)
    if (EX || i < k) put_product<4>(pt, i, cf{ac[i].re + shi * au[i].im, ac[i].im - shi * au[i].re});
  put_product<4>(pt, k, an);
  __syncthreads();
  cd acc{0.0, 0.0};
  row_reduce<4, 4>(pt, k + 1, acc);
  row_flush_all<4>(c, sys, ti.chunk, 0, k + 1, acc);
}

// Cycle start, second half (tiled form of k_defl_start): with g = G^-1 f,
// W <- W - C'g, Din += U g, V_0 = W (stored unnormalised), |V_0|^2 as chunk partials.
__global__ __launch_bounds__(kTSub) void k_defl_start_t(Ctx<cf> c, int grp, int flags) {
  __shared__ double wsum[kTSub / 64];
  const TileIdx ti = tile_idx(c.nchunks, grp, flags);
  const int sys = ti.sys;
  if (!c.st[sys].cyc_ran) return;
  const size_t N = (size_t)c.g.N;
  const int k = c.k, t = threadIdx.x;
  const SysParam p = c.prm[sys];
  const SysBuf bf = sys_buf(c, sys, p.rhs);
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  cf g[kTK];
#pragma unroll
  for (int i = 0; i < kTK; ++i) g[i] = i < k ? Store<cf>::from(coef[i]) : cf{0.f, 0.f};
  cf* wv = c.W + (size_t)sys * N;
  cf* din = c.Din + (size_t)sys * N;
  cf* v0 = c.V + (size_t)sys * c.vdim * N;
  double nrm = 0.0;
  for (int sub = 0; sub < kChunk / kTSub; ++sub) {
    const uint32_t n = ti.chunk * kChunk + sub * kTSub + t;
    if (n >= (uint32_t)c.g.N) break;
    float cr[kTK], ur[kTK];
    load_cu(bf, k, n * 4u, cr, ur);
    const cf w0 = ld_cf(bf.W, n * 8u, 0u);
    const double rho = (double)voxel_info(c.g, n).nrobin * c.g.inv_h;
    float br = 0.f, bi = 0.f;   // (U g)_n
#pragma unroll
    for (int i = 0; i < kTK; ++i)
      if (i < k) {
        br += ur[i] * g[i].re;
        bi += ur[i] * g[i].im;
      }
    const cf w = project_voxel<1>(w0, nullptr, cr, ur, g, nullptr, k, 0, voxel_shift(p, rho, mu_at(bf, n * 4u)));
    v0[n] = w;
    if (k > 0) {
      const cf d = din[n];
      din[n] = cf{d.re + br, d.im + bi};
    }
    nrm += (double)w.re * (double)w.re + (double)w.im * (double)w.im;
  }
  nrm = wave_sum(nrm);
  if ((t & 63) == 0) wsum[t >> 6] = nrm;
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < kTSub / 64; ++w) a += wsum[w];
    c.part[part_base(sys, c.nchunks, ti.chunk, c.ndots) + slot_norm(c.k, c.mkmax)] = cd{a, 0.0};
  }
}

}  // namespace hydot
