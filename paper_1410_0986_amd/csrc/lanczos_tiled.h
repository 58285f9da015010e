// Chunk-accumulating forms of the real FP32 Lanczos kernels (Alg. 1 step 1 on the mixed path).
// One block of 128 threads per (right-hand side, 2048-voxel chunk) walks the chunk's 16 sub-tiles
// of 128 voxels (voxel = chunk * 2048 + sub * 128 + thread), keeps FP32 running sums of its
// voxels' inner-product terms in registers and reduces them once per chunk, in FP64 across the
// block, into the partial-sum layout of the generic kernels (slot l: basis vector l; the norm in
// slot_norm(0, mkmax)), so k_reduce in its Lanczos mode is unchanged.  The basis of a right-hand
// side is read through one buffer resource (an offset past its end reads zero) and the x
// neighbours of the stencil come from the adjacent lanes by DPP.  An instance holds NV basis
// vectors in registers with no per-vector branch: the host takes the exact count up to 16 and the
// next multiple of 4 beyond, and vectors past the step's count read zero (an offset past the
// resource), so their rows are never used.
#pragma once

#include "krylov_tiled.h"
#include "lanczos.h"

namespace hydot {

constexpr int kLzTiledMax = 60;   // basis vectors of the largest chunk-accumulating instance

// non-temporal (streaming) FP32 load, for basis vectors read once per launch
__device__ inline float ld_f_nt(Rsrc r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 2));
}

// Block sums of rows [0, nrows) of the per-thread FP32 values (row NV: nrm, when with_norm):
// the rows go through LDS transposed (row r, thread t at tile[r][t]; the pitch of 129 words keeps
// both the writes and the row reads free of bank conflicts), then two threads sum each row in
// FP64 over 64 threads apiece.  Row r goes to out[r], the norm to out[norm_slot].
template <int NV>
struct LzTile {
  float v[NV + 1][kTSub + 1];
};
template <int NV>
__device__ inline void lz_flush_t(const float* acc, int nrows, bool with_norm, float nrm, LzTile<NV>& tile, cd* out,
                                  int norm_slot) {
  const int t = threadIdx.x;
#pragma unroll
  for (int l = 0; l < NV; ++l) tile.v[l][t] = acc[l];
  tile.v[NV][t] = nrm;
  __syncthreads();
  const int r = t >> 1, half = t & 1;
  const int row = r < nrows ? r : NV;   // threads past the rows sum the norm row (used when with_norm)
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (r < nrows || (with_norm && r == nrows)) {
    const float* src = &tile.v[row][half * (kTSub / 2)];
#pragma unroll 4
    for (int i = 0; i < kTSub / 2; i += 4) {
      s0 += (double)src[i];
      s1 += (double)src[i + 1];
      s2 += (double)src[i + 2];
      s3 += (double)src[i + 3];
    }
  }
  double s = (s0 + s1) + (s2 + s3);
  s += __shfl_xor(s, 1, 64);
  if (half == 0) {
    if (r < nrows) out[r] = cd{s, 0.0};
    else if (with_norm && r == nrows) out[norm_slot] = cd{s, 0.0};
  }
}

// step j, first pass: W = s_j K_hat V_j (stored), partials V_l . W for l <= j
template <int NV>
__global__ __launch_bounds__(kTSub) void k_lz_dots_t(LzCtx<float> c, int j) {
  static_assert(kTSub == 128 && kChunk % kTSub == 0, "two waves per block, whole sub-tiles per chunk");
  static_assert(NV + 1 <= kTSub / 2, "two threads per row in the block reduction");
  __shared__ LzTile<NV> tile;
  const int sys = blockIdx.y, chunk = blockIdx.x, t = threadIdx.x, lane = t & 63;
  if (!c.st[sys].in_cycle) return;
  const uint32_t N = (uint32_t)c.g.N;
  const uint32_t sv = N * 4u, sj_off = (uint32_t)j * sv;
  const Rsrc rv = make_rsrc(c.V + (size_t)sys * c.vdim * N, (uint32_t)c.vdim * sv);
  float* wv = c.W + (size_t)sys * N;
  const double sj = c.small[(size_t)sys * c.sl.total + c.sl.vs + j].re;
  const float ih2 = (float)(c.g.inv_h2 * sj), rob = (float)(c.sigp * c.g.inv_h * sj), tau = (float)(c.tau * sj);
  const uint32_t sy = (uint32_t)c.g.nx, sz = (uint32_t)c.g.nx * (uint32_t)c.g.ny;
  const int nv = j + 1;
  float acc[NV];
#pragma unroll
  for (int l = 0; l < NV; ++l) acc[l] = 0.f;
  for (int sub = 0; sub < kChunk / kTSub; ++sub) {
    const uint32_t n = (uint32_t)chunk * kChunk + (uint32_t)sub * kTSub + (uint32_t)t;
    const bool ok = n < N;
    const uint32_t vo = ok ? n * 4u : kOutside;
    const VoxelInfo vi = voxel_info(c.g, ok ? n : 0u);
    const float xc = ld_f(rv, vo, sj_off);
    float xm = ld_f(rv, lane == 0 && ok && vi.i > 0 ? (n - 1u) * 4u : kOutside, sj_off);
    float xp = ld_f(rv, lane == 63 && ok && vi.i < c.g.nx - 1 ? (n + 1u) * 4u : kOutside, sj_off);
    const float ym = ld_f(rv, ok && vi.j > 0 ? (n - sy) * 4u : kOutside, sj_off);
    const float yp = ld_f(rv, ok && vi.j < c.g.ny - 1 ? (n + sy) * 4u : kOutside, sj_off);
    const float zm = ld_f(rv, ok && vi.k > 0 ? (n - sz) * 4u : kOutside, sj_off);
    const float zp = ld_f(rv, ok && vi.k < c.g.nz - 1 ? (n + sz) * 4u : kOutside, sj_off);
    // basis vectors l < j (streamed; V_j is the centre); the rows past the step's j + 1 of a
    // larger instance read zero, and the last row needs no load
    float vr[NV];
#pragma unroll
    for (int l = 0; l + 1 < NV; ++l) vr[l] = ld_f_nt(rv, l < j ? vo : kOutside, (uint32_t)l * sv);
    vr[NV - 1] = 0.f;
    const float mu = c.mu && ok ? c.mu[n] : 0.f;
    // x neighbours of lanes 1..62 (and the inner one of lanes 0 and 63) from the adjacent lanes
    const float pv = lane_prev(xc), nxv = lane_next(xc);
    if (lane != 0) xm = vi.i > 0 ? pv : 0.f;
    if (lane != 63) xp = vi.i < c.g.nx - 1 ? nxv : 0.f;
    const float w = ok ? ih2 * (diag_k_of(vi) * xc - (((xm + xp) + (ym + yp)) + (zm + zp))) +
                             (rob * (float)vi.nrobin + tau * mu) * xc
                       : 0.f;
    if (ok) wv[n] = w;
#pragma unroll
    for (int l = 0; l < NV; ++l) acc[l] += (l == j ? xc : vr[l]) * w;
  }
  lz_flush_t<NV>(acc, nv, false, 0.f, tile, c.part + part_base(sys, c.nchunks, chunk, c.ndots), 0);
}

// step j, first projection w' = W - sum_l coefA_l V_l (stored as V_{j+1}), second-pass partials
// V_l . w' and |w'|^2
template <int NV>
__global__ __launch_bounds__(kTSub) void k_lz_update_t(LzCtx<float> c, int j) {
  static_assert(NV + 1 <= kTSub / 2, "two threads per row in the block reduction");
  __shared__ LzTile<NV> tile;
  const int sys = blockIdx.y, chunk = blockIdx.x, t = threadIdx.x;
  if (!c.st[sys].in_cycle) return;
  const uint32_t N = (uint32_t)c.g.N;
  const uint32_t sv = N * 4u;
  float* Vs = c.V + (size_t)sys * c.vdim * N;
  const Rsrc rv = make_rsrc(Vs, (uint32_t)c.vdim * sv);
  const Rsrc rw = make_rsrc(c.W + (size_t)sys * N, sv);
  float* vn = Vs + (size_t)(j + 1) * N;
  const cd* coef = c.small + (size_t)sys * c.sl.total + c.sl.coefA;
  const int nv = j + 1;
  float h[NV], acc[NV], nrm = 0.f;
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    h[l] = l < nv ? (float)coef[l].re : 0.f;
    acc[l] = 0.f;
  }
  for (int sub = 0; sub < kChunk / kTSub; ++sub) {
    const uint32_t n = (uint32_t)chunk * kChunk + (uint32_t)sub * kTSub + (uint32_t)t;
    const bool ok = n < N;
    const uint32_t vo = ok ? n * 4u : kOutside;
    // rows l >= j + 1 of an instance larger than the step read zero
    float vr[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) vr[l] = ld_f_nt(rv, l < nv ? vo : kOutside, (uint32_t)l * sv);
    float w = ld_f(rw, vo, 0u);
#pragma unroll
    for (int l = 0; l < NV; ++l) w -= h[l] * vr[l];
    if (ok) vn[n] = w;
#pragma unroll
    for (int l = 0; l < NV; ++l) acc[l] += vr[l] * w;
    nrm += w * w;
  }
  lz_flush_t<NV>(acc, nv, true, nrm, tile, c.part + part_base(sys, c.nchunks, chunk, c.ndots), slot_norm(0, c.mkmax));
}

}  // namespace hydot
