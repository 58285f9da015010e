// Matrix-free Born products (Sec. 2.1 integral equation with the adjoint field;
// rows of H in eq. measurement), never forming J:
//   J v  : y[c][l][s][d] = -h^3 sum_k phi_s(k) v_c(k) phi_d(k)   (per wavelength a
//          dense contraction Phi_s^T diag(v) Phi_d over the voxels),
//   J^H w: g[k] = -h^3 sum_l sum_d conj(phi_d(k)) sum_s conj(phi_s(k)) w[l][s][d].
//
// Complex products run on real MFMA tiles by real-ification: the operand rows
// are [Re; Im] of the complex rows, so one real product carries all four real
// partial products of the complex one.  FP32 fields use
// v_mfma_f32_16x16x4_f32 with per-stage FP64 accumulation and FP64 split-K
// sums; FP64 fields use v_mfma_f64_16x16x4_f64.
//
// J v stages coalesced row segments of Phi_s v and Phi_d through LDS (the MFMA
// operand layout puts 16 different rows in the lanes of one k-slot).  J^H w feeds
// its MFMA operands straight from global memory with no LDS and no barrier: the
// 16 lanes of a k-slot read 16 consecutive voxels of one source row.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "operator.h"

namespace hydot {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Both instructions take A[row = lane%16][k = lane/16] and B[k = lane/16][col = lane%16];
// accumulator register r of lane l holds column l%16 and row out_row(l, r), which
// differs between the two (measured on gfx950).
template <> struct Mfma<float> {
  using acc = f32x4;
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
  using acc = f64x4;
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int lane, int r) { return 4 * r + (lane >> 4); }
};

constexpr size_t kLdsCap = 64 * 1024;   // LDS budget per block of J v

inline int pad8(int x) { return (x + 7) / 8 * 8; }

// ---------------------------------------------------------------- J v
// Block = 4 waves on one (split, wavelength, probe vector).  Rows of the real
// product: a < Sp -> Re(phi_s v), a >= Sp -> Im(phi_s v); columns b < Dp ->
// Re phi_d, b >= Dp -> Im phi_d.  Wave w owns output tiles w, w+4, ...
template <typename T, int TPW, int kKT>
__global__ __launch_bounds__(kBlock) void k_born_apply(int N, int S, int D, int Sp, int Dp, int64_t lam_stride,
                                                      const cplx<T>* __restrict__ phs,
                                                      const cplx<T>* __restrict__ phd,
                                                      const T* __restrict__ v, int kb, int L,
                                                      double* __restrict__ part) {
  constexpr int kKTP = kKT + 4;         // padded LDS row
  extern __shared__ unsigned char smem_raw[];
  T* As = (T*)smem_raw;                 // [2Sp][kKTP]
  T* Bs = As + 2 * Sp * kKTP;           // [2Dp][kKTP]
  T* vs = Bs + 2 * Dp * kKTP;           // [kKT]
  const int split = blockIdx.x, l = blockIdx.y, c = blockIdx.z;
  const int nsplit = gridDim.x;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  const int TA = 2 * Sp / 16, TB = 2 * Dp / 16, T_all = TA * TB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const cplx<T>* ps = phs + (size_t)l * lam_stride * N;
  const cplx<T>* pd = phd + (size_t)l * lam_stride * N;
  const T* vc = v + (size_t)c * N;
  using MA = typename Mfma<T>::acc;
  MA acc[TPW];
  f64x4 tot[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    acc[t] = MA{0, 0, 0, 0};
    tot[t] = f64x4{0, 0, 0, 0};
  }
  for (int kbase = k0; kbase < k1; kbase += kKT) {
    const int kn = min(kKT, k1 - kbase);
    for (int i = threadIdx.x; i < kKT; i += kBlock) vs[i] = i < kn ? vc[kbase + i] : (T)0;
    __syncthreads();
    for (int i = threadIdx.x; i < Sp * kKT; i += kBlock) {
      const int s = i / kKT, kk = i % kKT;
      cplx<T> z{0, 0};
      if (s < S && kk < kn) z = ps[(size_t)s * N + kbase + kk];
      const T vv = vs[kk];
      As[s * kKTP + kk] = z.re * vv;
      As[(Sp + s) * kKTP + kk] = z.im * vv;
    }
    for (int i = threadIdx.x; i < Dp * kKT; i += kBlock) {
      const int d = i / kKT, kk = i % kKT;
      cplx<T> z{0, 0};
      if (d < D && kk < kn) z = pd[(size_t)d * N + kbase + kk];
      Bs[d * kKTP + kk] = z.re;
      Bs[(Dp + d) * kKTP + kk] = z.im;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile < T_all) {
        const int ta = tile / TB, tb = tile % TB;
        const T* arow = As + (ta * 16 + (lane & 15)) * kKTP + (lane >> 4);
        const T* brow = Bs + (tb * 16 + (lane & 15)) * kKTP + (lane >> 4);
#pragma unroll
        for (int kk = 0; kk < kKT; kk += 4) acc[t] = Mfma<T>::step(arow[kk], brow[kk], acc[t]);
        // FP64 accumulation across stages
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[t][r] += (double)acc[t][r];
        acc[t] = MA{0, 0, 0, 0};
      }
    }
    __syncthreads();
  }
  // partial tile sums: part[((c*L + l)*nsplit + split)][2Sp][2Dp]
  double* out = part + ((size_t)(c * L + l) * nsplit + split) * (size_t)(2 * Sp) * (2 * Dp);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile < T_all) {
      const int ta = tile / TB, tb = tile % TB;
      const int col = tb * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ta * 16 + Mfma<T>::out_row(lane, r);
        out[(size_t)row * (2 * Dp) + col] = tot[t][r];
      }
    }
  }
}

// Sum the split-K partials in a fixed order and assemble the complex result.
template <typename O>
__global__ void k_born_apply_finish(int S, int D, int Sp, int Dp, int nsplit, int L, const double* part,
                                    double scale, O* y) {
  const int cl = blockIdx.x;  // c*L + l
  const size_t tile = (size_t)(2 * Sp) * (2 * Dp);
  for (int e = threadIdx.x; e < S * D; e += blockDim.x) {
    const int s = e / D, d = e % D;
    double rr = 0, ii = 0, ri = 0, ir = 0;
    for (int sp = 0; sp < nsplit; ++sp) {
      const double* P = part + ((size_t)cl * nsplit + sp) * tile;
      rr += P[(size_t)s * 2 * Dp + d];
      ii += P[(size_t)(Sp + s) * 2 * Dp + Dp + d];
      ri += P[(size_t)s * 2 * Dp + Dp + d];
      ir += P[(size_t)(Sp + s) * 2 * Dp + d];
    }
    const cd z{scale * (rr - ii), scale * (ri + ir)};
    y[(size_t)cl * S * D + e] = Store<O>::from(z);
  }
}

// ---------------------------------------------------------------- J^H w
// Each wave owns 16 voxels and loops over all wavelengths, keeping g for its
// voxels in FP64 registers.  Per wavelength, T = A'' B'' on MFMA with
// A'' = [Re phi_s | Im phi_s] (voxels x 2Sp) and B'' = [[Re w, Im w], [Im w, -Re w]]
// (2Sp x 2Dp), giving [Re T | Im T] with T[k][d] = sum_s conj(phi_s(k)) w[s][d];
// the epilogue contracts T with conj(phi_d) per voxel.  Lane (voxel i = lane%16,
// slot gq = lane/16) loads the sources s = gq (mod 4) of its voxel once and uses
// their real parts for k-index s and imaginary parts for k-index Sp + s.
template <typename T, int TBM, int SQ>
__global__ __launch_bounds__(kBlock) void k_born_adjoint(int N, int S, int D, int Sp, int Dp, int64_t lam_stride,
                                                        int L, const cplx<T>* __restrict__ phs,
                                                        const cplx<T>* __restrict__ phd,
                                                        const cplx<T>* __restrict__ w, double scale,
                                                        cplx<T>* __restrict__ g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, gq = lane >> 4;
  const int vox0 = (blockIdx.x * 4 + wave) * 16;
  const int TB = 2 * Dp / 16;
  const int vox = vox0 + i16;
  const bool vok = vox < N;
  using MA = typename Mfma<T>::acc;
  double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
  for (int l = 0; l < L; ++l) {
    const cplx<T>* ps = phs + (size_t)l * lam_stride * N;
    const cplx<T>* pd = phd + (size_t)l * lam_stride * N;
    const cplx<T>* wl = w + (size_t)l * S * D;
    cplx<T> z[SQ];   // phi_s[s][vox] for s = gq + 4q
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int s = gq + 4 * q;
      z[q] = (q < Sp / 4 && s < S && vok) ? ps[(size_t)s * N + vox] : cplx<T>{0, 0};
    }
    MA acc[TBM];
#pragma unroll
    for (int t = 0; t < TBM; ++t) acc[t] = MA{0, 0, 0, 0};
    // k-index s = gq + 4q uses Re z[q], k-index Sp + s uses Im z[q]
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      if (q < Sp / 4) {
        const int s = gq + 4 * q;
#pragma unroll
        for (int t = 0; t < TBM; ++t) {
          if (t < TB) {
            const int col = t * 16 + i16;
            const bool imcol = col >= Dp;
            const int d = imcol ? col - Dp : col;
            const cplx<T> ww = (s < S && d < D) ? wl[s * D + d] : cplx<T>{0, 0};
            // B'' = [[Re w, Im w], [Im w, -Re w]]: rows of Re phi_s, then rows of Im phi_s
            acc[t] = Mfma<T>::step(z[q].re, imcol ? ww.im : ww.re, acc[t]);
            acc[t] = Mfma<T>::step(z[q].im, imcol ? -ww.re : ww.im, acc[t]);
          }
        }
      }
    }
    // epilogue: lane holds T[voxel vox0 + out_row(lane, r)][col t*16 + lane%16]
#pragma unroll
    for (int t = 0; t < TBM; ++t) {
      if (t < TB) {
        const int col = t * 16 + i16;
        const bool imcol = col >= Dp;
        const int d = imcol ? col - Dp : col;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int vv = vox0 + Mfma<T>::out_row(lane, r);
          cplx<T> ph{0, 0};
          if (d < D && vv < N) ph = pd[(size_t)d * N + vv];
          const double e = ph.re, f = ph.im;
          const double tv = (double)acc[t][r];
          if (!imcol) {          // Re T column
            gre[r] += e * tv;
            gim[r] -= f * tv;
          } else {               // Im T column
            gre[r] += f * tv;
            gim[r] += e * tv;
          }
        }
      }
    }
  }
  // reduce over the 16 lanes that share a voxel (lane & 15 varies)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      gre[r] += __shfl_xor(gre[r], off, 64);
      gim[r] += __shfl_xor(gim[r], off, 64);
    }
  }
  if (i16 == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vv = vox0 + Mfma<T>::out_row(lane, r);
      if (vv < N) g[vv] = cplx<T>{(T)(scale * gre[r]), (T)(scale * gim[r])};
    }
  }
}

template <typename T>
hydot_status born_apply_impl(const hydot_operator* op, const void* phs, int S, const void* phd, int D,
                             int64_t ls, const void* v, int n_v, void* y, hipStream_t stream) {
  const int N = op->gp.N, L = op->L;
  const int Sp = pad8(S), Dp = pad8(D);
  const int T_all = (2 * Sp / 16) * (2 * Dp / 16);
  const int tpw = (T_all + 3) / 4;
  // voxels per LDS stage: 32 when the staged rows fit the LDS budget (unless the tuning
  // asks for 16), else 16; larger stages lower the resident blocks per CU and measure slower
  const hydot_tuning tu = resolved_tuning(op->tune);
  const bool fits32 = (size_t)(2 * Sp + 2 * Dp) * 36 * sizeof(T) + 32 * sizeof(T) <= kLdsCap;
  const int kt = fits32 && tu.born_stage != 16 ? 32 : 16;
  // split-K over voxels so the grid has about born_blocks blocks
  const int max_split = (N + kt - 1) / kt;
  int nsplit = std::max(1, std::min(max_split, (tu.born_blocks + L * n_v - 1) / (L * n_v)));
  int kb = (N + nsplit - 1) / nsplit;
  kb = (kb + kt - 1) / kt * kt;
  nsplit = (N + kb - 1) / kb;
  const size_t pbytes = (size_t)n_v * L * nsplit * (2 * Sp) * (2 * Dp) * sizeof(double);
  void* part = nullptr;
  HYDOT_HIP(hipMallocAsync(&part, pbytes, stream));
  const size_t lds = (size_t)(2 * Sp + 2 * Dp) * (kt + 4) * sizeof(T) + kt * sizeof(T);
  dim3 grid(nsplit, L, n_v);
#define HYDOT_BA(TP, KT)                                                                                      \
  hipLaunchKernelGGL((k_born_apply<T, TP, KT>), grid, dim3(kBlock), lds, stream, N, S, D, Sp, Dp, ls,        \
                     (const cplx<T>*)phs, (const cplx<T>*)phd, (const T*)v, kb, L, (double*)part)
#define HYDOT_BA_T(TP) \
  if (kt == 32) HYDOT_BA(TP, 32); else HYDOT_BA(TP, 16);
  if (tpw <= 1) { HYDOT_BA_T(1) }
  else if (tpw <= 2) { HYDOT_BA_T(2) }
  else if (tpw <= 4) { HYDOT_BA_T(4) }
  else if (tpw <= 8) { HYDOT_BA_T(8) }
  else { HYDOT_BA_T(16) }
#undef HYDOT_BA_T
#undef HYDOT_BA
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_apply_finish<cplx<T>>), dim3(n_v * L), dim3(256), 0, stream, S, D, Sp, Dp, nsplit, L,
                     (const double*)part, -h * h * h, (cplx<T>*)y);
  hipError_t e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(part, stream);
  if (e != hipSuccess) return hip_check(e, "born_apply launch");
  if (e2 != hipSuccess) return hip_check(e2, "born_apply free");
  return HYDOT_OK;
}

template <typename T>
hydot_status born_adjoint_impl(const hydot_operator* op, const void* phs, int S, const void* phd, int D,
                               int64_t ls, const void* w, void* g, hipStream_t stream) {
  const int N = op->gp.N, L = op->L;
  const int Sp = pad8(S), Dp = pad8(D);
  const int TB = 2 * Dp / 16;
  dim3 grid((N + 63) / 64);
  const double h = op->grid.h_mm;
  const double sc = -h * h * h;
#define HYDOT_BJ(TBM, SQ)                                                                                   \
  hipLaunchKernelGGL((k_born_adjoint<T, TBM, SQ>), grid, dim3(kBlock), 0, stream, N, S, D, Sp, Dp, ls, L,   \
                     (const cplx<T>*)phs, (const cplx<T>*)phd, (const cplx<T>*)w, sc, (cplx<T>*)g)
#define HYDOT_BJ_S(TBM) \
  if (Sp <= 16) HYDOT_BJ(TBM, 4); else if (Sp <= 32) HYDOT_BJ(TBM, 8); else HYDOT_BJ(TBM, 16);
  if (TB <= 1) { HYDOT_BJ_S(1) }
  else if (TB <= 2) { HYDOT_BJ_S(2) }
  else if (TB <= 4) { HYDOT_BJ_S(4) }
  else { HYDOT_BJ_S(8) }
#undef HYDOT_BJ_S
#undef HYDOT_BJ
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

static hydot_status born_check(const hydot_operator* op, const void* phs, int S, const void* phd, int D,
                               int64_t ls, hydot_dtype dt) {
  if (!op) return fail(HYDOT_EINVAL, "born: null operator");
  if (!phs || !phd) return fail(HYDOT_EINVAL, "born: null field pointer");
  if (S < 1 || S > 64 || D < 1 || D > 64) return fail(HYDOT_EINVAL, "born: S and D must be in [1, 64]");
  if (ls < std::max(S, D)) return fail(HYDOT_EINVAL, "born: lam_stride must be >= max(S, D)");
  if (dt != HYDOT_C128 && dt != HYDOT_C64) return fail(HYDOT_EUNSUPPORTED, "born: field_dtype must be C128 or C64");
  return HYDOT_OK;
}

}  // namespace hydot

using namespace hydot;

extern "C" {

hydot_status hydot_born_apply(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                              int32_t D, int64_t lam_stride, hydot_dtype field_dtype, const void* v, int32_t n_v,
                              void* y, hipStream_t stream) {
  hydot_status s = born_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype);
  if (s != HYDOT_OK) return s;
  if (!v || !y) return fail(HYDOT_EINVAL, "born_apply: null v or y");
  if (n_v < 1 || n_v > 64) return fail(HYDOT_EINVAL, "born_apply: n_v must be in [1, 64]");
  if (field_dtype == HYDOT_C128) return born_apply_impl<double>(op, phi_src, S, phi_det, D, lam_stride, v, n_v, y, stream);
  return born_apply_impl<float>(op, phi_src, S, phi_det, D, lam_stride, v, n_v, y, stream);
}

hydot_status hydot_born_apply_adjoint(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                                      int32_t D, int64_t lam_stride, hydot_dtype field_dtype, const void* w, void* g,
                                      hipStream_t stream) {
  hydot_status s = born_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype);
  if (s != HYDOT_OK) return s;
  if (!w || !g) return fail(HYDOT_EINVAL, "born_apply_adjoint: null w or g");
  if (field_dtype == HYDOT_C128) return born_adjoint_impl<double>(op, phi_src, S, phi_det, D, lam_stride, w, g, stream);
  return born_adjoint_impl<float>(op, phi_src, S, phi_det, D, lam_stride, w, g, stream);
}

hydot_status hydot_autotune_born(hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det, int32_t D,
                                 int64_t lam_stride, hydot_dtype field_dtype, const void* v, int32_t n_v, void* y,
                                 hydot_tune_trial* trials, int32_t max_trials, int32_t* n_trials, hipStream_t stream) {
  if (!op) return fail(HYDOT_EINVAL, "autotune_born: null operator");
  if (max_trials < 0 || (max_trials > 0 && !trials)) return fail(HYDOT_EINVAL, "autotune_born: bad trials buffer");
  const hydot_tuning keep = op->tune;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HYDOT_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HYDOT_EDEVICE, "autotune_born: event create");
  }
  const int stages[2] = {16, 32};
  const int blocks[5] = {1024, 2048, 4096, 8192, 16384};
  int count = 0;
  double best = 1e300;
  hydot_tuning best_t = resolved_tuning(keep);
  hydot_status err = HYDOT_OK;
  for (int is = 0; is < 2 && err == HYDOT_OK; ++is)
    for (int ib = 0; ib < 5 && err == HYDOT_OK; ++ib) {
      hydot_tuning t = resolved_tuning(keep);
      t.born_stage = stages[is];
      t.born_blocks = blocks[ib];
      op->tune = t;
      float ms[5];
      for (int rep = 0; rep < 6 && err == HYDOT_OK; ++rep) {   // first call warms up
        if (hipEventRecord(e0, stream) != hipSuccess) err = fail(HYDOT_EDEVICE, "autotune_born: event record");
        if (err == HYDOT_OK)
          err = hydot_born_apply(op, phi_src, S, phi_det, D, lam_stride, field_dtype, v, n_v, y, stream);
        if (err == HYDOT_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
          err = fail(HYDOT_EDEVICE, "autotune_born: event wait");
        if (err == HYDOT_OK && rep > 0 && hipEventElapsedTime(&ms[rep - 1], e0, e1) != hipSuccess)
          err = fail(HYDOT_EDEVICE, "autotune_born: elapsed time");
      }
      if (err != HYDOT_OK) break;
      std::sort(ms, ms + 5);
      if (count < max_trials) trials[count] = hydot_tune_trial{t, (double)ms[2]};
      ++count;
      if (ms[2] < best) {
        best = ms[2];
        best_t = t;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != HYDOT_OK) {
    op->tune = keep;
    return err;
  }
  op->tune = best_t;
  if (n_trials) *n_trials = count;
  return HYDOT_OK;
}

}  // extern "C"
