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
#include <mutex>
#include <string>
#include <type_traits>

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
// Field storage: complex FP64, complex FP32 or complex BF16 (widened on load).
template <typename TS> struct Field;
template <> struct Field<cd> {
  using real = double;
  __device__ static inline cd get(const cd* p, size_t i) { return p[i]; }
};
template <> struct Field<cf> {
  using real = float;
  __device__ static inline cf get(const cf* p, size_t i) { return p[i]; }
};
template <> struct Field<cbf> {
  using real = float;
  __device__ static inline cf get(const cbf* p, size_t i) {
    const cbf z = p[i];
    return cf{bf16_value(z.re), bf16_value(z.im)};
  }
};

// Products of J v: CM_F64 / CM_F32 run the MFMA of the storage precision; CM_BF16
// rounds both operands (phi_s v formed in FP32, and phi_d) to BF16 for
// v_mfma_f32_16x16x32_bf16; CM_SPLIT splits each FP32 operand into hi + lo BF16 parts
// and accumulates hi*hi + hi*lo + lo*hi (three BF16 MFMAs).
enum BornCompute { CM_F64 = 0, CM_F32 = 1, CM_BF16 = 2, CM_SPLIT = 3 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline bf16x8 to_bf16x8(const float* x) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)x[i];
  return r;
}
__device__ inline bf16x8 bf16_residual(const float* x, bf16x8 hi) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)(x[i] - (float)hi[i]);
  return r;
}

// Block = 4 waves on one (split over voxels, wavelength, group of NVB probe vectors).
// Each stage of KT voxels stages the real-ified rows [Re; Im] of Phi_s (2Sp rows) and
// Phi_d (2Dp rows) and the NVB probe-vector segments in LDS once; every probe vector
// of the group then reuses them (v_c is applied to the A operand in registers).  The
// next stage's global loads are issued before this stage's MFMAs.  Wave w owns output
// tiles w, w+4, ... of the (2Sp x 2Dp) real product, per probe vector.
template <typename TS, int CM, int TPW, int NVB, int KT, int EM>
__global__ __launch_bounds__(kBlock) void k_born_jv(int N, int S, int D, int Sp, int Dp, int64_t lam_stride,
                                                   const TS* __restrict__ phs, const TS* __restrict__ phd,
                                                   const typename Field<TS>::real* __restrict__ v, int n_v, int kb,
                                                   int L, double* __restrict__ part) {
  using R = typename Field<TS>::real;   // LDS and operand precision before the BF16 rounding
  constexpr int KTP = KT + 4;           // padded LDS row
  constexpr int kMaxE = EM;             // staged elements per thread per row set (>= pad8(S)*KT/kBlock)
  constexpr bool kFold = NVB == 1;      // one probe vector: fold v into the staged Phi_s rows
  static_assert(CM == CM_F64 || CM == CM_F32 || KT == 32, "BF16 products take 32 voxels per MFMA");
  extern __shared__ unsigned char smem_raw[];
  R* As = (R*)smem_raw;                 // [2Sp][KTP]
  R* Bs = As + 2 * Sp * KTP;            // [2Dp][KTP]
  R* Vs = Bs + 2 * Dp * KTP;            // [NVB][KT]
  const int split = blockIdx.x, l = blockIdx.y, cv0 = blockIdx.z * NVB;
  const int nsplit = gridDim.x;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  const int TB = 2 * Dp / 16, T_all = (2 * Sp / 16) * TB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const TS* ps = phs + (size_t)l * lam_stride * N;
  const TS* pd = phd + (size_t)l * lam_stride * N;
  const int ns = Sp * KT, nd = Dp * KT;   // staged (row, voxel) pairs of each row set
  const int es = (ns + kBlock - 1) / kBlock, ed = (nd + kBlock - 1) / kBlock;
  using CM_ACC = typename std::conditional<CM == CM_F64, f64x4, f32x4>::type;
  CM_ACC acc[TPW][NVB];
  f64x4 tot[TPW][NVB];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < NVB; ++c) {
      acc[t][c] = CM_ACC{0, 0, 0, 0};
      tot[t][c] = f64x4{0, 0, 0, 0};
    }
  // register stage: element e of this thread is row i / KT, voxel i % KT with i = tid + e * kBlock
  cplx<R> rs[kMaxE], rd[kMaxE];
  R rv = 0;
  auto fetch = [&](int kbase) {
    const int kn = min(KT, k1 - kbase);
#pragma unroll
    for (int e = 0; e < kMaxE; ++e) {
      if (e < es && tid + e * kBlock < ns) {
        const int i = tid + e * kBlock, row = i / KT, kk = i % KT;
        rs[e] = row < S && kk < kn ? Field<TS>::get(ps, (size_t)row * N + kbase + kk) : cplx<R>{0, 0};
      }
      if (e < ed && tid + e * kBlock < nd) {
        const int i = tid + e * kBlock, row = i / KT, kk = i % KT;
        rd[e] = row < D && kk < kn ? Field<TS>::get(pd, (size_t)row * N + kbase + kk) : cplx<R>{0, 0};
      }
    }
    if (kFold) {
#pragma unroll
      for (int e = 0; e < kMaxE; ++e)
        if (e < es && tid + e * kBlock < ns) {
          const int kk = (tid + e * kBlock) % KT;
          const R vv = cv0 < n_v && kk < kn ? v[(size_t)cv0 * N + kbase + kk] : (R)0;
          rs[e].re *= vv;
          rs[e].im *= vv;
        }
    } else if (tid < NVB * KT) {
      const int c = tid / KT, kk = tid % KT;
      rv = cv0 + c < n_v && kk < kn ? v[(size_t)(cv0 + c) * N + kbase + kk] : (R)0;
    }
  };
  fetch(k0);
  for (int kbase = k0; kbase < k1; kbase += KT) {
#pragma unroll
    for (int e = 0; e < kMaxE; ++e) {
      if (e < es && tid + e * kBlock < ns) {
        const int i = tid + e * kBlock, row = i / KT, kk = i % KT;
        As[row * KTP + kk] = rs[e].re;
        As[(Sp + row) * KTP + kk] = rs[e].im;
      }
      if (e < ed && tid + e * kBlock < nd) {
        const int i = tid + e * kBlock, row = i / KT, kk = i % KT;
        Bs[row * KTP + kk] = rd[e].re;
        Bs[(Dp + row) * KTP + kk] = rd[e].im;
      }
    }
    if (!kFold && tid < NVB * KT) Vs[tid] = rv;
    __syncthreads();
    if (kbase + KT < k1) fetch(kbase + KT);   // in flight during the products
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile < T_all) {
        const int ta = tile / TB, tb = tile % TB;
        const int g = lane >> 4;
        const R* arow = As + (ta * 16 + (lane & 15)) * KTP;
        const R* brow = Bs + (tb * 16 + (lane & 15)) * KTP;
        if constexpr (CM == CM_F64 || CM == CM_F32) {
#pragma unroll
          for (int kk = 0; kk < KT; kk += 4) {
            const R a = arow[kk + g], b = brow[kk + g];
#pragma unroll
            for (int c = 0; c < NVB; ++c)
              acc[t][c] = Mfma<R>::step(kFold ? a : a * Vs[c * KT + kk + g], b, acc[t][c]);
          }
        } else {
          float bx[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) bx[i] = brow[8 * g + i];
          const bf16x8 bh = to_bf16x8(bx);
          bf16x8 bl;
          if constexpr (CM == CM_SPLIT) bl = bf16_residual(bx, bh);
#pragma unroll
          for (int c = 0; c < NVB; ++c) {
            float ax[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) ax[i] = kFold ? arow[8 * g + i] : arow[8 * g + i] * Vs[c * KT + 8 * g + i];
            const bf16x8 ah = to_bf16x8(ax);
            acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[t][c], 0, 0, 0);
            if constexpr (CM == CM_SPLIT) {
              const bf16x8 al = bf16_residual(ax, ah);
              acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[t][c], 0, 0, 0);
              acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[t][c], 0, 0, 0);
            }
          }
        }
        if constexpr (CM != CM_F64) {   // FP64 accumulation across stages
#pragma unroll
          for (int c = 0; c < NVB; ++c) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[t][c][r] += (double)acc[t][c][r];
            acc[t][c] = CM_ACC{0, 0, 0, 0};
          }
        }
      }
    }
    __syncthreads();
  }
  // partial tile sums: part[((c*L + l)*nsplit + split)][2Sp][2Dp]
#pragma unroll
  for (int c = 0; c < NVB; ++c) {
    if (cv0 + c >= n_v) break;
    double* out = part + ((size_t)((cv0 + c) * L + l) * nsplit + split) * (size_t)(2 * Sp) * (2 * Dp);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile < T_all) {
        const int ta = tile / TB, tb = tile % TB;
        const int col = tb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = ta * 16 + Mfma<R>::out_row(lane, r);
          out[(size_t)row * (2 * Dp) + col] = CM == CM_F64 ? (double)acc[t][c][r] : tot[t][c][r];
        }
      }
    }
  }
}

// Sum the split-K partials in a fixed order and assemble the complex result.
template <typename O>
__global__ void k_born_apply_finish(int S, int D, int Sp, int Dp, int nsplit, int L, const double* part,
                                    double scale, O* y) {
  const int cl = blockIdx.y;  // c*L + l
  const size_t tile = (size_t)(2 * Sp) * (2 * Dp);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;   // pair s*D + d
  if (e < S * D) {
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

// ---------------------------------------------------------------- J v, blocks of probe vectors
// With many probe vectors the contraction is regrouped over source-detector pairs:
//   y[c][l][s][d] = -h^3 sum_k P_l[s,d](k) v_c(k),   P_l[s,d](k) = phi_s(k) phi_d(k),
// a product of the (S D x N) complex pair matrix with the (N x n_v) real probe block.  The
// pair products are formed in registers, one complex multiply per pair and voxel shared by all
// probe vectors, and the MFMA runs on the rows [Re P; Im P] against V: 4 S D N real
// multiply-adds per probe vector where the real-ified complex product of k_born_jv takes
// 8 S D N, at the cost of padding the probe vectors to a multiple of 16.
// Block = 4 waves on (split over voxels, wavelength, tile of 8 sources x 8 detectors).  Wave w
// owns the 16 pairs (2w + i/8, i%8), i < 16, of the tile as an Re tile and an Im tile of 16
// rows, each against NCT tiles of 16 probe vectors.  Each stage of 32 voxels stages the 8 + 8
// field rows and the probe-vector segments in LDS; the next stage's global loads are issued
// before this stage's products.  FP32 products fold their stage sums into FP64 as k_born_jv.
// CM selects the product arithmetic as in k_born_jv: the MFMA of the field precision (CM_F32,
// CM_F64), or P formed in FP32 and rounded with the probe vectors to BF16 for
// v_mfma_f32_16x16x32_bf16 (CM_BF16; one MFMA k-step per 32-voxel stage, lane (i, g) supplying
// the pair products of voxels 8g..8g+7), or both split into hi + lo BF16 parts with
// hi*hi + hi*lo + lo*hi accumulated (CM_SPLIT).
constexpr int kPairsMinNv = HYDOT_BORN_PAIRS_MIN_NV;   // fewer: the padding to 16 costs more than it saves

template <typename TS, int CM, int NCT>
__global__ __launch_bounds__(kBlock) void k_born_jv_pairs(int N, int S, int D, int64_t lam_stride,
                                                         const TS* __restrict__ phs, const TS* __restrict__ phd,
                                                         const typename Field<TS>::real* __restrict__ v, int n_v,
                                                         int kb, int L, int ntd, double* __restrict__ part) {
  using R = typename Field<TS>::real;
  using C = cplx<R>;
  using ACC = typename Mfma<R>::acc;
  constexpr bool kFp32 = std::is_same<R, float>::value;
  constexpr int KT = 32, CP = KT + 4, VP = KT + 4;   // voxels per stage, padded LDS rows
  constexpr int NE = NCT * 16 * KT / kBlock;          // staged probe-vector elements per thread
  __shared__ C Ps[8 * CP], Pd[8 * CP];
  __shared__ R Vs[NCT * 16 * VP];
  const int split = blockIdx.x, l = blockIdx.y, nsplit = gridDim.x;
  const int s0 = (blockIdx.z / ntd) * 8, d0 = (blockIdx.z % ntd) * 8;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const TS* ps = phs + (size_t)l * lam_stride * N;
  const TS* pd = phd + (size_t)l * lam_stride * N;
  ACC acc[2][NCT];
  f64x4 tot[2][NCT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      acc[t][c] = ACC{0, 0, 0, 0};
      tot[t][c] = f64x4{0, 0, 0, 0};
    }
  // staging: thread tid holds voxel tid % 32 of field row tid / 32 (sources and detectors) and
  // of probe vectors tid / 32 + 8 e
  const int srow = tid >> 5, skk = tid & 31;
  C rs, rd;
  R rv[NE];
  auto fetch = [&](int kbase) {
    const bool ok = skk < k1 - kbase;
    const size_t k = (size_t)kbase + skk;
    rs = ok && s0 + srow < S ? Field<TS>::get(ps, (size_t)(s0 + srow) * N + k) : C{0, 0};
    rd = ok && d0 + srow < D ? Field<TS>::get(pd, (size_t)(d0 + srow) * N + k) : C{0, 0};
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int col = srow + 8 * e;
      rv[e] = ok && col < n_v ? v[(size_t)col * N + k] : (R)0;
    }
  };
  const int i = lane & 15, g = lane >> 4;
  const C* prs = Ps + (2 * wave + (i >> 3)) * CP + g;
  const C* prd = Pd + (i & 7) * CP + g;
  const R* pv = Vs + i * VP + g;
  fetch(k0);
  for (int kbase = k0; kbase < k1; kbase += KT) {
    Ps[srow * CP + skk] = rs;
    Pd[srow * CP + skk] = rd;
#pragma unroll
    for (int e = 0; e < NE; ++e) Vs[(srow + 8 * e) * VP + skk] = rv[e];
    __syncthreads();
    if (kbase + KT < k1) fetch(kbase + KT);   // in flight during the products
    if constexpr (CM == CM_F32 || CM == CM_F64) {
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const C a = prs[kk], b = prd[kk];
        const R pre = a.re * b.re - a.im * b.im, pim = a.re * b.im + a.im * b.re;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const R bv = pv[c * 16 * VP + kk];
          acc[0][c] = Mfma<R>::step(pre, bv, acc[0][c]);
          acc[1][c] = Mfma<R>::step(pim, bv, acc[1][c]);
        }
      }
    } else {
      // voxels 8g .. 8g + 7 of the stage for this lane's pair (prs, prd, pv start at voxel g)
      float pre[8], pim[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const C a = prs[7 * g + e], b = prd[7 * g + e];
        pre[e] = a.re * b.re - a.im * b.im;
        pim[e] = a.re * b.im + a.im * b.re;
      }
      const bf16x8 rh = to_bf16x8(pre), ih = to_bf16x8(pim);
      bf16x8 rl, il;
      if constexpr (CM == CM_SPLIT) {
        rl = bf16_residual(pre, rh);
        il = bf16_residual(pim, ih);
      }
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        float vb[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) vb[e] = pv[c * 16 * VP + 7 * g + e];
        const bf16x8 vh = to_bf16x8(vb);
        acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rh, vh, acc[0][c], 0, 0, 0);
        acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ih, vh, acc[1][c], 0, 0, 0);
        if constexpr (CM == CM_SPLIT) {
          const bf16x8 vl = bf16_residual(vb, vh);
          acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rh, vl, acc[0][c], 0, 0, 0);
          acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rl, vh, acc[0][c], 0, 0, 0);
          acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ih, vl, acc[1][c], 0, 0, 0);
          acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(il, vh, acc[1][c], 0, 0, 0);
        }
      }
    }
    if constexpr (kFp32) {   // FP64 accumulation across stages
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
#pragma unroll
          for (int r = 0; r < 4; ++r) tot[t][c][r] += (double)acc[t][c][r];
          acc[t][c] = ACC{0, 0, 0, 0};
        }
    }
    __syncthreads();
  }
  // partial sums: part[(((c * L + l) * nsplit + split) * S + s) * D + d] = (Re, Im)
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    const int cv = c * 16 + i;
    if (cv >= n_v) continue;
    double* out = part + ((size_t)(cv * L + l) * nsplit + split) * (size_t)S * D * 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Mfma<R>::out_row(lane, r);
      const int s = s0 + 2 * wave + (row >> 3), d = d0 + (row & 7);
      if (s < S && d < D) {
        const size_t o = ((size_t)s * D + d) * 2;
        out[o] = kFp32 ? tot[0][c][r] : (double)acc[0][c][r];
        out[o + 1] = kFp32 ? tot[1][c][r] : (double)acc[1][c][r];
      }
    }
  }
}

// Sum the split partials of k_born_jv_pairs in a fixed order and scale by -h^3.
template <typename O>
__global__ void k_born_pairs_finish(int SD, int nsplit, int nout, const double* part, double scale, O* y) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;   // (c * L + l) * S D + pair
  if (e >= nout) return;
  const int cl = e / SD, pair = e - cl * SD;
  double re = 0, im = 0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* P = part + (((size_t)cl * nsplit + sp) * SD + pair) * 2;
    re += P[0];
    im += P[1];
  }
  y[e] = Store<O>::from(cd{scale * re, scale * im});
}

// ---------------------------------------------------------------- J^H w
// Each wave owns 16 voxels and loops over all wavelengths, keeping g for its
// voxels in FP64 registers.  Per wavelength, T = A'' B'' on MFMA with
// A'' = [Re phi_s | Im phi_s] (voxels x 2Sp) and B'' = [[Re w, Im w], [Im w, -Re w]]
// (2Sp x 2Dp), giving [Re T | Im T] with T[k][d] = sum_s conj(phi_s(k)) w[s][d];
// the epilogue contracts T with conj(phi_d) per voxel.  Lane (voxel i = lane%16,
// slot gq = lane/16) loads the sources s = gq (mod 4) of its voxel once and uses
// their real parts for k-index s and imaginary parts for k-index Sp + s.
template <typename TS, int TBM, int SQ, int NW>
__global__ __launch_bounds__(kBlock) void k_born_adjoint(int N, int S, int D, int Sp, int Dp, int64_t lam_stride,
                                                        int L, const TS* __restrict__ phs,
                                                        const TS* __restrict__ phd,
                                                        const cplx<typename Field<TS>::real>* __restrict__ w,
                                                        int n_w, double scale,
                                                        cplx<typename Field<TS>::real>* __restrict__ g) {
  // NW data vectors w_c per block (blockIdx.y selects the group): the fields of each voxel
  // tile are loaded once per wavelength and serve all of them
  using T = typename Field<TS>::real;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i16 = lane & 15, gq = lane >> 4;
  const int vox0 = (blockIdx.x * 4 + wave) * 16;
  const int c0 = blockIdx.y * NW;
  const int TB = 2 * Dp / 16;
  const int vox = vox0 + i16;
  const bool vok = vox < N;
  using MA = typename Mfma<T>::acc;
  double gre[NW][4], gim[NW][4];
#pragma unroll
  for (int c = 0; c < NW; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) gre[c][r] = gim[c][r] = 0.0;
  // the fields of one wavelength: phi_s[s][vox] for s = gq + 4q, and phi_d at the voxels and
  // detectors of this lane's accumulator entries
  auto load = [&](int l, cplx<T> (&z)[SQ], cplx<T> (&ph)[TBM][4]) {
    const TS* ps = phs + (size_t)l * lam_stride * N;
    const TS* pd = phd + (size_t)l * lam_stride * N;
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int s = gq + 4 * q;
      z[q] = (q < Sp / 4 && s < S && vok) ? Field<TS>::get(ps, (size_t)s * N + vox) : cplx<T>{0, 0};
    }
#pragma unroll
    for (int t = 0; t < TBM; ++t) {
      const int col = t * 16 + i16;
      const int d = col >= Dp ? col - Dp : col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int vv = vox0 + Mfma<T>::out_row(lane, r);
        ph[t][r] = (t < TB && d < D && vv < N) ? Field<TS>::get(pd, (size_t)d * N + vv) : cplx<T>{0, 0};
      }
    }
  };
  cplx<T> zn[SQ], phn[TBM][4];   // the next wavelength's fields, loaded during this one's products
  load(0, zn, phn);
  for (int l = 0; l < L; ++l) {
    cplx<T> z[SQ], ph[TBM][4];
#pragma unroll
    for (int q = 0; q < SQ; ++q) z[q] = zn[q];
#pragma unroll
    for (int t = 0; t < TBM; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) ph[t][r] = phn[t][r];
    if (l + 1 < L) load(l + 1, zn, phn);
#pragma unroll
    for (int c = 0; c < NW; ++c) {
      if (c0 + c >= n_w) break;
      const cplx<T>* wl = w + ((size_t)(c0 + c) * L + l) * S * D;
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
          const bool imcol = t * 16 + i16 >= Dp;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double e = ph[t][r].re, f = ph[t][r].im;
            const double tv = (double)acc[t][r];
            if (!imcol) {          // Re T column
              gre[c][r] += e * tv;
              gim[c][r] -= f * tv;
            } else {               // Im T column
              gre[c][r] += f * tv;
              gim[c][r] += e * tv;
            }
          }
        }
      }
    }
  }
  // reduce over the 16 lanes that share a voxel (lane & 15 varies)
#pragma unroll
  for (int c = 0; c < NW; ++c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        gre[c][r] += __shfl_xor(gre[c][r], off, 64);
        gim[c][r] += __shfl_xor(gim[c][r], off, 64);
      }
    }
    if (i16 == 0 && c0 + c < n_w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int vv = vox0 + Mfma<T>::out_row(lane, r);
        if (vv < N)
          g[(size_t)(c0 + c) * N + vv] = cplx<T>{(T)(scale * gre[c][r]), (T)(scale * gim[c][r])};
      }
    }
  }
}

}  // namespace hydot

#include "born_wide.h"

namespace hydot {

template <typename TS, int CM, int NCT>
void launch_jv_pairs(dim3 grid, hipStream_t stream, int N, int S, int D, int64_t ls, const void* phs, const void* phd,
                     const void* v, int n_v, int kb, int L, int ntd, void* part) {
  using R = typename Field<TS>::real;
  hipLaunchKernelGGL((k_born_jv_pairs<TS, CM, NCT>), grid, dim3(kBlock), 0, stream, N, S, D, ls, (const TS*)phs,
                     (const TS*)phd, (const R*)v, n_v, kb, L, ntd, (double*)part);
}

// Launch plan of one J v call: which kernel, its stage and probe-vector grouping, the split of
// the voxels into ranges and the bytes of FP64 split partials it writes (the caller's scratch).
struct JvPlan {
  bool pairs = false;
  bool wide = false;                            // k_born_jv_wide(_bf) (S and D above 32)
  bool wide_vs = false;                         // its voxel-split form (one probe vector, S, D <= 32)
  int wide_tt = 2;                              // tiles per wave and dimension of that form
  int Sp = 0, Dp = 0;
  int kt = 32, tpw = 1, nvb = 1, ngroups = 1;   // real-ified kernel
  int nts = 1, ntd = 1, nct = 1;                // pair-product kernel
  int nsplit = 1, kb = 0;
  size_t part_bytes = 0;
};

inline bool bf16_compute(int cm) { return cm == CM_BF16 || cm == CM_SPLIT; }

// max_part_bytes > 0 lowers the split count until the partials fit (the allocation-free entry
// point); 0 keeps the split the tuning asks for.
static JvPlan jv_plan(const hydot_operator* op, const hydot_tuning& tune, int S, int D, int n_v, int cm,
                      size_t real_bytes, size_t max_part_bytes = 0) {
  JvPlan P;
  const int N = op->gp.N, L = op->L;
  const hydot_tuning tu = resolved_tuning(tune);
  P.Sp = pad8(S);
  P.Dp = pad8(D);
  if (n_v < kPairsMinNv && (cm == CM_F32 || cm == CM_F64) && S >= kWideMin && D >= kWideMin) {
    // one block per (voxel range, wavelength, probe vector), each holding all S x D pairs:
    // a quarter of the tuned block count fills the chip (about two blocks per CU by default)
    P.wide = true;
    P.kt = cm == CM_F64 ? 16 : 16 * kWideNS;   // FP32: voxel ranges hold whole FP32 partial sums
    const int target = std::max(1, tu.born_blocks / 4);
    P.nsplit = std::max(1, (target + L * n_v - 1) / (L * n_v));
  } else if (n_v < kPairsMinNv && bf16_compute(cm) && S >= kWideMin && D >= kWideMin) {
    // BF16 MFMA form, the same blocks as the FP32 one
    P.wide = true;
    P.kt = kWideBfKt;   // voxel ranges hold whole FP32 partial sums
    const int target = std::max(1, tu.born_blocks / 4);
    P.nsplit = std::max(1, (target + L * n_v - 1) / (L * n_v));
  } else if (n_v == 1 && cm == CM_F32 && S >= kWideVsMin && D >= kWideVsMin && S <= 32 && D <= 32) {
    // one probe vector and 9..32 sources and detectors: the wide kernel with its four waves
    // splitting the voxels (each holds every pair), so each field row is read once per block
    P.wide = true;
    P.wide_vs = true;
    P.wide_tt = std::max(S, D) > 16 ? 2 : 1;
    P.kt = 4 * 16 * kWideNS;   // every wave gets whole FP32 partial sums
    const int target = std::max(1, tu.born_blocks / 4);
    P.nsplit = std::max(1, (target + L * n_v - 1) / (L * n_v));
  } else if (n_v >= kPairsMinNv) {
    P.pairs = true;
    P.kt = 32;
    P.nts = (S + 7) / 8;
    P.ntd = (D + 7) / 8;
    P.nct = (n_v + 15) / 16;   // 1..4 tiles of 16 probe vectors (n_v <= 64)
    const int per_split = L * P.nts * P.ntd;
    P.nsplit = std::max(1, (tu.born_blocks + per_split - 1) / per_split);
  } else {
    const int T_all = (2 * P.Sp / 16) * (2 * P.Dp / 16);
    const int tpw_need = (T_all + 3) / 4;
    P.tpw = tpw_need <= 1 ? 1 : tpw_need <= 2 ? 2 : tpw_need <= 4 ? 4 : tpw_need <= 8 ? 8 : 16;
    // probe vectors per block: up to 8, with tiles-per-wave x vectors <= 8 (accumulator registers)
    while (P.nvb < 8 && P.nvb < n_v && P.tpw * P.nvb * 2 <= 8) P.nvb *= 2;
    // voxels per LDS stage: 32 when the staged rows fit the LDS budget (unless the tuning asks for
    // 16 on an FP32/FP64 product), else 16; BF16 products always take 32
    auto lds = [&](int kt) {
      return (size_t)(2 * P.Sp + 2 * P.Dp) * (kt + 4) * real_bytes + (P.nvb > 1 ? (size_t)P.nvb * kt * real_bytes : 0);
    };
    P.kt = bf16_compute(cm) ? 32 : (lds(32) <= kLdsCap && tu.born_stage != 16 ? 32 : 16);
    P.ngroups = (n_v + P.nvb - 1) / P.nvb;
    // a block's work grows with its output tiles: beyond 16 tiles, fewer blocks (and partials)
    const int tgt = T_all > 16 ? std::max(1, tu.born_blocks * 16 / T_all) : tu.born_blocks;
    P.nsplit = std::max(1, (tgt + L * P.ngroups - 1) / (L * P.ngroups));
  }
  // split over voxels so the grid has about born_blocks blocks; ranges are whole stages
  const int max_split = (N + P.kt - 1) / P.kt;
  const size_t per_split_bytes = P.pairs || P.wide ? (size_t)n_v * L * S * D * 2 * sizeof(double)
                                         : (size_t)n_v * L * (2 * P.Sp) * (2 * P.Dp) * sizeof(double);
  P.nsplit = std::min(P.nsplit, max_split);
  if (max_part_bytes > 0) P.nsplit = (int)std::max<long long>(1, std::min<long long>(P.nsplit, (long long)(max_part_bytes / per_split_bytes)));
  P.kb = (N + P.nsplit - 1) / P.nsplit;
  P.kb = (P.kb + P.kt - 1) / P.kt * P.kt;
  P.nsplit = (N + P.kb - 1) / P.kb;
  P.part_bytes = (size_t)P.nsplit * per_split_bytes;
  return P;
}

// J v for blocks of at least kPairsMinNv probe vectors (every product arithmetic).
template <typename TS, int CM>
hydot_status born_apply_pairs(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd,
                              int D, int64_t ls, const void* v, int n_v, void* y, void* part, hipStream_t stream) {
  using R = typename Field<TS>::real;
  const int N = op->gp.N, L = op->L;
  const dim3 grid(P.nsplit, L, P.nts * P.ntd);
  if (P.nct == 1) launch_jv_pairs<TS, CM, 1>(grid, stream, N, S, D, ls, phs, phd, v, n_v, P.kb, L, P.ntd, part);
  else if (P.nct == 2) launch_jv_pairs<TS, CM, 2>(grid, stream, N, S, D, ls, phs, phd, v, n_v, P.kb, L, P.ntd, part);
  else if (P.nct == 3) launch_jv_pairs<TS, CM, 3>(grid, stream, N, S, D, ls, phs, phd, v, n_v, P.kb, L, P.ntd, part);
  else launch_jv_pairs<TS, CM, 4>(grid, stream, N, S, D, ls, phs, phd, v, n_v, P.kb, L, P.ntd, part);
  const int nout = n_v * L * S * D;
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_pairs_finish<cplx<R>>), dim3((nout + 255) / 256), dim3(256), 0, stream, S * D,
                     P.nsplit, nout, (const double*)part, -h * h * h, (cplx<R>*)y);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// J v on k_born_jv_wide (complex FP32 fields, S and D above 32, fewer than kPairsMinNv probe
// vectors), then the fixed-order sum over the voxel ranges.
hydot_status born_apply_wide(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd,
                             int D, int64_t ls, const void* v, int n_v, void* y, void* part, hipStream_t stream) {
  const int N = op->gp.N, L = op->L;
  const dim3 grid(P.nsplit, L, n_v);
  // (the voxel-split form's 16-byte path reads through buffer resources over one wavelength's rows)
  const bool vec = N % 4 == 0 && aligned16(phs) && aligned16(phd) && aligned16(v) &&
                   (!P.wide_vs || (size_t)std::max(S, D) * (size_t)N * 8u < (size_t(1) << 31));
#define HYDOT_JVW(VEC, TT, VS)                                                                                   \
  hipLaunchKernelGGL((k_born_jv_wide<VEC, TT, VS>), grid, dim3(kBlock), 0, stream, N, S, D, ls, (const cf*)phs, \
                     (const cf*)phd, (const float*)v, P.kb, L, (double*)part)
  if (P.wide_vs && P.wide_tt == 1) {
    if (vec) HYDOT_JVW(true, 1, true); else HYDOT_JVW(false, 1, true);
  } else if (P.wide_vs) {
    if (vec) HYDOT_JVW(true, 2, true); else HYDOT_JVW(false, 2, true);
  } else {
    if (vec) HYDOT_JVW(true, 2, false); else HYDOT_JVW(false, 2, false);
  }
#undef HYDOT_JVW
  const int nout = n_v * L * S * D;
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_pairs_finish<cf>), dim3((nout + 255) / 256), dim3(256), 0, stream, S * D, P.nsplit,
                     nout, (const double*)part, -h * h * h, (cf*)y);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

// J v on k_born_jv_wide64 (complex FP64 fields, S and D above 32, fewer than kPairsMinNv probe
// vectors), then the fixed-order sum over the voxel ranges.
hydot_status born_apply_wide64(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd,
                               int D, int64_t ls, const void* v, int n_v, void* y, void* part, hipStream_t stream) {
  const int N = op->gp.N, L = op->L;
  // buffer resources: one wavelength's rows (and v) below 2 GiB
  const bool buf = (size_t)std::max(S, D) * (size_t)N * 16u < (size_t(1) << 31);
  if (buf)
    hipLaunchKernelGGL(k_born_jv_wide64<true>, dim3(P.nsplit, L, n_v), dim3(kBlock), 0, stream, N, S, D, ls,
                       (const cd*)phs, (const cd*)phd, (const double*)v, P.kb, L, (double*)part);
  else
    hipLaunchKernelGGL(k_born_jv_wide64<false>, dim3(P.nsplit, L, n_v), dim3(kBlock), 0, stream, N, S, D, ls,
                       (const cd*)phs, (const cd*)phd, (const double*)v, P.kb, L, (double*)part);
  const int nout = n_v * L * S * D;
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_pairs_finish<cd>), dim3((nout + 255) / 256), dim3(256), 0, stream, S * D, P.nsplit,
                     nout, (const double*)part, -h * h * h, (cd*)y);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

// J v on k_born_jv_wide_bf (BF16-stored fields with BF16 products, or FP32 fields with split-BF16
// products; S and D above 32), then the fixed-order sum over the voxel ranges.
template <typename TS, int CM>
hydot_status born_apply_wide_bf(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd,
                                int D, int64_t ls, const void* v, int n_v, void* y, void* part, hipStream_t stream) {
  using R = typename Field<TS>::real;
  const int N = op->gp.N, L = op->L;
  const dim3 grid(P.nsplit, L, n_v);
  // 16-byte buffer loads: N a multiple of 8, 16-byte aligned bases, every resource below 2 GiB
  const bool vec = N % 8 == 0 && aligned16(phs) && aligned16(phd) && aligned16(v) &&
                   (size_t)std::max(S, D) * N * sizeof(TS) < ((size_t)1 << 31);
  if (vec)
    hipLaunchKernelGGL((k_born_jv_wide_bf<TS, CM, true>), grid, dim3(kBlock), 0, stream, N, S, D, ls, (const TS*)phs,
                       (const TS*)phd, (const float*)v, P.kb, L, (double*)part);
  else
    hipLaunchKernelGGL((k_born_jv_wide_bf<TS, CM, false>), grid, dim3(kBlock), 0, stream, N, S, D, ls,
                       (const TS*)phs, (const TS*)phd, (const float*)v, P.kb, L, (double*)part);
  const int nout = n_v * L * S * D;
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_pairs_finish<cplx<R>>), dim3((nout + 255) / 256), dim3(256), 0, stream, S * D, P.nsplit,
                     nout, (const double*)part, -h * h * h, (cplx<R>*)y);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

template <typename TS, int CM>
hydot_status born_apply_impl(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd,
                             int D, int64_t ls, const void* v, int n_v, void* y, void* part, hipStream_t stream) {
  if constexpr (std::is_same<TS, cf>::value && CM == CM_F32) {
    if (P.wide) return born_apply_wide(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  }
  if constexpr ((std::is_same<TS, cbf>::value && CM == CM_BF16) || (std::is_same<TS, cf>::value && CM == CM_SPLIT)) {
    if (P.wide) return born_apply_wide_bf<TS, CM>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  }
  if constexpr (std::is_same<TS, cd>::value && CM == CM_F64) {
    if (P.wide) return born_apply_wide64(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  }
  if (P.pairs) return born_apply_pairs<TS, CM>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  using R = typename Field<TS>::real;
  const int N = op->gp.N, L = op->L;
  const int Sp = P.Sp, Dp = P.Dp, tpw = P.tpw, nvb = P.nvb, kt = P.kt, kb = P.kb;
  const size_t lds = (size_t)(2 * Sp + 2 * Dp) * (kt + 4) * sizeof(R) + (nvb > 1 ? (size_t)nvb * kt * sizeof(R) : 0);
  dim3 grid(P.nsplit, L, P.ngroups);
  // staged elements per thread: 2 covers up to 16 rows at 32 voxels per stage, 8 covers 64
  const bool em2 = std::max(Sp, Dp) * kt <= 2 * kBlock;
#define HYDOT_BA_E(TP, NB, KT, EM)                                                                               \
  hipLaunchKernelGGL((k_born_jv<TS, CM, TP, NB, KT, EM>), grid, dim3(kBlock), lds, stream, N, S, D, Sp, Dp, ls, \
                     (const TS*)phs, (const TS*)phd, (const R*)v, n_v, kb, L, (double*)part)
#define HYDOT_BA(TP, NB, KT) \
  if (em2) { HYDOT_BA_E(TP, NB, KT, 2); } else { HYDOT_BA_E(TP, NB, KT, (64 * KT / kBlock)); }
#define HYDOT_BA_K(TP, NB) \
  if (kt == 32) { HYDOT_BA(TP, NB, 32); } else if constexpr (!(CM == CM_BF16 || CM == CM_SPLIT)) { HYDOT_BA(TP, NB, 16); }
  if (tpw == 1) {
    if (nvb == 8) { HYDOT_BA_K(1, 8) } else if (nvb == 4) { HYDOT_BA_K(1, 4) }
    else if (nvb == 2) { HYDOT_BA_K(1, 2) } else { HYDOT_BA_K(1, 1) }
  } else if (tpw == 2) {
    if (nvb == 4) { HYDOT_BA_K(2, 4) } else if (nvb == 2) { HYDOT_BA_K(2, 2) } else { HYDOT_BA_K(2, 1) }
  } else if (tpw == 4) {
    if (nvb == 2) { HYDOT_BA_K(4, 2) } else { HYDOT_BA_K(4, 1) }
  } else if (tpw == 8) {
    HYDOT_BA_K(8, 1)
  } else {
    HYDOT_BA_K(16, 1)
  }
#undef HYDOT_BA_K
#undef HYDOT_BA
#undef HYDOT_BA_E
  const double h = op->grid.h_mm;
  hipLaunchKernelGGL((k_born_apply_finish<cplx<R>>), dim3((S * D + 255) / 256, n_v * L), dim3(256), 0, stream, S, D,
                     Sp, Dp, P.nsplit, L, (const double*)part, -h * h * h, (cplx<R>*)y);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

template <typename TS>
hydot_status born_adjoint_impl(const hydot_operator* op, const void* phs, int S, const void* phd, int D,
                               int64_t ls, const void* w, int n_w, void* g, hipStream_t stream) {
  using R = typename Field<TS>::real;
  const int N = op->gp.N, L = op->L;
  const double h = op->grid.h_mm;
  if constexpr (std::is_same<TS, cf>::value) {
    // many pairs: k_born_adjoint_wide, one data vector per launch; one data vector with 9..32
    // sources and detectors: its instances with fewer source steps and detector tiles (which
    // carry w in registers, four elements per thread: S D <= 1024)
    const bool wide = S >= kWideMin && D >= kWideMin;
    const bool mid = n_w == 1 && S >= kWideVsMin && D >= kWideVsMin && S <= 32 && D <= 32;
    if (wide || mid) {
      const bool vec = N % 4 == 0 && aligned16(phs) && aligned16(phd);
      const dim3 grid((N + 63) / 64);
      const int qn = wide ? 16 : S <= 16 ? 4 : 8, td = wide ? 4 : D <= 16 ? 1 : 2;
      for (int c = 0; c < n_w; ++c) {
        const cf* wc = (const cf*)w + (size_t)c * L * S * D;
        cf* gc = (cf*)g + (size_t)c * N;
#define HYDOT_ADJW(VEC, QN, TD, BUF)                                                                           \
  hipLaunchKernelGGL((k_born_adjoint_wide<VEC, QN, TD, BUF>), grid, dim3(kBlock), 0, stream, N, S, D, ls, L, \
                     (const cf*)phs, (const cf*)phd, wc, -h * h * h, gc)
#define HYDOT_ADJW_V(QN, TD) \
  if (vec) HYDOT_ADJW(true, QN, TD, false); else HYDOT_ADJW(false, QN, TD, false);
        // buffer resources over one wavelength's rows: below 2 GiB
        const bool buf = vec && (size_t)std::max(S, D) * (size_t)N * 8u < (size_t(1) << 31);
        if (qn == 16 && buf) { HYDOT_ADJW(true, 16, 4, true); }
        else if (qn == 16) { HYDOT_ADJW_V(16, 4) }
        else if (qn == 4 && td == 1) { HYDOT_ADJW_V(4, 1) }
        else if (qn == 4) { HYDOT_ADJW_V(4, 2) }
        else if (td == 1) { HYDOT_ADJW_V(8, 1) }
        else { HYDOT_ADJW_V(8, 2) }
#undef HYDOT_ADJW_V
#undef HYDOT_ADJW
      }
      HYDOT_HIP(hipGetLastError());
      return HYDOT_OK;
    }
  }
  if constexpr (std::is_same<TS, cd>::value) {
    // many pairs from FP64 fields: k_born_adjoint_wide64 (FP64 MFMA), one data vector per launch
    if (S >= kWideMin && D >= kWideMin) {
      const dim3 grid((N + 63) / 64);
      for (int c = 0; c < n_w; ++c)
        hipLaunchKernelGGL(k_born_adjoint_wide64, grid, dim3(kBlock), 0, stream, N, S, D, ls, L, (const cd*)phs,
                           (const cd*)phd, (const cd*)w + (size_t)c * L * S * D, -h * h * h, (cd*)g + (size_t)c * N);
      HYDOT_HIP(hipGetLastError());
      return HYDOT_OK;
    }
  }
  if constexpr (std::is_same<TS, cbf>::value) {
    // many pairs from BF16 fields: k_born_adjoint_wide_bf (BF16 MFMA, w split into BF16 hi + lo),
    // one data vector per launch; its buffer resources span one wavelength's rows
    if (S >= kWideMin && D >= kWideMin && (size_t)std::max(S, D) * (size_t)N * 4u < (size_t(1) << 31)) {
      const bool vec = N % 4 == 0 && aligned16(phs) && aligned16(phd);
      const dim3 grid((N + kAdjBfVox - 1) / kAdjBfVox);
      for (int c = 0; c < n_w; ++c) {
        const cf* wc = (const cf*)w + (size_t)c * L * S * D;
        cf* gc = (cf*)g + (size_t)c * N;
        if (vec)
          hipLaunchKernelGGL(k_born_adjoint_wide_bf<true>, grid, dim3(kBlock), 0, stream, N, S, D, ls, L,
                             (const cbf*)phs, (const cbf*)phd, wc, -h * h * h, gc);
        else
          hipLaunchKernelGGL(k_born_adjoint_wide_bf<false>, grid, dim3(kBlock), 0, stream, N, S, D, ls, L,
                             (const cbf*)phs, (const cbf*)phd, wc, -h * h * h, gc);
      }
      HYDOT_HIP(hipGetLastError());
      return HYDOT_OK;
    }
  }
  const int Sp = pad8(S), Dp = pad8(D);
  const int TB = 2 * Dp / 16;
  // four data vectors per block when the detector tiles are few (register budget)
  const int nw = n_w > 1 && TB <= 2 ? 4 : 1;
  dim3 grid((N + 63) / 64, (n_w + nw - 1) / nw);
  const double sc = -h * h * h;
#define HYDOT_BJ(TBM, SQ, NW)                                                                                  \
  hipLaunchKernelGGL((k_born_adjoint<TS, TBM, SQ, NW>), grid, dim3(kBlock), 0, stream, N, S, D, Sp, Dp, ls, L, \
                     (const TS*)phs, (const TS*)phd, (const cplx<R>*)w, n_w, sc, (cplx<R>*)g)
#define HYDOT_BJ_S(TBM, NW) \
  if (Sp <= 16) HYDOT_BJ(TBM, 4, NW); else if (Sp <= 32) HYDOT_BJ(TBM, 8, NW); else HYDOT_BJ(TBM, 16, NW);
  if (TB <= 1) { if (nw == 4) { HYDOT_BJ_S(1, 4) } else { HYDOT_BJ_S(1, 1) } }
  else if (TB <= 2) { if (nw == 4) { HYDOT_BJ_S(2, 4) } else { HYDOT_BJ_S(2, 1) } }
  else if (TB <= 4) { HYDOT_BJ_S(4, 1) }
  else { HYDOT_BJ_S(8, 1) }
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
  if (dt != HYDOT_C128 && dt != HYDOT_C64 && dt != HYDOT_CBF16)
    return fail(HYDOT_EUNSUPPORTED, "born: field_dtype must be C128, C64 or CBF16");
  return HYDOT_OK;
}

// Validation of a J v call shared by the entry points (no launch).
static hydot_status jv_check(const hydot_operator* op, const void* phs, int S, const void* phd, int D, int64_t ls,
                             hydot_dtype dt, hydot_born_compute compute, int n_v) {
  hydot_status s = born_check(op, phs, S, phd, D, ls, dt);
  if (s != HYDOT_OK) return s;
  if (n_v < 1 || n_v > 64) return fail(HYDOT_EINVAL, "born_apply: n_v must be in [1, 64]");
  if (compute != HYDOT_BORN_NATIVE && compute != HYDOT_BORN_SPLIT_BF16)
    return fail(HYDOT_EINVAL, "born_apply: unknown compute mode");
  if (compute == HYDOT_BORN_SPLIT_BF16 && dt != HYDOT_C64)
    return fail(HYDOT_EUNSUPPORTED, "born_apply: split-BF16 products take C64 fields");
  return HYDOT_OK;
}

static int jv_cm(hydot_dtype dt, hydot_born_compute compute) {
  if (dt == HYDOT_C128) return CM_F64;
  if (dt == HYDOT_CBF16) return CM_BF16;
  return compute == HYDOT_BORN_SPLIT_BF16 ? CM_SPLIT : CM_F32;
}

static size_t jv_real_bytes(hydot_dtype dt) { return dt == HYDOT_C128 ? sizeof(double) : sizeof(float); }

// Launch J v with the scratch `part` (>= P.part_bytes, 256-byte aligned).
static hydot_status jv_launch(const hydot_operator* op, const JvPlan& P, const void* phs, int S, const void* phd, int D,
                              int64_t ls, hydot_dtype dt, int cm, const void* v, int n_v, void* y, void* part,
                              hipStream_t stream) {
  if (cm == CM_F64) return born_apply_impl<cd, CM_F64>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  if (cm == CM_BF16) return born_apply_impl<cbf, CM_BF16>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  if (cm == CM_SPLIT) return born_apply_impl<cf, CM_SPLIT>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
  (void)dt;
  return born_apply_impl<cf, CM_F32>(op, P, phs, S, phd, D, ls, v, n_v, y, part, stream);
}

// ---------------------------------------------------------------- allocation-free J v
// The FP64 split partials of hydot_born_apply_noalloc live in this file-scope device array: one
// copy per GPU, held until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in symbol): the device address of each GPU's
// copy is looked up once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = HYDOT_BORN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up on the first call on that device)
static hydot_status noalloc_scratch(void** out) {
  int dev = -1;
  HYDOT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDOT_EUNSUPPORTED, "born_apply_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HYDOT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255u)) return fail(HYDOT_EDEVICE, "born_apply_noalloc: scratch address lookup failed");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HYDOT_OK;
}

}  // namespace hydot

using namespace hydot;

extern "C" {

hydot_status hydot_born_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D, hydot_dtype field_dtype,
                                        hydot_born_compute compute, int32_t n_v, size_t* bytes) {
  if (!bytes) return fail(HYDOT_EINVAL, "born_workspace_bytes: null bytes");
  if (!op) return fail(HYDOT_EINVAL, "born_workspace_bytes: null operator");
  if (S < 1 || S > 64 || D < 1 || D > 64) return fail(HYDOT_EINVAL, "born_workspace_bytes: S and D must be in [1, 64]");
  if (n_v < 1 || n_v > 64) return fail(HYDOT_EINVAL, "born_workspace_bytes: n_v must be in [1, 64]");
  if (field_dtype != HYDOT_C128 && field_dtype != HYDOT_C64 && field_dtype != HYDOT_CBF16)
    return fail(HYDOT_EUNSUPPORTED, "born_workspace_bytes: field_dtype must be C128, C64 or CBF16");
  if (compute != HYDOT_BORN_NATIVE && compute != HYDOT_BORN_SPLIT_BF16)
    return fail(HYDOT_EINVAL, "born_workspace_bytes: unknown compute mode");
  *bytes = jv_plan(op, op->tune, S, D, n_v, jv_cm(field_dtype, compute), jv_real_bytes(field_dtype)).part_bytes;
  return HYDOT_OK;
}

hydot_status hydot_born_apply_ex(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                                 int32_t D, int64_t lam_stride, hydot_dtype field_dtype, hydot_born_compute compute,
                                 const void* v, int32_t n_v, void* y, void* workspace, size_t ws_bytes,
                                 hipStream_t stream) {
  hydot_status s = jv_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype, compute, n_v);
  if (s != HYDOT_OK) return s;
  if (!v || !y) return fail(HYDOT_EINVAL, "born_apply: null v or y");
  if (!workspace || ((uintptr_t)workspace & 255u)) return fail(HYDOT_EINVAL, "born_apply: workspace must be a 256-byte aligned device pointer");
  const int cm = jv_cm(field_dtype, compute);
  const JvPlan P = jv_plan(op, op->tune, S, D, n_v, cm, jv_real_bytes(field_dtype));
  if (ws_bytes < P.part_bytes) return fail(HYDOT_ENOMEM, "born_apply: workspace smaller than hydot_born_workspace_bytes");
  return jv_launch(op, P, phi_src, S, phi_det, D, lam_stride, field_dtype, cm, v, n_v, y, workspace, stream);
}

hydot_status hydot_born_apply_noalloc(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                                      int32_t D, int64_t lam_stride, hydot_dtype field_dtype,
                                      hydot_born_compute compute, const void* v, int32_t n_v, void* y,
                                      hipStream_t stream) {
  hydot_status s = jv_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype, compute, n_v);
  if (s != HYDOT_OK) return s;
  if (!v || !y) return fail(HYDOT_EINVAL, "born_apply_noalloc: null v or y");
  const int cm = jv_cm(field_dtype, compute);
  // the tuned split, lowered until the partials fit the static scratch
  const JvPlan P = jv_plan(op, op->tune, S, D, n_v, cm, jv_real_bytes(field_dtype), kNoAllocScratchBytes);
  if (P.part_bytes > kNoAllocScratchBytes)
    return fail(HYDOT_ENOMEM, "born_apply_noalloc: the partial sums of one voxel range (" +
                                  std::to_string(P.part_bytes) + " bytes for n_v * n_lambda * S * D) exceed the " +
                                  std::to_string(kNoAllocScratchBytes) + "-byte static scratch");
  void* part = nullptr;
  s = noalloc_scratch(&part);
  if (s != HYDOT_OK) return s;
  return jv_launch(op, P, phi_src, S, phi_det, D, lam_stride, field_dtype, cm, v, n_v, y, part, stream);
}

hydot_status hydot_born_apply(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                              int32_t D, int64_t lam_stride, hydot_dtype field_dtype, const void* v, int32_t n_v,
                              void* y, void* workspace, size_t ws_bytes, hipStream_t stream) {
  return hydot_born_apply_ex(op, phi_src, S, phi_det, D, lam_stride, field_dtype, HYDOT_BORN_NATIVE, v, n_v, y,
                             workspace, ws_bytes, stream);
}

hydot_status hydot_born_apply_adjoint_ex(const hydot_operator* op, const void* phi_src, int32_t S,
                                         const void* phi_det, int32_t D, int64_t lam_stride, hydot_dtype field_dtype,
                                         const void* w, int32_t n_w, void* g, hipStream_t stream) {
  hydot_status s = born_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype);
  if (s != HYDOT_OK) return s;
  if (!w || !g) return fail(HYDOT_EINVAL, "born_apply_adjoint: null w or g");
  if (n_w < 1 || n_w > 1024) return fail(HYDOT_EINVAL, "born_apply_adjoint: n_w must be in [1, 1024]");
  if (field_dtype == HYDOT_C128)
    return born_adjoint_impl<cd>(op, phi_src, S, phi_det, D, lam_stride, w, n_w, g, stream);
  if (field_dtype == HYDOT_CBF16)
    return born_adjoint_impl<cbf>(op, phi_src, S, phi_det, D, lam_stride, w, n_w, g, stream);
  return born_adjoint_impl<cf>(op, phi_src, S, phi_det, D, lam_stride, w, n_w, g, stream);
}

hydot_status hydot_born_apply_adjoint(const hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det,
                                      int32_t D, int64_t lam_stride, hydot_dtype field_dtype, const void* w, void* g,
                                      hipStream_t stream) {
  return hydot_born_apply_adjoint_ex(op, phi_src, S, phi_det, D, lam_stride, field_dtype, w, 1, g, stream);
}

static const int kTuneStages[2] = {32, 16};
static const int kTuneBlocks[5] = {4096, 2048, 8192, 1024, 16384};

hydot_status hydot_autotune_born_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D,
                                                 hydot_dtype field_dtype, int32_t n_v, size_t* bytes) {
  if (!bytes || !op) return fail(HYDOT_EINVAL, "autotune_born_workspace_bytes: null argument");
  size_t need = 0;
  hydot_status s = hydot_born_workspace_bytes(op, S, D, field_dtype, HYDOT_BORN_NATIVE, n_v, &need);   // validates
  if (s != HYDOT_OK) return s;
  for (int is = 0; is < 2; ++is)
    for (int ib = 0; ib < 5; ++ib) {
      hydot_tuning t = resolved_tuning(op->tune);
      t.born_stage = kTuneStages[is];
      t.born_blocks = kTuneBlocks[ib];
      need = std::max(need, jv_plan(op, t, S, D, n_v, jv_cm(field_dtype, HYDOT_BORN_NATIVE),
                                    jv_real_bytes(field_dtype)).part_bytes);
    }
  *bytes = need;
  return HYDOT_OK;
}

hydot_status hydot_autotune_born(hydot_operator* op, const void* phi_src, int32_t S, const void* phi_det, int32_t D,
                                 int64_t lam_stride, hydot_dtype field_dtype, const void* v, int32_t n_v, void* y,
                                 void* workspace, size_t ws_bytes, hydot_tune_trial* trials, int32_t max_trials,
                                 int32_t* n_trials, hipStream_t stream) {
  if (!op) return fail(HYDOT_EINVAL, "autotune_born: null operator");
  if (max_trials < 0 || (max_trials > 0 && !trials)) return fail(HYDOT_EINVAL, "autotune_born: bad trials buffer");
  {
    hydot_status s = jv_check(op, phi_src, S, phi_det, D, lam_stride, field_dtype, HYDOT_BORN_NATIVE, n_v);
    if (s != HYDOT_OK) return s;
    size_t need = 0;
    s = hydot_autotune_born_workspace_bytes(op, S, D, field_dtype, n_v, &need);
    if (s != HYDOT_OK) return s;
    if (!workspace || ((uintptr_t)workspace & 255u)) return fail(HYDOT_EINVAL, "autotune_born: workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(HYDOT_ENOMEM, "autotune_born: workspace smaller than hydot_autotune_born_workspace_bytes");
  }
  const hydot_tuning keep = op->tune;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HYDOT_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HYDOT_EDEVICE, "autotune_born: event create");
  }
  // default first; later candidates must be more than 2% faster to replace the best
  int count = 0;
  double best = 1e300;
  hydot_tuning best_t = resolved_tuning(keep);
  hydot_status err = HYDOT_OK;
  for (int is = 0; is < 2 && err == HYDOT_OK; ++is)
    for (int ib = 0; ib < 5 && err == HYDOT_OK; ++ib) {
      hydot_tuning t = resolved_tuning(keep);
      t.born_stage = kTuneStages[is];
      t.born_blocks = kTuneBlocks[ib];
      op->tune = t;
      float ms[5];
      for (int rep = 0; rep < 6 && err == HYDOT_OK; ++rep) {   // first call warms up
        if (hipEventRecord(e0, stream) != hipSuccess) err = fail(HYDOT_EDEVICE, "autotune_born: event record");
        if (err == HYDOT_OK)
          err = hydot_born_apply(op, phi_src, S, phi_det, D, lam_stride, field_dtype, v, n_v, y, workspace, ws_bytes,
                                 stream);
        if (err == HYDOT_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
          err = fail(HYDOT_EDEVICE, "autotune_born: event wait");
        if (err == HYDOT_OK && rep > 0 && hipEventElapsedTime(&ms[rep - 1], e0, e1) != hipSuccess)
          err = fail(HYDOT_EDEVICE, "autotune_born: elapsed time");
      }
      if (err != HYDOT_OK) break;
      std::sort(ms, ms + 5);
      if (count < max_trials) trials[count] = hydot_tune_trial{t, (double)ms[2]};
      ++count;
      if (ms[2] < 0.98 * best) {
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
