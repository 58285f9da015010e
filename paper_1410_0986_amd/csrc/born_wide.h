// Born products for many source-detector pairs (more than 32 sources and more than 32
// detectors) from complex FP32 fields on the FP32 MFMA.  At these shapes one probe vector
// already gives S/2 >= 16 flop per field byte, so the products are bound by the MFMA and HBM
// together; these kernels feed the MFMA straight from registers loaded from HBM (no LDS
// staging of the fields, no operand reloads per output tile).
//
// Operand layout shared by both kernels.  v_mfma_f32_16x16x4f32 takes A[row = lane%16][k =
// lane/16] and B[k = lane/16][col = lane%16].  The contraction index of J v is the voxel, and a
// sum over voxels may take them in any order as long as both operands agree; lane (r = lane%16,
// g = lane/16) therefore loads voxels 4g..4g+3 of a 16-voxel step of its field row (32
// contiguous bytes, the four groups of a row covering one 128-byte line), and the i-th of the
// four MFMA k-steps of the step takes voxel 4g + i in every group.
#pragma once

namespace hydot {

constexpr int kWideMin = 33;     // S and D above 32: the real-ified / pair kernels pad less below
constexpr int kWideNS = 8;       // 16-voxel steps per FP32 partial sum (128 voxels) before FP64
constexpr int kWideVsMin = 9;    // one probe vector, 9..32 sources and detectors: the voxel-split form

// Raw buffer resource over nbytes at p (an offset at or past nbytes reads zero)
__device__ inline __amdgpu_buffer_rsrc_t wide_rsrc(const void* p, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
constexpr uint32_t kWideOut = 0x80000000u;   // a byte offset past every resource here

// 16-byte loads of two complex FP32 values / four floats (the caller checks the alignment)
__device__ inline void ld2cf(const cf* p, cf& a, cf& b) {
  const f32x4 x = *reinterpret_cast<const f32x4*>(p);
  a = cf{x[0], x[1]};
  b = cf{x[2], x[3]};
}

// ---------------------------------------------------------------- J v
// y[c][l][s][d] = -h^3 sum_k phi_s(k) v_c(k) phi_d(k) for one probe vector per block.
// Block = 4 waves on (split over voxels, wavelength, probe vector).  Wave (wa, wb) = (w/2, w%2)
// owns the pairs s in [32 wa, 32 wa + 32), d in [32 wb, 32 wb + 32) as 2 x 2 tiles of 16 x 16:
// the A operand is a = phi_s v, the B operand phi_d, and Re y accumulates Re a Re b + (-Im a) Im b,
// Im y accumulates Re a Im b + Im a Re b, in FP32 over kWideNS steps and then in FP64.  Each
// block writes its FP64 partial sums as part[((c L + l) nsplit + split) S D + s D + d] (Re, Im),
// summed over the splits by k_born_pairs_finish.  VEC: 16-byte loads (N a multiple of 4 and
// every base pointer 16-byte aligned).
template <bool VEC, int TT = 2, bool VS = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_jv_wide(int N, int S, int D, int64_t lam_stride,
                                                        const cf* __restrict__ phs, const cf* __restrict__ phd,
                                                        const float* __restrict__ v, int kb, int L,
                                                        double* __restrict__ part) {
  const int split = blockIdx.x, l = blockIdx.y, c = blockIdx.z, nsplit = gridDim.x;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  static_assert(VS || TT == 2, "the row-split form holds 2 x 2 tiles per wave");
  // row split (VS false): wave (wa, wb) takes sources [32 wa, 32 wa + 32) and detectors
  // [32 wb, 32 wb + 32); voxel split (VS true, S and D up to 16 TT): every wave takes all the
  // pairs and every fourth 16-voxel step of the block's range
  const int wa = VS ? 0 : wave >> 1, wb = VS ? 0 : wave & 1;
  const size_t Nz = (size_t)N;
  // this lane's TT A rows (sources) and TT B rows (detectors); rows past S or D read zero
  int srow[TT], drow[TT];
  bool sok[TT], dok[TT];
  const cf* pa[TT];
  const cf* pb[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    srow[t] = 32 * wa + 16 * t + r16;
    drow[t] = 32 * wb + 16 * t + r16;
    sok[t] = srow[t] < S;
    dok[t] = drow[t] < D;
    pa[t] = phs + ((size_t)l * lam_stride + (sok[t] ? srow[t] : 0)) * Nz;
    pb[t] = phd + ((size_t)l * lam_stride + (dok[t] ? drow[t] : 0)) * Nz;
  }
  const float* vc = v + (size_t)c * Nz;
  struct Stage {
    cf a[TT][4], b[TT][4];
    float vv[4];
  };
  auto fetch = [&](int kbase, Stage& st) {
    const int kq = kbase + 4 * g;
    if (VEC && kq + 4 <= k1) {
      const f32x4 x = *reinterpret_cast<const f32x4*>(vc + kq);
#pragma unroll
      for (int i = 0; i < 4; ++i) st.vv[i] = x[i];
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        if (sok[t]) {
          ld2cf(pa[t] + kq, st.a[t][0], st.a[t][1]);
          ld2cf(pa[t] + kq + 2, st.a[t][2], st.a[t][3]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) st.a[t][i] = cf{0.f, 0.f};
        }
        if (dok[t]) {
          ld2cf(pb[t] + kq, st.b[t][0], st.b[t][1]);
          ld2cf(pb[t] + kq + 2, st.b[t][2], st.b[t][3]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) st.b[t][i] = cf{0.f, 0.f};
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = kq + i;
        const bool ok = k < k1;
        st.vv[i] = ok ? vc[k] : 0.f;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          st.a[t][i] = ok && sok[t] ? pa[t][k] : cf{0.f, 0.f};
          st.b[t][i] = ok && dok[t] ? pb[t][k] : cf{0.f, 0.f};
        }
      }
    }
  };
  // voxel split with 16-byte loads: every operand through a buffer resource over this
  // wavelength's rows (a missing row or a piece past the range reads zero), so the loads are
  // unconditional and their waits can sit steps back (loads under a branch are waited for at
  // its end)
  const __amdgpu_buffer_rsrc_t ra = wide_rsrc(phs + (size_t)l * lam_stride * Nz, VS && VEC ? (uint32_t)S * (uint32_t)N * 8u : 0u);
  const __amdgpu_buffer_rsrc_t rb = wide_rsrc(phd + (size_t)l * lam_stride * Nz, VS && VEC ? (uint32_t)D * (uint32_t)N * 8u : 0u);
  const __amdgpu_buffer_rsrc_t rvv = wide_rsrc(vc, VS && VEC ? (uint32_t)N * 4u : 0u);
  auto fetch_buf = [&](int kbase, Stage& st) {
    const int kq = kbase + 4 * g;
    const bool in = kq < k1;   // N and the range ends are multiples of 4
    const f32x4 x =
        __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rvv, in ? (uint32_t)kq * 4u : kWideOut, 0, 0));
#pragma unroll
    for (int i = 0; i < 4; ++i) st.vv[i] = x[i];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const uint32_t oa = in && sok[t] ? ((uint32_t)srow[t] * (uint32_t)N + (uint32_t)kq) * 8u : kWideOut;
      const uint32_t ob = in && dok[t] ? ((uint32_t)drow[t] * (uint32_t)N + (uint32_t)kq) * 8u : kWideOut;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 xa = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ra, oa + 16u * h, 0, 0));
        const f32x4 xb = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb, ob + 16u * h, 0, 0));
        st.a[t][2 * h] = cf{xa[0], xa[1]};
        st.a[t][2 * h + 1] = cf{xa[2], xa[3]};
        st.b[t][2 * h] = cf{xb[0], xb[1]};
        st.b[t][2 * h + 1] = cf{xb[2], xb[3]};
      }
    }
  };
  f32x4 accR[TT][TT], accI[TT][TT];
  double totR[TT][TT][4], totI[TT][TT][4];
#pragma unroll
  for (int ta = 0; ta < TT; ++ta)
#pragma unroll
    for (int tb = 0; tb < TT; ++tb) {
      accR[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
      accI[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) totR[ta][tb][r] = totI[ta][tb][r] = 0.0;
    }
  // this wave's steps: all of the block's (row split) or every fourth (voxel split)
  const int nst_all = k1 > k0 ? (k1 - k0 + 15) / 16 : 0;
  const int s0 = VS ? wave : 0, sstr = VS ? 4 : 1;
  const int nst = VS ? (nst_all > wave ? (nst_all - wave + 3) / 4 : 0) : nst_all;
  auto kstep = [&](int st) { return k0 + 16 * (s0 + sstr * st); };
  auto compute = [&](const Stage& cur, int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float ar[TT], ai[TT], nai[TT];
#pragma unroll
      for (int ta = 0; ta < TT; ++ta) {
        ar[ta] = cur.a[ta][i].re * cur.vv[i];
        ai[ta] = cur.a[ta][i].im * cur.vv[i];
        nai[ta] = -ai[ta];
      }
      // eight independent accumulators between two products into the same one
#pragma unroll
      for (int tb = 0; tb < TT; ++tb)
#pragma unroll
        for (int ta = 0; ta < TT; ++ta) {
          accR[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ta], cur.b[tb][i].re, accR[ta][tb], 0, 0, 0);
          accI[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ta], cur.b[tb][i].im, accI[ta][tb], 0, 0, 0);
        }
#pragma unroll
      for (int tb = 0; tb < TT; ++tb)
#pragma unroll
        for (int ta = 0; ta < TT; ++ta) {
          accR[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[ta], cur.b[tb][i].im, accR[ta][tb], 0, 0, 0);
          accI[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[ta], cur.b[tb][i].re, accI[ta][tb], 0, 0, 0);
        }
    }
    if ((st + 1) % kWideNS == 0 || st + 1 == nst) {
#pragma unroll
      for (int ta = 0; ta < TT; ++ta)
#pragma unroll
        for (int tb = 0; tb < TT; ++tb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            totR[ta][tb][r] += (double)accR[ta][tb][r];
            totI[ta][tb][r] += (double)accI[ta][tb][r];
          }
          accR[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
          accI[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  if constexpr (VS && VEC) {
    // three stage buffers taken in rotation (unrolled by three, so no stage is copied: a copy
    // would wait for its loads), the operands two steps ahead of the products
    // steps past the range read zeros and add nothing (at most two per wave), so nothing in the
    // loop is conditional
    Stage q0, q1, q2;
    fetch_buf(kstep(0), q0);
    fetch_buf(kstep(1), q1);
    for (int st = 0; st < nst; st += 3) {
      fetch_buf(kstep(st + 2), q2);
      compute(q0, st);
      fetch_buf(kstep(st + 3), q0);
      compute(q1, st + 1);
      fetch_buf(kstep(st + 4), q1);
      compute(q2, st + 2);
    }
  } else {
    Stage cur, nxt;
    if (nst > 0) fetch(kstep(0), cur);
    for (int st = 0; st < nst; ++st) {
      if (st + 1 < nst) fetch(kstep(st + 1), nxt);
      compute(cur, st);
      cur = nxt;
    }
  }
  if constexpr (VS) {
    // the four waves' sums of the same pairs, added in wave order through LDS
    __shared__ double red[3][TT * TT * 8][64];
    if (wave > 0) {
#pragma unroll
      for (int ta = 0; ta < TT; ++ta)
#pragma unroll
        for (int tb = 0; tb < TT; ++tb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            red[wave - 1][((ta * TT + tb) * 4 + r) * 2][lane] = totR[ta][tb][r];
            red[wave - 1][((ta * TT + tb) * 4 + r) * 2 + 1][lane] = totI[ta][tb][r];
          }
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int ta = 0; ta < TT; ++ta)
#pragma unroll
        for (int tb = 0; tb < TT; ++tb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            totR[ta][tb][r] += red[w][((ta * TT + tb) * 4 + r) * 2][lane];
            totI[ta][tb][r] += red[w][((ta * TT + tb) * 4 + r) * 2 + 1][lane];
          }
  }
  // accumulator register r of lane (col = lane%16, g) holds row 4g + r of the tile
  double* out = part + ((size_t)(c * L + l) * nsplit + split) * (size_t)S * D * 2;
#pragma unroll
  for (int ta = 0; ta < TT; ++ta)
#pragma unroll
    for (int tb = 0; tb < TT; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = 32 * wa + 16 * ta + 4 * g + r, d = 32 * wb + 16 * tb + r16;
        if (s < S && d < D) {
          const size_t o = ((size_t)s * D + d) * 2;
          out[o] = totR[ta][tb][r];
          out[o + 1] = totI[ta][tb][r];
        }
      }
}

// J v for complex FP64 fields with S and D above 32 (fewer than 12 probe vectors) on the FP64
// MFMA (v_mfma_f64_16x16x4f64), in the block and wave layout of k_born_jv_wide: wave (wa, wb)
// owns sources [32 wa, 32 wa + 32) and detectors [32 wb, 32 wb + 32) as 2 x 2 tiles of 16 x 16.
// Per 16-voxel step lane (r16, g) supplies row r16 of each tile at voxels g, g + 4, g + 8, g + 12
// (k-step i takes voxel 4i + g, so the four lanes of a row read 64 contiguous bytes per load),
// A = phi_s v and B = phi_d; Re y and Im y accumulate in FP64 on the MFMA
// over the block's whole voxel range (accumulator register r of a lane holds row 4r + g).  The
// next step's operands are loaded while the current step's products run.  Partials as
// k_born_jv_wide.  BUF: the operands through buffer resources over this wavelength's rows (one
// wavelength's rows below 2 GiB), so no load sits under a branch (loads under a branch are
// waited for at its end) and steps past the range read zeros; two stage buffers in rotation.
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <bool BUF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_jv_wide64(
    int N, int S, int D, int64_t lam_stride, const cd* __restrict__ phs, const cd* __restrict__ phd,
    const double* __restrict__ v, int kb, int L, double* __restrict__ part) {
  const int split = blockIdx.x, l = blockIdx.y, c = blockIdx.z, nsplit = gridDim.x;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int wa = wave >> 1, wb = wave & 1;
  const size_t Nz = (size_t)N;
  bool sok[2], dok[2];
  int srow[2], drow[2];
  const cd* pa[2];
  const cd* pb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    srow[t] = 32 * wa + 16 * t + r16;
    drow[t] = 32 * wb + 16 * t + r16;
    sok[t] = srow[t] < S;
    dok[t] = drow[t] < D;
    pa[t] = phs + ((size_t)l * lam_stride + (sok[t] ? srow[t] : 0)) * Nz;
    pb[t] = phd + ((size_t)l * lam_stride + (dok[t] ? drow[t] : 0)) * Nz;
  }
  const double* vc = v + (size_t)c * Nz;
  struct Stage {
    cd a[2][4], b[2][4];
    double vv[4];
  };
  auto fetch = [&](int kbase, Stage& st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = kbase + 4 * i + g;
      const bool ok = k < k1;
      st.vv[i] = ok ? vc[k] : 0.0;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        st.a[t][i] = ok && sok[t] ? pa[t][k] : cd{0.0, 0.0};
        st.b[t][i] = ok && dok[t] ? pb[t][k] : cd{0.0, 0.0};
      }
    }
  };
  const __amdgpu_buffer_rsrc_t ra = wide_rsrc(phs + (size_t)l * lam_stride * Nz, BUF ? (uint32_t)S * (uint32_t)N * 16u : 0u);
  const __amdgpu_buffer_rsrc_t rb = wide_rsrc(phd + (size_t)l * lam_stride * Nz, BUF ? (uint32_t)D * (uint32_t)N * 16u : 0u);
  const __amdgpu_buffer_rsrc_t rv = wide_rsrc(vc, BUF ? (uint32_t)N * 8u : 0u);
  auto fetch_buf = [&](int kbase, Stage& st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = kbase + 4 * i + g;
      const bool in = k < k1;
      st.vv[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rv, in ? (uint32_t)k * 8u : kWideOut, 0, 0));
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const uint32_t oa = in && sok[t] ? ((uint32_t)srow[t] * (uint32_t)N + (uint32_t)k) * 16u : kWideOut;
        const uint32_t ob = in && dok[t] ? ((uint32_t)drow[t] * (uint32_t)N + (uint32_t)k) * 16u : kWideOut;
        const f64x2 xa = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(ra, oa, 0, 0));
        const f64x2 xb = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rb, ob, 0, 0));
        st.a[t][i] = cd{xa[0], xa[1]};
        st.b[t][i] = cd{xb[0], xb[1]};
      }
    }
  };
  f64x4 accR[2][2], accI[2][2];
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      accR[ta][tb] = f64x4{0.0, 0.0, 0.0, 0.0};
      accI[ta][tb] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
  auto compute = [&](const Stage& cur) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double ar[2], ai[2], nai[2];
#pragma unroll
      for (int ta = 0; ta < 2; ++ta) {
        ar[ta] = cur.a[ta][i].re * cur.vv[i];
        ai[ta] = cur.a[ta][i].im * cur.vv[i];
        nai[ta] = -ai[ta];
      }
      // Re y += Re a Re b - Im a Im b, Im y += Re a Im b + Im a Re b
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int ta = 0; ta < 2; ++ta) {
          accR[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ta], cur.b[tb][i].re, accR[ta][tb], 0, 0, 0);
          accI[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ta], cur.b[tb][i].im, accI[ta][tb], 0, 0, 0);
        }
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int ta = 0; ta < 2; ++ta) {
          accR[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[ta], cur.b[tb][i].im, accR[ta][tb], 0, 0, 0);
          accI[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[ta], cur.b[tb][i].re, accI[ta][tb], 0, 0, 0);
        }
    }
  };
  const int nst = k1 > k0 ? (k1 - k0 + 15) / 16 : 0;
  if constexpr (BUF) {
    // two stage buffers in rotation (unrolled by two, so no stage is copied: a copy would wait
    // for its loads); a step past the range reads zeros and adds nothing
    // (the scheduling barriers keep each step's loads ahead of the products before them)
    Stage q0, q1;
    fetch_buf(k0, q0);
    for (int st = 0; st < nst; st += 2) {
      fetch_buf(k0 + 16 * (st + 1), q1);
      __builtin_amdgcn_sched_barrier(0);
      compute(q0);
      __builtin_amdgcn_sched_barrier(0);
      fetch_buf(k0 + 16 * (st + 2), q0);
      __builtin_amdgcn_sched_barrier(0);
      compute(q1);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    Stage cur, nxt;
    if (nst > 0) fetch(k0, cur);
    for (int st = 0; st < nst; ++st) {
      if (st + 1 < nst) fetch(k0 + 16 * (st + 1), nxt);
      compute(cur);
      cur = nxt;
    }
  }
  double* out = part + ((size_t)(c * L + l) * nsplit + split) * (size_t)S * D * 2;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = 32 * wa + 16 * ta + 4 * r + g, d = 32 * wb + 16 * tb + r16;
        if (s < S && d < D) {
          const size_t o = ((size_t)s * D + d) * 2;
          out[o] = accR[ta][tb][r];
          out[o + 1] = accI[ta][tb][r];
        }
      }
}

// ---------------------------------------------------------------- J v on the BF16 MFMA
// The same products from BF16 operands on v_mfma_f32_16x16x32_bf16: CM_BF16 takes BF16-stored
// fields (cbf) and rounds a = phi_s v (formed in FP32) to BF16, phi_d entering as stored;
// CM_SPLIT takes FP32 fields and splits a and phi_d into hi + lo BF16 parts, accumulating
// hi*hi + hi*lo + lo*hi.  Lane (r = lane%16, g = lane/16) supplies row r at voxels 8g..8g+7 of a
// 32-voxel step for both operands (one MFMA k-step per step).  Block and waves as
// k_born_jv_wide: wave (wa, wb) owns 32 sources x 32 detectors as 2 x 2 tiles, so each converted
// operand feeds two tiles.  FP32 MFMA sums cover wide_bf_ns steps and are then folded into FP64
// running sums held in LDS; the four waves synchronise once per such stage; with BF16 storage the
// raw field words of the next steps (four with 16-byte loads) are in flight while the current
// step's products run; partials as k_born_jv_wide.  VEC: 16-byte loads (N a multiple of 8, base
// pointers 16-byte aligned).
typedef __bf16 wbf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// 32-voxel steps per FP32 partial sum: 256 voxels for BF16 products (their rounding, 2^-9, far
// exceeds the FP32 summation error), 128 for the split
template <int CM>
constexpr int wide_bf_ns() { return CM == CM_SPLIT ? 4 : 8; }
constexpr int kWideBfKt = 256;   // voxel ranges: a multiple of both

// raw words of eight voxels of one field row: BF16 storage (re, im) pairs in 8 words, FP32 in 16
template <typename TS>
struct Raw8 {
  static constexpr int nw = std::is_same<TS, cbf>::value ? 8 : 16;
  unsigned int w[nw];
};

// Voxel of lane-local index i within a 32-voxel step: lane g takes voxels 8g..8g+7 (its two
// 16-byte loads of a BF16 row, four of an FP32 row, are contiguous), the MFMA k-step 8g + i
template <typename TS>
__device__ inline int vox_in_step(int i, int g) {
  return 8 * g + i;
}

// VEC: N and every range end are multiples of 8, so a lane's eight voxels lie all inside the range
// or all past it; rows are read through buffer resources (row_off = byte offset of the row, or
// kWideOut for a missing row; a piece past the range reads zeros without a branch)
template <typename TS>
__device__ inline void load_raw8_buf(__amdgpu_buffer_rsrc_t r, uint32_t row_off, int kbase, int g, int k1,
                                     Raw8<TS>& q) {
  constexpr int nw = Raw8<TS>::nw;
  const int first = kbase + 8 * g;
  const uint32_t off = row_off != kWideOut && first < k1 ? row_off + (uint32_t)first * (uint32_t)sizeof(TS) : kWideOut;
#pragma unroll
  for (int j = 0; j < nw / 4; ++j) {
    const u32x4 x = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u * j, 0, 0));
#pragma unroll
    for (int i = 0; i < 4; ++i) q.w[4 * j + i] = x[i];
  }
}
// element by element (any N), zeros past the range or for a missing row
template <typename TS>
__device__ inline void load_raw8(const TS* p, int kbase, int g, int k1, bool row_ok, Raw8<TS>& r) {
  constexpr int nw = Raw8<TS>::nw;
  const unsigned int* q = reinterpret_cast<const unsigned int*>(p);
  constexpr int wpv = nw / 8;   // words per voxel
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = kbase + vox_in_step<TS>(i, g);
    const bool ok = row_ok && k < k1;
#pragma unroll
    for (int u = 0; u < wpv; ++u) r.w[wpv * i + u] = ok ? q[(size_t)k * wpv + u] : 0u;
  }
}
// FP32 (re, im) of voxel i from the raw words
template <typename TS>
__device__ inline float raw_re(const Raw8<TS>& r, int i) {
  if constexpr (std::is_same<TS, cbf>::value) return __builtin_bit_cast(float, r.w[i] << 16);
  else return __builtin_bit_cast(float, r.w[2 * i]);
}
template <typename TS>
__device__ inline float raw_im(const Raw8<TS>& r, int i) {
  if constexpr (std::is_same<TS, cbf>::value) return __builtin_bit_cast(float, r.w[i] & 0xffff0000u);
  else return __builtin_bit_cast(float, r.w[2 * i + 1]);
}

__device__ inline wbf16x8 bf8_round(const float* x) {
  wbf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)x[i];
  return r;
}
// x - hi rounded to BF16 (the lo part of the split)
__device__ inline wbf16x8 bf8_lo(const float* x, wbf16x8 hi) {
  wbf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = (__bf16)(x[i] - (float)hi[i]);
  return r;
}
__device__ inline wbf16x8 bf8_neg(wbf16x8 x) {   // exact: flips the sign bits
  return __builtin_bit_cast(wbf16x8, __builtin_bit_cast(u32x4, x) ^ u32x4{0x80008000u, 0x80008000u, 0x80008000u,
                                                                           0x80008000u});
}

// BF16 storage: the re (low halves) and im (high halves) of eight voxels packed straight into
// MFMA operands (exact, no widening)
__device__ inline void bf8_unzip(const unsigned int* w, wbf16x8& re, wbf16x8& im) {
  u32x4 r, i;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    r[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x05040100u);   // low halves of w[2j], w[2j+1]
    i[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], 0x07060302u);   // high halves
  }
  re = __builtin_bit_cast(wbf16x8, r);
  im = __builtin_bit_cast(wbf16x8, i);
}

template <typename TS, int CM>
struct BfOps {   // BF16 operands of one row and step: hi (and lo for the split)
  wbf16x8 re, im, re_lo, im_lo;
};
template <typename TS, int CM>
__device__ inline BfOps<TS, CM> bf_ops(const float* re, const float* im) {
  BfOps<TS, CM> o;
  o.re = bf8_round(re);
  o.im = bf8_round(im);
  if constexpr (CM == CM_SPLIT) {
    o.re_lo = bf8_lo(re, o.re);
    o.im_lo = bf8_lo(im, o.im);
  }
  return o;
}
// acc += x y over the BF16 parts: x.hi y.hi (+ x.hi y.lo + x.lo y.hi for the split)
template <int CM>
__device__ inline f32x4 bf_mac(wbf16x8 xh, wbf16x8 xl, wbf16x8 yh, wbf16x8 yl, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);
  if constexpr (CM == CM_SPLIT) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
  }
  return acc;
}

template <typename TS, int CM, bool VEC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_jv_wide_bf(int N, int S, int D, int64_t lam_stride,
                                                           const TS* __restrict__ phs, const TS* __restrict__ phd,
                                                           const float* __restrict__ v, int kb, int L,
                                                           double* __restrict__ part) {
  static_assert(CM == CM_BF16 || CM == CM_SPLIT, "BF16 MFMA products");
  const int split = blockIdx.x, l = blockIdx.y, c = blockIdx.z, nsplit = gridDim.x;
  const int k0 = split * kb, k1 = min(N, k0 + kb);
  auto kstep = [&](int st) { return k0 + 32 * st; };
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int wa = wave >> 1, wb = wave & 1;
  const size_t Nz = (size_t)N;
  bool sok[2], dok[2];
  const TS* pa[2];
  const TS* pb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int s = 32 * wa + 16 * t + r16, d = 32 * wb + 16 * t + r16;
    sok[t] = s < S;
    dok[t] = d < D;
    pa[t] = phs + ((size_t)l * lam_stride + (sok[t] ? s : 0)) * Nz;
    pb[t] = phd + ((size_t)l * lam_stride + (dok[t] ? d : 0)) * Nz;
  }
  const float* vc = v + (size_t)c * Nz;
  // one step's raw words: two source rows, two detector rows, eight probe-vector values
  struct Step {
    Raw8<TS> ra[2], rb[2];
    float vv[8];
  };
  // VEC: buffer resources over this wavelength's source rows, detector rows and the probe vector
  // (the host keeps each below 2 GiB)
  const uint32_t rowb = (uint32_t)(Nz * sizeof(TS));
  const __amdgpu_buffer_rsrc_t rsA = wide_rsrc(phs + (size_t)l * lam_stride * Nz, (uint32_t)S * rowb);
  const __amdgpu_buffer_rsrc_t rsB = wide_rsrc(phd + (size_t)l * lam_stride * Nz, (uint32_t)D * rowb);
  const __amdgpu_buffer_rsrc_t rsV = wide_rsrc(vc, (uint32_t)(Nz * sizeof(float)));
  uint32_t offA[2], offB[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    offA[t] = sok[t] ? (uint32_t)(32 * wa + 16 * t + r16) * rowb : kWideOut;
    offB[t] = dok[t] ? (uint32_t)(32 * wb + 16 * t + r16) * rowb : kWideOut;
  }
  auto fetch = [&](int kbase, Step& q) {
    if constexpr (VEC) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        load_raw8_buf(rsA, offA[t], kbase, g, k1, q.ra[t]);
        load_raw8_buf(rsB, offB[t], kbase, g, k1, q.rb[t]);
      }
      // the probe vector at the same voxels
      const int first = kbase + 8 * g;
      const uint32_t vo = first < k1 ? (uint32_t)first * 4u : kWideOut;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsV, vo + 16u * j, 0, 0));
#pragma unroll
        for (int i = 0; i < 4; ++i) q.vv[4 * j + i] = x[i];
      }
    } else {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        load_raw8(pa[t], kbase, g, k1, sok[t], q.ra[t]);
        load_raw8(pb[t], kbase, g, k1, dok[t], q.rb[t]);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = kbase + vox_in_step<TS>(i, g);
        q.vv[i] = k < k1 ? vc[k] : 0.f;
      }
    }
  };
  f32x4 accR[2][2], accI[2][2];
  // FP64 running sums in LDS, one slot per (wave, tile, entry, part) and lane: their registers
  // hold loads in flight instead
  __shared__ double tot[4 * 2 * 2 * 4 * 2 * 64];
  auto tslot = [&](int ta, int tb, int r, int part) {
    return ((((wave * 2 + ta) * 2 + tb) * 4 + r) * 2 + part) * 64 + lane;
  };
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      accR[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
      accI[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) tot[tslot(ta, tb, r, 0)] = tot[tslot(ta, tb, r, 1)] = 0.0;
    }
  // BF16 operands of step st from its raw words, then (BF16 storage) the loads of step
  // st + kDepth into the same buffer, then the products; steps rotate over kDepth buffers
  // BF16 storage: the raw words of the next kDepth steps are in flight while step st runs (two
  // waves per SIMD); the split's FP32 rows would leave one, so it loads each step's words at
  // its start
  constexpr bool kPrefetch = CM == CM_BF16;
  constexpr int kDepth = VEC ? 4 : 2;   // element loads (any N) take more registers
  auto step = [&](int st, Step& q) {
    if (!kPrefetch) fetch(kstep(st), q);
    BfOps<TS, CM> A[2], An[2], B[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float xr[8], xi[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        xr[i] = raw_re(q.ra[t], i) * q.vv[i];
        xi[i] = raw_im(q.ra[t], i) * q.vv[i];
      }
      A[t] = bf_ops<TS, CM>(xr, xi);
      An[t].im = bf8_neg(A[t].im);
      if constexpr (CM == CM_SPLIT) An[t].im_lo = bf8_neg(A[t].im_lo);
      if constexpr (std::is_same<TS, cbf>::value) {
        bf8_unzip(q.rb[t].w, B[t].re, B[t].im);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          xr[i] = raw_re(q.rb[t], i);
          xi[i] = raw_im(q.rb[t], i);
        }
        B[t] = bf_ops<TS, CM>(xr, xi);
      }
    }
    if (kPrefetch) fetch(kstep(st + kDepth), q);   // past the range it reads zeros
    // Re y += Re a Re b - Im a Im b, Im y += Re a Im b + Im a Re b
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int ta = 0; ta < 2; ++ta) {
        accR[ta][tb] = bf_mac<CM>(A[ta].re, A[ta].re_lo, B[tb].re, B[tb].re_lo, accR[ta][tb]);
        accR[ta][tb] = bf_mac<CM>(An[ta].im, An[ta].im_lo, B[tb].im, B[tb].im_lo, accR[ta][tb]);
        accI[ta][tb] = bf_mac<CM>(A[ta].re, A[ta].re_lo, B[tb].im, B[tb].im_lo, accI[ta][tb]);
        accI[ta][tb] = bf_mac<CM>(A[ta].im, A[ta].im_lo, B[tb].re, B[tb].re_lo, accI[ta][tb]);
      }
  };
  // whole FP32 stages of NS steps (a partial last stage runs its missing steps on zeros)
  constexpr int NS = wide_bf_ns<CM>();
  const int nst = k1 > k0 ? (k1 - k0 + 31) / 32 : 0;
  static_assert(NS % kDepth == 0, "stages hold whole rotations of the step buffers");
  Step q[kDepth];
  if (kPrefetch) {
#pragma unroll
    for (int u = 0; u < kDepth; ++u) fetch(kstep(u), q[u]);
  }
  for (int st0 = 0; st0 < nst; st0 += NS) {
    // the four waves stay within one FP32 stage of each other, so that the second read of a row
    // shared by two waves finds it in the cache (1.0x instead of 1.27-1.33x the field bytes
    // fetched; the FP32-MFMA kernel is slower with it and has none)
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NS; ++u) step(st0 + u, q[u % kDepth]);
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tot[tslot(ta, tb, r, 0)] += (double)accR[ta][tb][r];
          tot[tslot(ta, tb, r, 1)] += (double)accI[ta][tb][r];
        }
        accR[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
        accI[ta][tb] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  }
  // accumulator register r of lane (col = lane%16, g) holds row 4g + r of the tile
  double* out = part + ((size_t)(c * L + l) * nsplit + split) * (size_t)S * D * 2;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = 32 * wa + 16 * ta + 4 * g + r, d = 32 * wb + 16 * tb + r16;
        if (s < S && d < D) {
          const size_t o = ((size_t)s * D + d) * 2;
          out[o] = tot[tslot(ta, tb, r, 0)];
          out[o + 1] = tot[tslot(ta, tb, r, 1)];
        }
      }
}

// ---------------------------------------------------------------- J^H w
// g[k] = scale sum_l sum_d conj(phi_d(k)) T_l[k][d],  T_l[k][d] = sum_s conj(phi_s(k)) w_l[s][d].
// Block = 4 waves on 64 voxels (16 per wave), looping over the wavelengths.  Per wavelength the
// block stages w_l (S x D, zero-padded to 64 x 64) in LDS; each wave forms T for its 16 voxels
// and the 64 detector columns on the MFMA: A[row = voxel][k] = conj(phi_s), lane (voxel
// vox0 + lane%16, group g = lane/16) holding the sources s = g + 4q, q < 16 (each load reads 16
// consecutive voxels of one source row across the lanes: 128 bytes), so that the q-th k-step
// takes source g + 4q in every group; B[k][col] = w[g + 4q][16 t + lane%16] from LDS, t < 4
// column tiles.  Re T accumulates Re phi Re w + Im phi Im w and Im T accumulates
// Re phi Im w + (-Im phi) Re w (FP32 over the 64 sources of one wavelength).  The epilogue
// contracts T with conj(phi_d) at the lane's accumulator entries (voxel vox0 + 4g + r,
// detector 16 t + lane%16) into FP64 sums over the wavelengths, which are reduced over the 16
// detector lanes at the end.  The next wavelength's source values and w_l are loaded while
// the current products run.  VEC: 16-byte loads of the detector fields (N a multiple of 4,
// base pointers 16-byte aligned).
constexpr int kWPitch = 66;    // LDS row pitch of w (complex elements)

// QN source k-steps of 4 (sources up to 4 QN) and TD detector tiles of 16 (detectors up to
// 16 TD): 16 and 4 above 32 sources and detectors, fewer for smaller S and D (one data vector)
// BUF (the 64 x 64 instance with 16-byte loads, one wavelength's rows below 2 GiB): w_l, the
// detector fields of wavelength l and the source values of l + 1 through buffer resources, all
// issued at the top of the wavelength with no load under a branch (loads under a branch are
// waited for at its end), so only w_l is waited for before the LDS stores.
template <bool VEC, int QN = 16, int TD = 4, bool BUF = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_adjoint_wide(int N, int S, int D, int64_t lam_stride, int L,
                                                             const cf* __restrict__ phs,
                                                             const cf* __restrict__ phd,
                                                             const cf* __restrict__ w, double scale,
                                                             cf* __restrict__ gout) {
  __shared__ cf Ws[64 * kWPitch];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int vox0 = (blockIdx.x * 4 + wave) * 16;
  const int vox = vox0 + r16;               // A row of this lane
  const bool vok = vox < N;
  const size_t Nz = (size_t)N;
  // w_l staging.  With all 16 source steps thread tid copies the elements e = tid + 256 j of the
  // 64 x 64 padded tile, between two barriers per wavelength.  With fewer (S, D <= 32, so
  // S D <= 4 x 256) each thread carries the elements e = tid + 256 j, j < 4, of w_{l+1} in
  // registers while wavelength l is computed and then stores them into the other half of Ws
  // (two 32-row buffers whose padding is cleared once): one barrier per wavelength, and the
  // loads of w overlap the products.
  auto stage_w = [&](int l) {
    const cf* wl = w + (size_t)l * S * D;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int e = tid + 256 * j, s = e >> 6, d = e & 63;
      Ws[s * kWPitch + d] = s < S && d < D ? wl[s * D + d] : cf{0.f, 0.f};
    }
  };
  constexpr int kWHalf = 32 * kWPitch;
  constexpr int kWE = QN == 16 ? 1 : 4;
  int woff[kWE];
  cf wr[kWE];
  if constexpr (QN != 16) {
    const int SD = S * D;
#pragma unroll
    for (int j = 0; j < kWE; ++j) {
      const int e = tid + 256 * j, s = e / D;
      woff[j] = e < SD ? s * kWPitch + (e - s * D) : -1;
    }
    for (int e = tid; e < 64 * kWPitch; e += kBlock) Ws[e] = cf{0.f, 0.f};
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kWE; ++j)
      if (woff[j] >= 0) Ws[woff[j]] = w[tid + 256 * j];
    __syncthreads();
  }
  // sources s = g + 4q of this lane's voxel
  cf za[QN], zn[QN];
  auto fetch_s = [&](int l, cf (&z)[QN]) {
    const cf* ps = phs + (size_t)l * lam_stride * Nz;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int s = g + 4 * q;
      z[q] = vok && s < S ? ps[(size_t)s * Nz + vox] : cf{0.f, 0.f};
    }
  };
  // detector fields at the accumulator entries: detector 16 t + r16, voxels vox0 + 4g + r
  auto fetch_d = [&](int l, cf (&ph)[TD][4]) {
    const cf* pd = phd + (size_t)l * lam_stride * Nz;
    const int vb = vox0 + 4 * g;
#pragma unroll
    for (int t = 0; t < TD; ++t) {
      const int d = 16 * t + r16;
      const bool dk = d < D;
      const cf* row = pd + (size_t)(dk ? d : 0) * Nz;
      if (VEC && vb + 4 <= N) {
        if (dk) {
          ld2cf(row + vb, ph[t][0], ph[t][1]);
          ld2cf(row + vb + 2, ph[t][2], ph[t][3]);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) ph[t][r] = cf{0.f, 0.f};
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) ph[t][r] = dk && vb + r < N ? row[vb + r] : cf{0.f, 0.f};
      }
    }
  };
  double gre[4], gim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) gre[r] = gim[r] = 0.0;
  if constexpr (BUF) {
    static_assert(QN == 16 && TD == 4 && VEC, "the buffer form is the 64 x 64 instance with 16-byte loads");
    // source values of wavelength l (none past the last one)
    auto fetch_s_buf = [&](int l, cf (&z)[QN]) {
      const __amdgpu_buffer_rsrc_t r =
          wide_rsrc(phs + (size_t)l * lam_stride * Nz, l < L ? (uint32_t)S * (uint32_t)N * 8u : 0u);
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int s = g + 4 * q;
        const uint32_t off = vok && s < S ? ((uint32_t)s * (uint32_t)N + (uint32_t)vox) * 8u : kWideOut;
        z[q] = __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
      }
    };
    fetch_s_buf(0, za);
    const int vb = vox0 + 4 * g;
    for (int l = 0; l < L; ++l) {
      // w_l (16 elements of the padded 64 x 64 tile per thread), then the detector fields of l
      // and the source values of l + 1
      const __amdgpu_buffer_rsrc_t rw = wide_rsrc(w + (size_t)l * S * D, (uint32_t)S * (uint32_t)D * 8u);
      cf wt[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int e = tid + 256 * j, s = e >> 6, d = e & 63;
        const uint32_t off = s < S && d < D ? (uint32_t)(s * D + d) * 8u : kWideOut;
        wt[j] = __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(rw, off, 0, 0));
      }
      const __amdgpu_buffer_rsrc_t rd = wide_rsrc(phd + (size_t)l * lam_stride * Nz, (uint32_t)D * (uint32_t)N * 8u);
      cf ph[TD][4];
#pragma unroll
      for (int t = 0; t < TD; ++t) {
        const int d = 16 * t + r16;
        const uint32_t off = d < D && vb < N ? ((uint32_t)d * (uint32_t)N + (uint32_t)vb) * 8u : kWideOut;
        const f32x4 x0 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rd, off, 0, 0));
        const f32x4 x1 = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rd, off + 16u, 0, 0));
        ph[t][0] = cf{x0[0], x0[1]};
        ph[t][1] = cf{x0[2], x0[3]};
        ph[t][2] = cf{x1[0], x1[1]};
        ph[t][3] = cf{x1[2], x1[3]};
      }
      fetch_s_buf(l + 1, zn);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();        // the previous wavelength's reads of Ws are done
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int e = tid + 256 * j;
        Ws[(e >> 6) * kWPitch + (e & 63)] = wt[j];
      }
      __syncthreads();
      f32x4 accR[TD], accI[TD];
#pragma unroll
      for (int t = 0; t < TD; ++t) {
        accR[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        accI[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const float pr = za[q].re, pi = za[q].im, npi = -pi;
        const cf* wrow = Ws + (g + 4 * q) * kWPitch + r16;
        cf ww[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t) ww[t] = wrow[16 * t];
#pragma unroll
        for (int t = 0; t < TD; ++t) {
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, ww[t].re, accR[t], 0, 0, 0);
          accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, ww[t].im, accI[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < TD; ++t) {
          accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pi, ww[t].im, accR[t], 0, 0, 0);
          accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(npi, ww[t].re, accI[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int t = 0; t < TD; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double e = ph[t][r].re, f = ph[t][r].im;
          const double tr = (double)accR[t][r], ti = (double)accI[t][r];
          gre[r] += e * tr + f * ti;
          gim[r] += e * ti - f * tr;
        }
#pragma unroll
      for (int q = 0; q < QN; ++q) za[q] = zn[q];
    }
  } else {
  fetch_s(0, za);
  for (int l = 0; l < L; ++l) {
    const cf* Wc = Ws;
    if constexpr (QN == 16) {
      __syncthreads();        // the previous wavelength's reads of Ws are done
      stage_w(l);
      __syncthreads();
    } else {
      Wc = Ws + (l & 1) * kWHalf;
      if (l + 1 < L) {
        const cf* wn = w + (size_t)(l + 1) * S * D;
#pragma unroll
        for (int j = 0; j < kWE; ++j) wr[j] = woff[j] >= 0 ? wn[tid + 256 * j] : cf{0.f, 0.f};
      }
    }
    cf ph[TD][4];
    fetch_d(l, ph);           // used by the epilogue, after the products
    if (l + 1 < L) fetch_s(l + 1, zn);
    f32x4 accR[TD], accI[TD];
#pragma unroll
    for (int t = 0; t < TD; ++t) {
      accR[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      accI[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const float pr = za[q].re, pi = za[q].im, npi = -pi;
      const cf* wrow = Wc + (g + 4 * q) * kWPitch + r16;
      cf ww[TD];
#pragma unroll
      for (int t = 0; t < TD; ++t) ww[t] = wrow[16 * t];
      // 2 TD independent accumulators between two products into the same one
#pragma unroll
      for (int t = 0; t < TD; ++t) {
        accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, ww[t].re, accR[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, ww[t].im, accI[t], 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < TD; ++t) {
        accR[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pi, ww[t].im, accR[t], 0, 0, 0);
        accI[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(npi, ww[t].re, accI[t], 0, 0, 0);
      }
    }
    // conj(phi_d) T, FP64; accumulator register r of lane (col r16, g) is voxel vox0 + 4g + r
#pragma unroll
    for (int t = 0; t < TD; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double e = ph[t][r].re, f = ph[t][r].im;
        const double tr = (double)accR[t][r], ti = (double)accI[t][r];
        gre[r] += e * tr + f * ti;
        gim[r] += e * ti - f * tr;
      }
    if constexpr (QN != 16) {
      // w_{l+1} into the buffer not read in this wavelength; the barrier also ends this
      // wavelength's reads of Wc before the next one overwrites it
      if (l + 1 < L) {
        cf* Wn = Ws + ((l + 1) & 1) * kWHalf;
#pragma unroll
        for (int j = 0; j < kWE; ++j)
          if (woff[j] >= 0) Wn[woff[j]] = wr[j];
      }
      __syncthreads();
    }
    if (l + 1 < L) {
#pragma unroll
      for (int q = 0; q < QN; ++q) za[q] = zn[q];
    }
  }
  }
  // sum over the 16 detector lanes of each voxel
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      gre[r] += __shfl_xor(gre[r], off, 64);
      gim[r] += __shfl_xor(gim[r], off, 64);
    }
  }
  if (r16 == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vv = vox0 + 4 * g + r;
      if (vv < N) gout[vv] = cf{(float)(scale * gre[r]), (float)(scale * gim[r])};
    }
  }
}

// J^H w for complex FP64 fields with S and D above 32 (one data vector per launch) on the FP64
// MFMA (v_mfma_f64_16x16x4f64), in the layout of k_born_adjoint_wide: a wave takes 16 voxels,
// lane (r16 = lane%16, g = lane/16) holds the sources s = g + 4q (q < 16) of voxel vox0 + r16 as
// A[row = voxel][k], and B[k][col] = w[g + 4q][16 t + r16] comes from LDS (t < 4 column tiles,
// the 64 x 64 tile of w_l staged once per block and wavelength).  Re T and Im T accumulate in
// FP64 over the sources; the FP64 accumulator register r of a lane holds row 4 r + g, so the
// epilogue contracts T with conj(phi_d) at voxels vox0 + 4 r + g and detectors 16 t + r16, and
// the sums over the 16 detector lanes follow at the end.  Two waves per SIMD: the fields of one
// wavelength are loaded at its start (the other wave's products cover the wait).
constexpr int kWPitch64 = 65;   // LDS row pitch of w (complex FP64 elements)

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_adjoint_wide64(
    int N, int S, int D, int64_t lam_stride, int L, const cd* __restrict__ phs, const cd* __restrict__ phd,
    const cd* __restrict__ w, double scale, cd* __restrict__ gout) {
  __shared__ cd Ws[64 * kWPitch64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int vox0 = (blockIdx.x * 4 + wave) * 16;
  const int vox = vox0 + r16;
  const bool vok = vox < N;
  const size_t Nz = (size_t)N;
  double gre[4], gim[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) gre[r] = gim[r] = 0.0;
  for (int l = 0; l < L; ++l) {
    const cd* ps = phs + (size_t)l * lam_stride * Nz;
    const cd* pd = phd + (size_t)l * lam_stride * Nz;
    cd z[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int s = g + 4 * q;
      z[q] = vok && s < S ? ps[(size_t)s * Nz + vox] : cd{0.0, 0.0};
    }
    __syncthreads();          // the previous wavelength's reads of Ws are done
    const cd* wl = w + (size_t)l * S * D;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int e = tid + 256 * j, s = e >> 6, d = e & 63;
      Ws[s * kWPitch64 + d] = s < S && d < D ? wl[s * D + d] : cd{0.0, 0.0};
    }
    __syncthreads();
    // two passes of two detector tiles over the same source values
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      cd ph[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int d = 16 * (2 * p + u) + r16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int vv = vox0 + 4 * r + g;
          ph[u][r] = d < D && vv < N ? pd[(size_t)d * Nz + vv] : cd{0.0, 0.0};
        }
      }
      f64x4 accR[2], accI[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        accR[u] = f64x4{0.0, 0.0, 0.0, 0.0};
        accI[u] = f64x4{0.0, 0.0, 0.0, 0.0};
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double pr = z[q].re, pi = z[q].im, npi = -pi;
        const cd* wrow = Ws + (g + 4 * q) * kWPitch64 + 32 * p + r16;
        const cd w0 = wrow[0], w1 = wrow[16];
        // Re T += Re phi Re w + Im phi Im w, Im T += Re phi Im w - Im phi Re w
        accR[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, w0.re, accR[0], 0, 0, 0);
        accI[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, w0.im, accI[0], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, w1.re, accR[1], 0, 0, 0);
        accI[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, w1.im, accI[1], 0, 0, 0);
        accR[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, w0.im, accR[0], 0, 0, 0);
        accI[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(npi, w0.re, accI[0], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, w1.im, accR[1], 0, 0, 0);
        accI[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(npi, w1.re, accI[1], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double e = ph[u][r].re, f = ph[u][r].im, tr = accR[u][r], ti = accI[u][r];
          gre[r] += e * tr + f * ti;
          gim[r] += e * ti - f * tr;
        }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      gre[r] += __shfl_xor(gre[r], off, 64);
      gim[r] += __shfl_xor(gim[r], off, 64);
    }
  }
  if (r16 == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vv = vox0 + 4 * r + g;
      if (vv < N) gout[vv] = cd{scale * gre[r], scale * gim[r]};
    }
  }
}

// J^H w for BF16 fields with S and D above 32, on the BF16 MFMA.  Block = 4 waves on 256 voxels
// (64 per wave, in two passes of two 16-voxel tiles), looping over the wavelengths.  With the k
// index k = 2s + c (c = 0: real part, c = 1: imaginary part of source s) the product
// T[voxel][d] = sum_s conj(phi_s) w[s][d] is real: A[voxel][2s + c] = (Re phi_s, Im phi_s) is a
// BF16 field word as stored (two k values per 32-bit word), and
//   Re T = A B_re,  B_re[2s + c][d] = (Re w[s][d], Im w[s][d]),
//   Im T = A B_im,  B_im[2s + c][d] = (Im w[s][d], -Re w[s][d]).
// w is split exactly enough into BF16 hi + lo (hi = bf16(w), lo = bf16(w - hi); relative error of
// the pair about 2^-16), so the fields' BF16 storage is the only rounding of the operands.  Per
// wavelength the block stages the hi and lo words of B_re in LDS (rows d, columns s; a pitch of
// 68 words keeps each 16-byte operand read aligned); a B_im word is B_re's with its halves swapped
// and the sign bit of the new upper half flipped (exact).  Lane (r = lane%16, g = lane/16) of a
// tile takes, for k-step q, the four words of sources 16q + 4g + i (i < 4) at its voxel r from
// HBM and the four words of the same sources at detector 16t + r from LDS, one 16-byte read per
// operand, each operand serving both tiles of the pass.  T accumulates in FP32 over the sources;
// the epilogue contracts it with conj(phi_d) in FP64 at the lane's accumulator entries (voxels
// 4g + j of the tile, detector 16t + r: the four voxels of one detector row are one 16-byte word
// group), summed over the detectors and wavelengths and, at the end, over the 16 detector lanes.
// VEC: 16-byte loads of the detector words (N a multiple of 4, base pointers 16-byte aligned).
constexpr int kAdjBfPitch = 68;   // LDS row pitch (words) of the staged B operands
constexpr int kAdjBfVox = 256;    // voxels per block

template <bool VEC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_born_adjoint_wide_bf(int N, int S, int D, int64_t lam_stride, int L,
                                                                const cbf* __restrict__ phs,
                                                                const cbf* __restrict__ phd,
                                                                const cf* __restrict__ w, double scale,
                                                                cf* __restrict__ gout) {
  static_assert(kBlock == 256, "the staging maps 256 threads onto the 64 x 64 operand tile");
  __shared__ __attribute__((aligned(16))) unsigned int Bhi[64 * kAdjBfPitch];
  __shared__ __attribute__((aligned(16))) unsigned int Blo[64 * kAdjBfPitch];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int wbase = blockIdx.x * kAdjBfVox + wave * 64;   // this wave's 64 voxels
  const uint32_t rowb = (uint32_t)N * 4u;                 // bytes per field row
  double gre[2][2][4], gim[2][2][4];                      // [pass][tile][j]
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) gre[p][mt][j] = gim[p][mt][j] = 0.0;

  for (int l = 0; l < L; ++l) {
    __syncthreads();   // the previous wavelength's operand reads are done
    {
      const cf* wl = w + (size_t)l * S * D;
#pragma unroll 4
      for (int j = 0; j < 16; ++j) {
        const int s = 4 * j + wave, d = lane;   // element (s, d) of the padded 64 x 64 tile
        const cf x = s < S && d < D ? wl[s * D + d] : cf{0.f, 0.f};
        const __bf16 hr = (__bf16)x.re, hi_ = (__bf16)x.im;
        const __bf16 lr = (__bf16)(x.re - (float)hr), li = (__bf16)(x.im - (float)hi_);
        Bhi[d * kAdjBfPitch + s] = (unsigned)__builtin_bit_cast(unsigned short, hr) |
                                   ((unsigned)__builtin_bit_cast(unsigned short, hi_) << 16);
        Blo[d * kAdjBfPitch + s] = (unsigned)__builtin_bit_cast(unsigned short, lr) |
                                   ((unsigned)__builtin_bit_cast(unsigned short, li) << 16);
      }
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rs = wide_rsrc(phs + (size_t)l * lam_stride * N, (uint32_t)S * rowb);
    const __amdgpu_buffer_rsrc_t rd = wide_rsrc(phd + (size_t)l * lam_stride * N, (uint32_t)D * rowb);
#pragma unroll 1
    for (int p = 0; p < 2; ++p) {
      const int tb = wbase + 32 * p;   // first voxel of the pass's two tiles
      u32x4 a[2][4];                   // [tile][k-step]: words of sources 16q + 4g + i at voxel r
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int v = tb + 16 * mt + r16;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int s = 16 * q + 4 * g + i;
            const uint32_t off = s < S && v < N ? (uint32_t)s * rowb + (uint32_t)v * 4u : kWideOut;
            a[mt][q][i] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
          }
      }
      u32x4 ph[2][4];                  // [tile][detector tile]: words of voxels 4g + j at detector 16t + r
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int v0 = tb + 16 * mt + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int d = 16 * t + r16;
          if (VEC) {
            const uint32_t off = d < D && v0 < N ? (uint32_t)d * rowb + (uint32_t)v0 * 4u : kWideOut;
            ph[mt][t] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rd, off, 0, 0));
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t off = d < D && v0 + j < N ? (uint32_t)d * rowb + (uint32_t)(v0 + j) * 4u : kWideOut;
              ph[mt][t][j] = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(rd, off, 0, 0);
            }
          }
        }
      }
      f32x4 accR[2][4], accI[2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          accR[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
          accI[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      // the (k-step, detector tile) operands from LDS one step ahead of their products; the
      // scheduling barrier keeps the reads from being hoisted further (their registers)
      auto lds_op = [&](int it, u32x4& h, u32x4& lo) {
        const int o = (16 * (it & 3) + r16) * kAdjBfPitch + 16 * (it >> 2) + 4 * g;
        h = *reinterpret_cast<const u32x4*>(&Bhi[o]);
        lo = *reinterpret_cast<const u32x4*>(&Blo[o]);
      };
      u32x4 nbh, nbl;
      lds_op(0, nbh, nbl);
#pragma unroll
      for (int it = 0; it < 16; ++it) {
        const int q = it >> 2, t = it & 3;
        const u32x4 bh = nbh, bl = nbl;
        if (it + 1 < 16) lds_op(it + 1, nbh, nbl);
        u32x4 ih, il;   // B_im words: halves swapped, the new upper half negated
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ih[i] = __builtin_amdgcn_alignbit(bh[i], bh[i], 16) ^ 0x80000000u;
          il[i] = __builtin_amdgcn_alignbit(bl[i], bl[i], 16) ^ 0x80000000u;
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const wbf16x8 av = __builtin_bit_cast(wbf16x8, a[mt][q]);
          accR[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(wbf16x8, bh), accR[mt][t], 0, 0, 0);
          accI[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(wbf16x8, ih), accI[mt][t], 0, 0, 0);
          accR[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(wbf16x8, bl), accR[mt][t], 0, 0, 0);
          accI[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(wbf16x8, il), accI[mt][t], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // conj(phi_d) T in FP64: accumulator entry j of lane (r, g) is voxel 4g + j, detector 16t + r
      double er[2][4], ei[2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          er[mt][j] = ei[mt][j] = 0.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const unsigned x = ph[mt][t][j];
            const double e = __builtin_bit_cast(float, x << 16), f = __builtin_bit_cast(float, x & 0xffff0000u);
            const double tr = (double)accR[mt][t][j], ti = (double)accI[mt][t][j];
            er[mt][j] += e * tr + f * ti;
            ei[mt][j] += e * ti - f * tr;
          }
        }
      // added to the pass's own registers by a uniform branch (the pass loop stays rolled)
      if (p == 0) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            gre[0][mt][j] += er[mt][j];
            gim[0][mt][j] += ei[mt][j];
          }
      } else {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            gre[1][mt][j] += er[mt][j];
            gim[1][mt][j] += ei[mt][j];
          }
      }
    }
  }
  // sum over the 16 detector lanes of each voxel
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          gre[p][mt][j] += __shfl_xor(gre[p][mt][j], off, 64);
          gim[p][mt][j] += __shfl_xor(gim[p][mt][j], off, 64);
        }
      }
  if (r16 == 0) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int vv = wbase + 32 * p + 16 * mt + 4 * g + j;
          if (vv < N) gout[vv] = cf{(float)(scale * gre[p][mt][j]), (float)(scale * gim[p][mt][j])};
        }
  }
}

}  // namespace hydot
