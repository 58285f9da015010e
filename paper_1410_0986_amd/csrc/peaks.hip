// Achievable peaks of the GPU the library runs on, measured with hand-written probe kernels, so
// that rooflines can be stated against measured figures beside the published ones: HBM read
// streaming, a device copy, the read/write mix of an Arnoldi update (ten vectors read, one
// written), and loops of independent FP32 and BF16 MFMA instructions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace hydot {
namespace {

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kProbeBlock = 256;
constexpr int kProbeGrid = 8192;

// read NV vectors of M complex FP32 values (non-temporal) and write their sum (WRITE) or keep it
template <int NV, bool WRITE>
__global__ __launch_bounds__(kProbeBlock) void k_probe_stream(const f2v* __restrict__ v, f2v* __restrict__ out,
                                                              size_t M, float* __restrict__ sink) {
  f2v acc = {0.f, 0.f};
  for (size_t i = blockIdx.x * (size_t)kProbeBlock + threadIdx.x; i < M; i += (size_t)gridDim.x * kProbeBlock) {
    f2v s = {0.f, 0.f};
#pragma unroll
    for (int l = 0; l < NV; ++l) s += __builtin_nontemporal_load(&v[(size_t)l * M + i]);
    if (WRITE) __builtin_nontemporal_store(s, &out[i]);
    else acc += s;
  }
  // the sum is kept only so that the loads cannot be dropped; sink is written when it is NaN
  if (!WRITE && acc.x != acc.x) sink[blockIdx.x] = acc.y;
}

// independent MFMA chains per wave, operands in registers
__global__ __launch_bounds__(kProbeBlock) void k_probe_mfma_f32(int iters, float* __restrict__ sink) {
  f16v a0 = {}, a1 = {}, a2 = {}, a3 = {};
  const float x = (float)threadIdx.x * 1e-7f, y = 1.0f;
  for (int i = 0; i < iters; ++i) {
    a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a1, 0, 0, 0);
    a2 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a2, 0, 0, 0);
    a3 = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, a3, 0, 0, 0);
  }
  const float s = a0[0] + a1[1] + a2[2] + a3[3];
  if (s != s) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_mfma_bf16(int iters, float* __restrict__ sink) {
  f4v a0 = {}, a1 = {}, a2 = {}, a3 = {};
  bf8v x, y;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    x[i] = (__bf16)((float)threadIdx.x * 1e-7f);
    y[i] = (__bf16)1.0f;
  }
  for (int i = 0; i < iters; ++i) {
    a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, a1, 0, 0, 0);
    a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, a2, 0, 0, 0);
    a3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, a3, 0, 0, 0);
  }
  const float s = a0[0] + a1[1] + a2[2] + a3[3];
  if (s != s) sink[blockIdx.x] = s;
}

// median of five timed launches (after one untimed), in ms
template <typename F>
hydot_status time_ms(F launch, hipStream_t stream, double* out) {
  hipEvent_t e0, e1;
  HYDOT_HIP(hipEventCreate(&e0));
  HYDOT_HIP(hipEventCreate(&e1));
  float t[5];
  launch();
  for (int r = 0; r < 5; ++r) {
    HYDOT_HIP(hipEventRecord(e0, stream));
    launch();
    HYDOT_HIP(hipEventRecord(e1, stream));
    HYDOT_HIP(hipEventSynchronize(e1));
    HYDOT_HIP(hipEventElapsedTime(&t[r], e0, e1));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(t, t + 5);
  *out = t[2];
  return HYDOT_OK;
}

}  // namespace
}  // namespace hydot

using namespace hydot;

extern "C" hydot_status hydot_measure_peaks(void* buffer, size_t bytes, hydot_peaks* out, hipStream_t stream) {
  if (!buffer || !out) return fail(HYDOT_EINVAL, "measure_peaks: null argument");
  if (((uintptr_t)buffer & 255u) != 0) return fail(HYDOT_EINVAL, "measure_peaks: buffer must be 256-byte aligned");
  if (bytes < ((size_t)1 << 30)) return fail(HYDOT_EINVAL, "measure_peaks: buffer must hold at least 1 GiB");
  // eleven equal vectors of M complex FP32 values (ten read, one written) fill the buffer
  const size_t M = bytes / 11 / sizeof(f2v) / 1024 * 1024;
  f2v* v = (f2v*)buffer;
  f2v* w = v + 10 * M;
  float* sink = (float*)w;   // written only on NaN, which the zeroed buffer never produces
  HYDOT_HIP(hipMemsetAsync(buffer, 0, 11 * M * sizeof(f2v), stream));
  const double vb = (double)M * sizeof(f2v);
  double ms = 0.0;
  hydot_status s;
  s = time_ms([&] { hipLaunchKernelGGL((k_probe_stream<10, false>), dim3(kProbeGrid), dim3(kProbeBlock), 0, stream, v, w, M, sink); },
              stream, &ms);
  if (s != HYDOT_OK) return s;
  out->read_GBps = 10.0 * vb / (ms * 1e-3) / 1e9;
  s = time_ms([&] { hipLaunchKernelGGL((k_probe_stream<1, true>), dim3(kProbeGrid), dim3(kProbeBlock), 0, stream, v, w, M, sink); },
              stream, &ms);
  if (s != HYDOT_OK) return s;
  out->copy_GBps = 2.0 * vb / (ms * 1e-3) / 1e9;
  s = time_ms([&] { hipLaunchKernelGGL((k_probe_stream<10, true>), dim3(kProbeGrid), dim3(kProbeBlock), 0, stream, v, w, M, sink); },
              stream, &ms);
  if (s != HYDOT_OK) return s;
  out->read10_write1_GBps = 11.0 * vb / (ms * 1e-3) / 1e9;
  hipDeviceProp_t prop;
  int dev = 0;
  HYDOT_HIP(hipGetDevice(&dev));
  HYDOT_HIP(hipGetDeviceProperties(&prop, dev));
  const int blocks = prop.multiProcessorCount * 8;   // 8 blocks of 4 waves per CU: 8 waves per SIMD
  const int iters = 4000;
  s = time_ms([&] { hipLaunchKernelGGL(k_probe_mfma_f32, dim3(blocks), dim3(kProbeBlock), 0, stream, iters, sink); },
              stream, &ms);
  if (s != HYDOT_OK) return s;
  out->mfma_f32_TFLOPs = (double)blocks * 4 * iters * 4 * (32.0 * 32 * 2 * 2) / (ms * 1e-3) / 1e12;
  s = time_ms([&] { hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(blocks), dim3(kProbeBlock), 0, stream, iters, sink); },
              stream, &ms);
  if (s != HYDOT_OK) return s;
  out->mfma_bf16_TFLOPs = (double)blocks * 4 * iters * 4 * (16.0 * 16 * 32 * 2) / (ms * 1e-3) / 1e12;
  out->compute_units = prop.multiProcessorCount;
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}
