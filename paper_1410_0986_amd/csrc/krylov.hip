// Host driver of the field solver: Algorithm 1 (augmented GMRES for
// parametric systems, Sec. 3.1) batched over right-hand sides and wavelengths,
// restarted with a fixed per-wavelength deflation space, with FP64 residual
// refinement around FP64 or FP32 inner solves.
#include <algorithm>
#include <cmath>
#include <complex>
#include <type_traits>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "krylov_kernels.h"
#include "krylov_tiled.h"
#include "lanczos.h"
#include "lanczos_tiled.h"
#include "precond.h"
#include "operator.h"
#include "small_dense.h"

namespace hydot {

// The small per-right-hand-side and per-system algebra of the set-up (harmonic Ritz pairs,
// Gram Cholesky factors, multi-shift least squares) is independent between systems: it runs
// on up to kHostThreads host threads while the GPU waits for it.  f(i) returns false on
// failure (an exception thrown by f counts as one); the result is the lowest failing index,
// or -1.
constexpr int kHostThreads = 16;
template <typename F>
int host_parallel_for(int n, const F& f) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({n, kHostThreads, hw});
  std::vector<int> bad(std::max(nt, 1), -1);
  auto safe = [&](int i) {
    try {
      return f(i);
    } catch (...) {
      return false;
    }
  };
  auto work = [&](int t) {
    for (int i = t; i < n; i += nt)
      if (!safe(i)) {
        bad[t] = i;
        return;
      }
  };
  if (nt <= 1) {
    for (int i = 0; i < n; ++i)
      if (!safe(i)) return i;
    return -1;
  }
  std::vector<std::thread> th;
  std::vector<char> started(nt, 0);
  for (int t = 1; t < nt; ++t) {
    try {
      th.emplace_back(work, t);
      started[t] = 1;
    } catch (...) {   // no thread available: that share runs on the calling thread
    }
  }
  work(0);
  for (int t = 1; t < nt; ++t)
    if (!started[t]) work(t);
  for (std::thread& x : th) x.join();
  int first = -1;
  for (int b : bad)
    if (b >= 0 && (first < 0 || b < first)) first = b;
  return first;
}

// Per-system blocks uploaded contiguously ([nb][len]) into each system's small block at
// offset `at`: one host copy instead of one row per system.
__global__ void k_put_small(cd* small, int total, int at, const cd* src, int len, int nb) {
  const int sys = blockIdx.y;
  if (sys >= nb) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x)
    small[(size_t)sys * total + at + e] = src[(size_t)sys * len + e];
}

// Shift-invariant basis -> U (from V_n) and C (from V_{n+1}) for each right-hand side:
// U[r][i] = sum_l VL[r][l] cu[r][l][i], C[r][i] = sum_l VL[r][l] cu[r][l][k+i].
template <int KM, typename VT>
__global__ __launch_bounds__(kBlock) void k_combine_uc(GridP g, const VT* VL, int vldim, int nl1,
                                                      const double* ucoef, int k, double* U64, double* C64,
                                                      float* U32, float* C32, int rhs_off) {
  const int r = blockIdx.y;
  const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= (uint32_t)g.N) return;
  const size_t N = (size_t)g.N;
  const VT* Vb = VL + (size_t)r * vldim * N;
  const double* cf = ucoef + (size_t)r * nl1 * 2 * k;
  double acc[2 * KM];
#pragma unroll
  for (int i = 0; i < 2 * KM; ++i) acc[i] = 0.0;
  for (int l = 0; l < nl1; ++l) {
    const double v = (double)Vb[(size_t)l * N + n];
#pragma unroll
    for (int i = 0; i < 2 * KM; ++i)
      if (i < 2 * k) acc[i] += v * cf[l * 2 * k + i];
  }
  const size_t rr = (size_t)(r + rhs_off);
  for (int i = 0; i < k; ++i) {
    U64[(rr * k + i) * N + n] = acc[i];
    C64[(rr * k + i) * N + n] = acc[k + i];
    if (U32) {
      U32[(rr * k + i) * N + n] = (float)acc[i];
      C32[(rr * k + i) * N + n] = (float)acc[k + i];
    }
  }
}

// Partial Gram sums of X = [C_0..C_{k-1}, U_0.., rho U_0..] per (chunk, rhs):
// out[r][chunk][p] for pairs p = (a <= b) in row-major upper-triangle order.
// Gram of [C, U, rho U] (ng = 3) or [C, U, rho U, mu U] (ng = 4, absorption perturbation mu)
__global__ __launch_bounds__(kBlock) void k_gram(GridP g, const double* U64, const double* C64, int k, int ng,
                                                const double* mu, int rhs_off, double* part, int nchunks) {
  const int r = blockIdx.y + rhs_off;
  const int chunk = blockIdx.x;
  const size_t N = (size_t)g.N;
  const int m = ng * k;
  const int npairs = m * (m + 1) / 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t base = chunk * kChunk;
  double* out = part + ((size_t)blockIdx.y * nchunks + chunk) * npairs;
  for (int p = wave; p < npairs; p += kWaves) {
    // decode p -> (a, b), a <= b
    int a = 0, rem = p;
    while (rem >= m - a) { rem -= m - a; ++a; }
    const int b = a + rem;
    double acc = 0.0;
    for (int q = lane; q < kChunk; q += 64) {
      const uint32_t n = base + q;
      if (n >= (uint32_t)g.N) break;
      double va, vb;
      {
        const int t = a / k, i = a % k;
        const double* src = t == 0 ? C64 : U64;
        va = src[((size_t)r * k + i) * N + n];
        if (t == 2) va *= (double)voxel_info(g, n).nrobin * g.inv_h;
        if (t == 3) va *= mu[n];
      }
      {
        const int t = b / k, i = b % k;
        const double* src = t == 0 ? C64 : U64;
        vb = src[((size_t)r * k + i) * N + n];
        if (t == 2) vb *= (double)voxel_info(g, n).nrobin * g.inv_h;
        if (t == 3) vb *= mu[n];
      }
      acc += va * vb;
    }
    acc = wave_sum(acc);
    if (lane == 0) out[p] = acc;
  }
}

__global__ void k_gram_reduce(const double* part, int nchunks, int npairs, int nr, double* gram) {
  const int r = blockIdx.x;
  for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < nchunks; ++c) a += part[((size_t)r * nchunks + c) * npairs + p];
    gram[(size_t)r * npairs + p] = a;
  }
}

namespace {

// ------------------------------------------------------------ measurement
// Optional per-kernel timing of the Arnoldi step kernels with HIP events on the
// solve stream, plus their algorithmic bytes (unique data each launch must move
// for the systems it actually processes).
struct ProfRec {
  const char* name;
  int64_t launches;
  double ms;
  double bytes;
};
bool g_prof = false;
// block-order flags of tile_map for a launch shape (step_order 1, 3, 4 -> bits 0, 1, 2; 2: none)
inline int step_flags(const hydot_tuning& tu) {
  return tu.step_order == 1 ? 1 : tu.step_order == 3 ? 2 : tu.step_order == 4 ? 4 : 0;
}

ProfRec g_rec[3] = {{"k_step_dots", 0, 0.0, 0.0}, {"k_step_update", 0, 0.0, 0.0}, {"k_step_finish", 0, 0.0, 0.0}};
const char* kTiledNames[3] = {"k_step_dots_t", "k_step_update_t", "k_step_finish_t"};
const char* kGenericNames[3] = {"k_step_dots", "k_step_update", "k_step_finish"};
const char* kPairNames[3] = {"k_step_pair_t<dots>", "k_step_pair_t<update>", "k_step_finish_t"};

struct Plan {
  int R, L, N;
  int k, mk, nl, mkmax;
  int prec;
  bool recycle, per_system, graph, mean_shift;
  int shift_kind;   // sigma' moved into K_hat: 0 mean, 1 min, 2 max (when mean_shift)
  int nb;       // systems per batch
  int rl;       // right-hand sides per Lanczos batch (and in the U/C buffers)
  int nchunks, ndots;
  int npairs;
  int ng;       // Gram vector blocks: 3 ([C, U, rho U]) or 4 (+ mu U with an absorption perturbation)
  int precond;  // 0 none, 1 separable P_j = K_hat + sigma_j I, 2 one shift (the mean sigma) for all
  Small sl;
  size_t esz;   // inner storage bytes per complex
  // byte offsets
  size_t o_prm, o_st, o_VL, o_U64, o_C64, o_U32, o_C32, o_gpart, o_gram, o_ucoef;
  size_t o_V, o_W, o_Din, o_Rin, o_X, o_Rout, o_part, o_small, o_lcy, o_cnt, o_final, o_Z, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

hydot_status make_plan(const hydot_operator* op, int n_rhs, const hydot_solve_opts* o, Plan& p) {
  if (!op) return fail(HYDOT_EINVAL, "solve: null operator");
  if (!o) return fail(HYDOT_EINVAL, "solve: null options");
  if (n_rhs < 1) return fail(HYDOT_EINVAL, "solve: n_rhs must be >= 1");
  if (!(o->rel_tol > 0.0) || !std::isfinite(o->rel_tol)) return fail(HYDOT_EINVAL, "solve: rel_tol must be > 0");
  if (o->max_iter < 1) return fail(HYDOT_EINVAL, "solve: max_iter must be >= 1");
  if (o->precision != HYDOT_PREC_FP64 && o->precision != HYDOT_PREC_MIXED)
    return fail(HYDOT_EINVAL, "solve: precision must be HYDOT_PREC_FP64 or HYDOT_PREC_MIXED");
  if (o->flags & ~0x1FFu) return fail(HYDOT_EINVAL, "solve: unknown flag bits");
  if ((o->flags & HYDOT_FLAG_PRECOND_SEP) && (o->flags & HYDOT_FLAG_PRECOND_SEP_FIXED))
    return fail(HYDOT_EINVAL, "solve: at most one of PRECOND_SEP, PRECOND_SEP_FIXED");
  {
    const uint32_t sh = o->flags & (HYDOT_FLAG_MEAN_SHIFT | HYDOT_FLAG_SHIFT_MIN | HYDOT_FLAG_SHIFT_MAX);
    if (sh & (sh - 1)) return fail(HYDOT_EINVAL, "solve: at most one of MEAN_SHIFT, SHIFT_MIN, SHIFT_MAX");
  }
  p.recycle = !(o->flags & HYDOT_FLAG_NO_RECYCLE);
  p.k = p.recycle ? o->recycle_k : 0;
  if (p.k < 0 || p.k > kMaxK) return fail(HYDOT_EINVAL, "solve: recycle_k must be in [0, 32]");
  p.mk = o->restart_m - p.k;
  if (p.mk < 1 || p.mk > kMaxMK) return fail(HYDOT_EINVAL, "solve: restart_m - recycle_k must be in [1, 128]");
  p.nl = p.recycle ? o->lanczos_n : 0;
  if (p.recycle && (p.nl < 1 || p.nl > kMaxMK)) return fail(HYDOT_EINVAL, "solve: lanczos_n must be in [1, 128]");
  if (p.recycle && p.k >= p.nl) return fail(HYDOT_EINVAL, "solve: recycle_k must be < lanczos_n");
  if (o->precision == HYDOT_PREC_MIXED && !(o->inner_tol > 0.0 && o->inner_tol < 1.0))
    return fail(HYDOT_EINVAL, "solve: inner_tol must be in (0, 1) for the mixed path");
  if (o->max_batch < 0) return fail(HYDOT_EINVAL, "solve: max_batch must be >= 0");
  p.R = n_rhs;
  p.L = op->L;
  p.N = op->gp.N;
  if ((int64_t)p.R * p.L > 1 << 24) return fail(HYDOT_EINVAL, "solve: too many systems");
  p.prec = o->precision;
  p.per_system = (o->flags & HYDOT_FLAG_PER_SYSTEM) != 0;
  p.graph = (o->flags & HYDOT_FLAG_GRAPH) != 0;
  p.mean_shift = (o->flags & (HYDOT_FLAG_MEAN_SHIFT | HYDOT_FLAG_SHIFT_MIN | HYDOT_FLAG_SHIFT_MAX)) != 0;
  p.shift_kind = (o->flags & HYDOT_FLAG_SHIFT_MIN) ? 1 : (o->flags & HYDOT_FLAG_SHIFT_MAX) ? 2 : 0;
  p.mkmax = std::max(p.mk, p.nl);
  // the FP32 step kernels address each system's basis and each right-hand side's C and U
  // through buffer resources of 32-bit byte offsets
  if (o->precision == HYDOT_PREC_MIXED &&
      ((uint64_t)(p.mk + 1) * (uint64_t)p.N * 8u >= (1ull << 31) || (uint64_t)p.k * (uint64_t)p.N * 4u >= (1ull << 31)))
    return fail(HYDOT_EUNSUPPORTED, "solve: a system's Krylov basis or a right-hand side's C or U block would "
                                    "exceed 2 GiB; lower restart_m or recycle_k");
  p.precond = (o->flags & HYDOT_FLAG_PRECOND_SEP) ? 1 : (o->flags & HYDOT_FLAG_PRECOND_SEP_FIXED) ? 2 : 0;
  if (p.precond) {
    // right preconditioning lives in the register-resident FP32 step kernels only
    if (o->precision != HYDOT_PREC_MIXED)
      return fail(HYDOT_EUNSUPPORTED, "solve: the preconditioner needs the mixed-precision path");
    if (p.k > kTK || p.mk > kTNV)
      return fail(HYDOT_EUNSUPPORTED, "solve: the preconditioner needs recycle_k <= 10 and restart_m - recycle_k <= 32");
    if (op->gp.nx > kPrecMaxN || op->gp.ny > kPrecMaxN || op->gp.nz > kPrecMaxN)
      return fail(HYDOT_EUNSUPPORTED, "solve: the preconditioner needs grid axes of at most 256 cells");
  }
  const int total_sys = p.R * p.L;
  if (p.per_system) {
    p.nb = 1;
    p.rl = 1;
  } else {
    p.nb = o->max_batch > 0 ? std::min(o->max_batch, total_sys) : total_sys;
    p.rl = p.R;
  }
  if (p.nb > 65535 || p.rl > 65535) return fail(HYDOT_EINVAL, "solve: batch above 65535 systems; set max_batch");
  p.nchunks = (p.N + kChunk - 1) / kChunk;
  p.ndots = ndots_for(p.k, p.mkmax);
  p.ng = op->has_pert ? 4 : 3;
  p.npairs = p.ng * p.k * (p.ng * p.k + 1) / 2;
  p.sl = make_small(p.k, p.mkmax, p.nl);
  p.esz = p.prec == HYDOT_PREC_FP64 ? sizeof(cd) : sizeof(cf);
  const size_t N = (size_t)p.N;
  const int ns = std::max(p.nb, p.rl);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
  p.o_prm = take((size_t)ns * sizeof(SysParam));
  p.o_st = take((size_t)ns * sizeof(SysState));
  // real Lanczos basis: FP32 for the mixed path, FP64 for the FP64 path
  p.o_VL = take(p.recycle ? (size_t)p.rl * (p.nl + 1) * N * (p.prec == HYDOT_PREC_MIXED ? sizeof(float) : sizeof(double)) : 0);
  const size_t ucount = (size_t)p.rl * p.k * N;
  p.o_U64 = take(ucount * sizeof(double));
  p.o_C64 = take(ucount * sizeof(double));
  p.o_U32 = take(p.prec == HYDOT_PREC_MIXED ? ucount * sizeof(float) : 0);
  p.o_C32 = take(p.prec == HYDOT_PREC_MIXED ? ucount * sizeof(float) : 0);
  p.o_gpart = take((size_t)p.rl * p.nchunks * p.npairs * sizeof(double));
  p.o_gram = take((size_t)p.rl * p.npairs * sizeof(double));
  p.o_ucoef = take((size_t)p.rl * (p.nl + 1) * 2 * p.k * sizeof(double));
  p.o_V = take((size_t)p.nb * (p.mk + 1) * N * p.esz);
  p.o_W = take(std::max((size_t)p.nb * p.esz, (size_t)p.rl * sizeof(cd)) * N);
  p.o_Din = take((size_t)p.nb * N * p.esz);
  p.o_Rin = take((size_t)p.nb * N * p.esz);
  p.o_X = take((size_t)p.nb * N * sizeof(cd));
  p.o_Rout = take((size_t)p.nb * N * sizeof(cd));
  p.o_part = take((size_t)ns * p.nchunks * p.ndots * sizeof(cd));
  p.o_small = take((size_t)ns * p.sl.total * sizeof(cd));
  p.o_lcy = take((size_t)ns * (p.k * p.k + p.nl) * sizeof(cd));   // staging of the per-system set-up
  p.o_cnt = take(kCounters * sizeof(int));
  p.o_final = take((size_t)ns * sizeof(double));
  p.o_Z = take(p.precond ? (size_t)p.nb * N * sizeof(cf) : 0);
  p.total = off;
  return HYDOT_OK;
}

// host-side per-right-hand-side set-up data
struct RhsSetup {
  std::vector<double> Hbar;   // (nl+1) x nl
  std::vector<double> gram;   // npairs
  std::vector<double> vs;     // scales of the stored Lanczos vectors: v_l = vs[l] * V_l (nl+1)
};

struct Solver {
  const hydot_operator* op;
  Plan p;
  char* ws;
  hipStream_t stream;
  const hydot_solve_opts* o;
  std::vector<RhsSetup> rs;   // per right-hand side (global index)
  const int64_t* rhs_vox;

  template <typename T> T* at(size_t off) const { return (T*)(ws + off); }

  // Robin shift moved into K_hat (Sec. 6.1): the mean, minimum or maximum of sigma'_j, or none
  double sigp_mean() const {
    if (!p.mean_shift) return 0.0;
    return p.shift_kind == 1 ? op->sigp_min : p.shift_kind == 2 ? op->sigp_max : op->sigp_mean;
  }
  // part of the absorption perturbation moved into K_hat (its mean, with the mean shift)
  double tau_shift() const { return p.mean_shift && op->has_pert ? op->tau_mean : 0.0; }

  template <typename S>
  Ctx<S> ctx(int k, bool lanczos) const {
    Ctx<S> c{};
    c.g = op->gp;
    c.k = k;
    c.mkmax = p.mkmax;
    c.nchunks = p.nchunks;
    c.prm = at<SysParam>(p.o_prm);
    c.st = at<SysState>(p.o_st);
    c.V = lanczos ? (S*)at<cd>(p.o_VL) : at<S>(p.o_V);
    c.vdim = lanczos ? p.nl + 1 : p.mk + 1;
    c.W = at<S>(p.o_W);
    c.Din = at<S>(p.o_Din);
    c.Rin = at<S>(p.o_Rin);
    c.X = at<cd>(p.o_X);
    c.Rout = at<cd>(p.o_Rout);
    using R = typename Store<S>::real;
    if (sizeof(R) == sizeof(double)) {
      c.C = (const R*)at<double>(p.o_C64);
      c.U = (const R*)at<double>(p.o_U64);
    } else {
      c.C = (const R*)at<float>(p.o_C32);
      c.U = (const R*)at<float>(p.o_U32);
    }
    c.mu = op->has_pert ? (sizeof(R) == sizeof(double) ? (const R*)op->mu64 : (const R*)op->mu32) : nullptr;
    c.part = at<cd>(p.o_part);
    c.ndots = p.ndots;
    c.small = at<cd>(p.o_small);
    c.sl = p.sl;
    c.counter = at<int>(p.o_cnt);
    if (p.precond && !lanczos && std::is_same<S, cf>::value) c.Z = at<S>(p.o_Z);
    return c;
  }

  hydot_status read_counters(int* h) {
    HYDOT_HIP(hipMemcpyAsync(h, at<int>(p.o_cnt), kCounters * sizeof(int), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    return HYDOT_OK;
  }

  // systems per block group of the tiled kernels (see krylov_tiled.h)
  int tile_grp = 1;
  // the batch holds whole right-hand sides with an even number of wavelengths, in order
  bool pair_ok = false;
  PrecP pc{};   // separable preconditioner (p.precond != 0)

  // P^{-1} applied to one vector per system: in (system stride in_stride) -> Z
  template <typename S>
  void precond_apply(const Ctx<S>& c, const S* in, size_t in_stride, int pred, int nb) {
    if constexpr (std::is_same<S, cf>::value) {
      PrecIO io{};
      io.in = in;
      io.out = c.Z;
      io.in_stride = in_stride;
      io.out_stride = (size_t)p.N;
      io.st = c.st;
      io.pred = pred;
      io.prm = c.prm;
      io.fixed = p.precond == 2 ? 1 : 0;
      io.sig_fixed = op->sigma_mean;
      prec_apply(pc, io, nb, stream);
    }
  }
  bool used_tiled = false;   // the last cycle ran the register-resident FP32 kernels
  bool used_pairs = false;   // ... in their two-system form

  // event pairs around the step kernels of one cycle (profiling only)
  std::vector<hipEvent_t> ev;
  hydot_status prof_events() {
    if (!ev.empty()) return HYDOT_OK;
    ev.resize(2 * 3 * kMaxMK, nullptr);
    for (auto& e : ev) HYDOT_HIP(hipEventCreate(&e));
    return HYDOT_OK;
  }
  void prof_free() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    ev.clear();
  }
  // accumulate the timings of the cycle just synchronised
  hydot_status prof_collect(const int* cnt, int k) {
    const double N = (double)p.N, b = (double)p.esz;
    for (int j = 0; j < p.mk; ++j) {
      // per system: the basis vectors read plus the vector written; per right-hand side: C, U
      const double act_k[3] = {(double)cnt[2 + j], (double)cnt[2 + j], (double)cnt[2 + kMaxMK + j]};
      const double rhs = (double)cnt[2 + 2 * kMaxMK + j];
      const double rhs_k[3] = {rhs, rhs, std::min(rhs, act_k[2])};
      // the register-resident instances for up to 16 basis vectors keep W out of HBM unless the
      // preconditioner is on (the update recomputes A V_j from the stencil)
      const bool w_free = used_tiled && !p.precond && j + 1 <= 16;
      const double extra[3] = {(double)(j + (w_free ? 1 : 2)), (double)(j + (w_free ? 2 : 3)), (double)(j + 3)};
      for (int kind = 0; kind < 3; ++kind) {
        if (kind == 2 && j + 1 >= p.mk) continue;   // no finish after the last step
        float ms = 0.f;
        HYDOT_HIP(hipEventElapsedTime(&ms, ev[2 * (3 * j + kind)], ev[2 * (3 * j + kind) + 1]));
        g_rec[kind].name = used_pairs ? kPairNames[kind] : used_tiled ? kTiledNames[kind] : kGenericNames[kind];
        g_rec[kind].launches += 1;
        g_rec[kind].ms += ms;
        g_rec[kind].bytes += (act_k[kind] * extra[kind] + rhs_k[kind] * k) * N * b;
      }
    }
    return HYDOT_OK;
  }

  // ---------------------------------------------------------------- Lanczos
  // nl steps of the real Lanczos process for the nr right-hand sides of the buffer
  template <typename T>
  void lanczos_run(const Ctx<cd>& c, const ReduceArgs& ra, int nr) {
    LzCtx<T> lc;
    lc.g = op->gp;
    lc.nchunks = p.nchunks;
    lc.vdim = p.nl + 1;
    lc.ndots = p.ndots;
    lc.sigp = sigp_mean();
    lc.tau = tau_shift();
    lc.mu = op->has_pert ? (sizeof(T) == sizeof(double) ? (const T*)op->mu64 : (const T*)op->mu32) : nullptr;
    lc.prm = c.prm;
    lc.st = c.st;
    lc.V = at<T>(p.o_VL);
    lc.W = at<T>(p.o_W);
    lc.part = c.part;
    lc.small = c.small;
    lc.sl = c.sl;
    lc.mkmax = p.mkmax;
    const dim3 gv(p.nchunks, nr);
    hipLaunchKernelGGL(k_lz_v0<T>, gv, dim3(kBlock), 0, stream, lc, c.small);
    // FP32 basis: chunk-accumulating kernels while the basis fits their registers and one buffer
    // resource (below 2 GiB per right-hand side); the generic kernels otherwise
    const bool tiled = std::is_same<T, float>::value && (size_t)lc.vdim * p.N * sizeof(float) < ((size_t)1 << 31);
    for (int j = 0; j < p.nl; ++j) {
      const int nv = j + 1;
      if constexpr (std::is_same<T, float>::value) {
        if (tiled && nv <= kLzTiledMax) lz_tiled(0, lc, j, gv);
        else hipLaunchKernelGGL(k_lz_dots<T>, gv, dim3(kBlock), 0, stream, lc, j);
      } else {
        hipLaunchKernelGGL(k_lz_dots<T>, gv, dim3(kBlock), 0, stream, lc, j);
      }
      hipLaunchKernelGGL(k_reduce<cd>, dim3(nr), dim3(64), 0, stream, c, ra, (int)PH_STEP_A, j);
      if constexpr (std::is_same<T, float>::value) {
        if (tiled && nv <= kLzTiledMax) lz_tiled(1, lc, j, gv);
        else hipLaunchKernelGGL(k_lz_update<T>, gv, dim3(kBlock), 0, stream, lc, j);
      } else {
        hipLaunchKernelGGL(k_lz_update<T>, gv, dim3(kBlock), 0, stream, lc, j);
      }
      hipLaunchKernelGGL(k_reduce<cd>, dim3(nr), dim3(64), 0, stream, c, ra, (int)PH_STEP_B, j);
      hipLaunchKernelGGL(k_lz_finish<T>, gv, dim3(kBlock), 0, stream, lc, j);
    }
  }
  // chunk-accumulating Lanczos launch (kind 0: dots, 1: update): the instance with exactly the
  // j + 1 basis vectors up to 16, the next multiple of 4 beyond
  void lz_tiled(int kind, const LzCtx<float>& lc, int j, dim3 gv) {
    const int nv = j + 1;
#define HYDOT_LZ_T(NV)                                                                            \
  case NV:                                                                                        \
    if (kind == 0) hipLaunchKernelGGL((k_lz_dots_t<NV>), gv, dim3(kTSub), 0, stream, lc, j);      \
    else hipLaunchKernelGGL((k_lz_update_t<NV>), gv, dim3(kTSub), 0, stream, lc, j);              \
    break;
    switch (nv <= 16 ? nv : (nv + 3) / 4 * 4) {
      HYDOT_LZ_T(1) HYDOT_LZ_T(2) HYDOT_LZ_T(3) HYDOT_LZ_T(4) HYDOT_LZ_T(5) HYDOT_LZ_T(6) HYDOT_LZ_T(7)
      HYDOT_LZ_T(8) HYDOT_LZ_T(9) HYDOT_LZ_T(10) HYDOT_LZ_T(11) HYDOT_LZ_T(12) HYDOT_LZ_T(13) HYDOT_LZ_T(14)
      HYDOT_LZ_T(15) HYDOT_LZ_T(16) HYDOT_LZ_T(20) HYDOT_LZ_T(24) HYDOT_LZ_T(28) HYDOT_LZ_T(32) HYDOT_LZ_T(36)
      HYDOT_LZ_T(40) HYDOT_LZ_T(44) HYDOT_LZ_T(48) HYDOT_LZ_T(52) HYDOT_LZ_T(56) HYDOT_LZ_T(60)
      default: break;
    }
#undef HYDOT_LZ_T
  }

  // Shift-invariant Krylov basis of K_hat for right-hand sides [r0, r0+nr) (Alg. 1 step 1),
  // then U, C (steps 2-4) and the Gram blocks used by the per-wavelength update (Sec. 3.2).
  hydot_status setup_rhs(int r0, int nr, int buf_off) {
    const size_t N = (size_t)p.N;
    const int nl = p.nl, k = p.k;
    std::vector<SysParam> prm(nr);
    std::vector<SysState> st(nr);
    for (int i = 0; i < nr; ++i) {
      SysParam& q = prm[i];
      std::memset(&q, 0, sizeof(q));
      q.sig = cd{0.0, 0.0};
      q.sigp_abs = sigp_mean();
      q.sigp_rel = 0.0;
      q.tau_abs = tau_shift();
      q.tau_rel = 0.0;
      q.rhs = i;
      q.voxel = (int32_t)rhs_vox[r0 + i];
      std::memset(&st[i], 0, sizeof(SysState));
      st[i].in_cycle = 1;
      st[i].cyc_ran = 1;
    }
    HYDOT_HIP(hipMemcpyAsync(at<SysParam>(p.o_prm), prm.data(), nr * sizeof(SysParam), hipMemcpyHostToDevice, stream));
    HYDOT_HIP(hipMemcpyAsync(at<SysState>(p.o_st), st.data(), nr * sizeof(SysState), hipMemcpyHostToDevice, stream));
    Ctx<cd> c = ctx<cd>(0, true);   // partials, coefficients and state for k_reduce
    ReduceArgs ra{};
    ra.mk = nl;
    ra.lanczos = 1;
    ra.max_iter = 1 << 30;
    // FP32 basis: the second Gram-Schmidt pass only where the first leaves a projection above
    // 1e-6 of the vector (C = V_{n+1} Q inherits the basis' orthogonality, so the bar is tighter
    // than the Arnoldi one); a skipped pass leaves V_{j+1} unnormalised with its scale recorded
    ra.cgs_tau = p.prec == HYDOT_PREC_MIXED && !(o->flags & HYDOT_FLAG_FULL_REORTH) ? 1e-6 : 0.0;
    if (p.prec == HYDOT_PREC_MIXED) lanczos_run<float>(c, ra, nr);
    else lanczos_run<double>(c, ra, nr);
    HYDOT_HIP(hipGetLastError());
    // Hessenberg matrices back to the host
    std::vector<cd> smalls((size_t)nr * p.sl.total);
    std::vector<SysState> st_out(nr);
    HYDOT_HIP(hipMemcpyAsync(smalls.data(), at<cd>(p.o_small), smalls.size() * sizeof(cd), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipMemcpyAsync(st_out.data(), at<SysState>(p.o_st), nr * sizeof(SysState), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    const int ldh = p.mkmax + 1;
    std::vector<double> ucoef((size_t)nr * (nl + 1) * 2 * k, 0.0);
    for (int i = 0; i < nr; ++i)
      if (st_out[i].nsteps < nl)
        return fail(HYDOT_EUNSUPPORTED, "solve: shift-invariant Krylov space exhausted before lanczos_n steps; lower lanczos_n");
    const int bad = host_parallel_for(nr, [&](int i) {
      RhsSetup& R = rs[r0 + i];
      R.Hbar.assign((size_t)(nl + 1) * nl, 0.0);
      const cd* H = smalls.data() + (size_t)i * p.sl.total + p.sl.H;
      for (int jj = 0; jj < nl; ++jj)
        for (int ii = 0; ii <= std::min(jj + 1, nl); ++ii) R.Hbar[ii + (size_t)(nl + 1) * jj] = H[ii + ldh * jj].re;
      const cd* vsc = smalls.data() + (size_t)i * p.sl.total + p.sl.vs;
      R.vs.resize((size_t)nl + 1);
      for (int l = 0; l <= nl; ++l) R.vs[l] = vsc[l].re;
      if (k == 0) return true;
      std::vector<double> Zk, th;
      if (!dense::harmonic_ritz(nl, k, R.Hbar, Zk, th)) return false;
      // P = Hbar Zk, thin QR P = Qs Y, U = V_n Zk Y^-1, C = V_{n+1} Qs  (Alg. 1 steps 3-4)
      std::vector<double> P((size_t)(nl + 1) * k, 0.0);
      for (int cc = 0; cc < k; ++cc)
        for (int rr = 0; rr <= nl; ++rr) {
          double s = 0.0;
          for (int q = 0; q < nl; ++q) s += R.Hbar[rr + (size_t)(nl + 1) * q] * Zk[q + (size_t)nl * cc];
          P[rr + (size_t)(nl + 1) * cc] = s;
        }
      std::vector<double> Qs, Y;
      dense::thin_qr(nl + 1, k, P, Qs, Y);
      std::vector<double> ZY((size_t)nl * k, 0.0);   // Zk Y^-1 (row-wise triangular solve)
      for (int rr = 0; rr < nl; ++rr)
        for (int cc = 0; cc < k; ++cc) {
          double s = Zk[rr + (size_t)nl * cc];
          for (int q = 0; q < cc; ++q) s -= ZY[rr + (size_t)nl * q] * Y[q + (size_t)k * cc];
          ZY[rr + (size_t)nl * cc] = s / Y[cc + (size_t)k * cc];
        }
      // coefficients of the stored vectors V_l (v_l = vs[l] V_l)
      double* uc = ucoef.data() + (size_t)i * (nl + 1) * 2 * k;
      for (int l = 0; l <= nl; ++l)
        for (int cc = 0; cc < k; ++cc) {
          uc[l * 2 * k + cc] = l < nl ? R.vs[l] * ZY[l + (size_t)nl * cc] : 0.0;
          uc[l * 2 * k + k + cc] = R.vs[l] * Qs[l + (size_t)(nl + 1) * cc];
        }
      return true;
    });
    if (bad >= 0) return fail(HYDOT_EDEVICE, "solve: projected operator not positive definite in harmonic-Ritz step");
    if (k == 0) return HYDOT_OK;
    HYDOT_HIP(hipMemcpyAsync(at<double>(p.o_ucoef), ucoef.data(), ucoef.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    dim3 gu((p.N + kBlock - 1) / kBlock, nr);
    const bool mixed = p.prec == HYDOT_PREC_MIXED;
    float* U32 = mixed ? at<float>(p.o_U32) : nullptr;
    float* C32 = mixed ? at<float>(p.o_C32) : nullptr;
#define HYDOT_UC(KM, VT)                                                                                      \
  hipLaunchKernelGGL((k_combine_uc<KM, VT>), gu, dim3(kBlock), 0, stream, op->gp, at<VT>(p.o_VL), nl + 1, nl + 1, \
                     at<double>(p.o_ucoef), k, at<double>(p.o_U64), at<double>(p.o_C64), U32, C32, buf_off)
#define HYDOT_UC_T(VT)                 \
  if (k <= 8) HYDOT_UC(8, VT);         \
  else if (k <= 16) HYDOT_UC(16, VT);  \
  else HYDOT_UC(32, VT);
    if (mixed) { HYDOT_UC_T(float) } else { HYDOT_UC_T(double) }
#undef HYDOT_UC_T
#undef HYDOT_UC
    hipLaunchKernelGGL(k_gram, dim3(p.nchunks, nr), dim3(kBlock), 0, stream, op->gp, at<double>(p.o_U64),
                       at<double>(p.o_C64), k, p.ng, (const double*)(op->has_pert ? op->mu64 : nullptr), buf_off, at<double>(p.o_gpart), p.nchunks);
    hipLaunchKernelGGL(k_gram_reduce, dim3(nr), dim3(256), 0, stream, at<double>(p.o_gpart), p.nchunks, p.npairs, nr,
                       at<double>(p.o_gram));
    HYDOT_HIP(hipGetLastError());
    std::vector<double> gram((size_t)nr * p.npairs);
    HYDOT_HIP(hipMemcpyAsync(gram.data(), at<double>(p.o_gram), gram.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < nr; ++i) rs[r0 + i].gram.assign(gram.begin() + (size_t)i * p.npairs, gram.begin() + (size_t)(i + 1) * p.npairs);
    return HYDOT_OK;
  }

  // Per-wavelength deflation basis (Alg. 1 steps 7-8 with the Gram update of Sec. 3.2):
  // G_j = C_j'^H C_j' from the Gram of [C, U, rho U] with weights (1, sigma, sigma'_rel);
  // returns its lower Cholesky factor (false if G_j is not positive definite).  Thread-safe.
  bool gram_factor(int r, cd sig, double sp, double tr, std::vector<dense::zc>& Lf) const {
    const int k = p.k, m = p.ng * k;
    const std::vector<double>& gm = rs[r].gram;
    auto gam = [&](int a, int b) -> double {
      if (a > b) std::swap(a, b);
      // row-major upper triangle index
      const int idx = a * m - a * (a - 1) / 2 + (b - a);
      return gm[idx];
    };
    // C' = C + sigma U + sigma'_rel (rho U) + tau_rel (mu U)
    const dense::zc w[4] = {dense::zc(1.0, 0.0), dense::zc(sig.re, sig.im), dense::zc(sp, 0.0), dense::zc(tr, 0.0)};
    std::vector<dense::zc> G((size_t)k * k);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) {
        dense::zc s(0.0, 0.0);
        for (int t = 0; t < p.ng; ++t)
          for (int u = 0; u < p.ng; ++u) s += std::conj(w[t]) * w[u] * gam(t * k + i, u * k + j);
        G[i + (size_t)k * j] = s;
      }
    return dense::chol_herm(k, G, Lf);
  }

  // ----------------------------------------------------------- one batch
  // Arnoldi step kernels: kind 0 = operator + first dots, 1 = CGS2 update + dots,
  // 2 = second projection + normalisation.  Complex FP32 storage with k <= 16 and
  // at most 32 basis vectors uses the LDS-tiled kernels; everything else the generic ones.
  template <typename S>
  void step_kernel(int kind, const Ctx<S>& c, int j, int nb) {
    dim3 gv(p.nchunks, nb);
    if constexpr (std::is_same<S, cf>::value) {
      if (c.k <= kTK && j + 1 <= kTNV) {
        used_tiled = true;
        const dim3 gt((unsigned)(nb * p.nchunks));
        const int grp = tile_grp;
        const hydot_tuning tu = resolved_tuning(op->tune, &op->gp);
        const int fl = step_flags(tu);
        const bool small = j + 1 <= 16;
        const bool plain = c.mu == nullptr && c.Z == nullptr;
        // the chunk-accumulating instances take x rows of at most one sub-tile
        const bool rows_fit = op->gp.nx <= kTSub;
#define HYDOT_STEP_T(KER, NV, P) hipLaunchKernelGGL((KER<NV, P, 1>), gt, dim3(kTSub), 0, stream, c, j, grp, fl)
// the chunk-accumulating instances come with exact deflation dimensions k = 5 and 10
// (k = 5 also without a perturbation or preconditioner, the plain instances)
#define HYDOT_STEP_T16(KER, NV)                                                                                 \
  if (c.k == 5 && plain) hipLaunchKernelGGL((KER<NV, 16, 1, 5, true>), gt, dim3(kTSub), 0, stream, c, j, grp, fl); \
  else if (c.k == 5) hipLaunchKernelGGL((KER<NV, 16, 1, 5>), gt, dim3(kTSub), 0, stream, c, j, grp, fl);      \
  else if (c.k == 10) hipLaunchKernelGGL((KER<NV, 16, 1, 10>), gt, dim3(kTSub), 0, stream, c, j, grp, fl);    \
  else HYDOT_STEP_T(KER, NV, 16);
#define HYDOT_STEP_P(KER, NV)                                                                           \
  if (tu.step_presum == 16 && NV <= 16 && rows_fit) { HYDOT_STEP_T16(KER, NV) }                         \
  else if (tu.step_presum == 4 && tu.step_vx == 2 && NV <= 16)                                          \
    hipLaunchKernelGGL((KER<NV, 4, (NV <= 16 ? 2 : 1)>), gt, dim3(kTSub), 0, stream, c, j, grp, fl);   \
  else if (tu.step_presum == 4 || tu.step_presum == 16) HYDOT_STEP_T(KER, NV, 4);                       \
  else if (tu.step_presum == 2) HYDOT_STEP_T(KER, NV, 2);                                               \
  else HYDOT_STEP_T(KER, NV, 1);
// exact basis-count instances for j + 1 <= 16
#define HYDOT_STEP_NV(KER)                                                                               \
  switch (j + 1) {                                                                                       \
    case 1: { HYDOT_STEP_P(KER, 1) } break;   case 2: { HYDOT_STEP_P(KER, 2) } break;                     \
    case 3: { HYDOT_STEP_P(KER, 3) } break;   case 4: { HYDOT_STEP_P(KER, 4) } break;                     \
    case 5: { HYDOT_STEP_P(KER, 5) } break;   case 6: { HYDOT_STEP_P(KER, 6) } break;                     \
    case 7: { HYDOT_STEP_P(KER, 7) } break;   case 8: { HYDOT_STEP_P(KER, 8) } break;                     \
    case 9: { HYDOT_STEP_P(KER, 9) } break;   case 10: { HYDOT_STEP_P(KER, 10) } break;                   \
    case 11: { HYDOT_STEP_P(KER, 11) } break; case 12: { HYDOT_STEP_P(KER, 12) } break;                   \
    case 13: { HYDOT_STEP_P(KER, 13) } break; case 14: { HYDOT_STEP_P(KER, 14) } break;                   \
    case 15: { HYDOT_STEP_P(KER, 15) } break; default: { HYDOT_STEP_P(KER, 16) } break;                   \
  }
        // two systems per block where they are plain and share their right-hand side
        const bool pairs = kind != 2 && small && tu.step_pair == 2 && pair_ok && plain && rows_fit &&
                           tu.step_presum == 16;
        used_pairs = pairs;
        if (pairs) {
          const dim3 gp((unsigned)(nb / 2 * p.nchunks));
          const int pg = tile_grp > 1 ? tile_grp / 2 : 1;
#define HYDOT_PAIR(NV)                                                                                        \
  if (kind == 0) {                                                                                            \
    if (c.k == 5) hipLaunchKernelGGL((k_step_pair_t<NV, 0, 5>), gp, dim3(kTSub), 0, stream, c, j, pg, fl);     \
    else hipLaunchKernelGGL((k_step_pair_t<NV, 0, 0>), gp, dim3(kTSub), 0, stream, c, j, pg, fl);              \
  } else {                                                                                                    \
    if (c.k == 5) hipLaunchKernelGGL((k_step_pair_t<NV, 1, 5>), gp, dim3(kTSub), 0, stream, c, j, pg, fl);     \
    else hipLaunchKernelGGL((k_step_pair_t<NV, 1, 0>), gp, dim3(kTSub), 0, stream, c, j, pg, fl);              \
  }
          switch (j + 1) {
            case 1: { HYDOT_PAIR(1) } break;   case 2: { HYDOT_PAIR(2) } break;
            case 3: { HYDOT_PAIR(3) } break;   case 4: { HYDOT_PAIR(4) } break;
            case 5: { HYDOT_PAIR(5) } break;   case 6: { HYDOT_PAIR(6) } break;
            case 7: { HYDOT_PAIR(7) } break;   case 8: { HYDOT_PAIR(8) } break;
            case 9: { HYDOT_PAIR(9) } break;   case 10: { HYDOT_PAIR(10) } break;
            case 11: { HYDOT_PAIR(11) } break; case 12: { HYDOT_PAIR(12) } break;
            case 13: { HYDOT_PAIR(13) } break; case 14: { HYDOT_PAIR(14) } break;
            case 15: { HYDOT_PAIR(15) } break; default: { HYDOT_PAIR(16) } break;
          }
#undef HYDOT_PAIR
        } else if (kind == 0) {
          if (small) { HYDOT_STEP_NV(k_step_dots_t) } else { HYDOT_STEP_P(k_step_dots_t, 32) }
        } else if (kind == 1) {
          if (small) { HYDOT_STEP_NV(k_step_update_t) } else { HYDOT_STEP_P(k_step_update_t, 32) }
        } else {
          if (small) hipLaunchKernelGGL(k_step_finish_t<16>, gt, dim3(kTSub), 0, stream, c, j, grp, fl);
          else hipLaunchKernelGGL(k_step_finish_t<32>, gt, dim3(kTSub), 0, stream, c, j, grp, fl);
        }
#undef HYDOT_STEP_NV
#undef HYDOT_STEP_P
#undef HYDOT_STEP_T16
#undef HYDOT_STEP_T
        return;
      }
    }
    used_tiled = false;
    used_pairs = false;
    if (kind == 0) hipLaunchKernelGGL(k_step_dots<S>, gv, dim3(kBlock), 0, stream, c, j);
    else if (kind == 1) hipLaunchKernelGGL(k_step_update<S>, gv, dim3(kBlock), 0, stream, c, j);
    else hipLaunchKernelGGL(k_step_finish<S>, gv, dim3(kBlock), 0, stream, c, j);
  }

  // Cycle start (Alg. 1 step 9) with the register-resident FP32 kernels; false if the
  // generic kernels must run (FP64 storage or k above the tiled limit).
  template <typename S>
  bool cycle_start_tiled(const Ctx<S>& c, const ReduceArgs& ra, int nb) {
    if constexpr (std::is_same<S, cf>::value) {
      if (c.k > kTK) return false;
      const dim3 gt((unsigned)(nb * p.nchunks)), gr(nb);
      const hydot_tuning tu = resolved_tuning(op->tune, &op->gp);
      const int fl = step_flags(tu);
      const bool plain = c.mu == nullptr && c.Z == nullptr;
      // the chunk-accumulating form under the same conditions as the step kernels' (rows of at
      // most one sub-tile), with the same exact-k and plain instances
      if (tu.step_presum == 16 && op->gp.nx <= kTSub) {
        if (c.k == 5 && plain) hipLaunchKernelGGL((k_inner_resid_acc<5, true>), gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
        else if (c.k == 5) hipLaunchKernelGGL((k_inner_resid_acc<5, false>), gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
        else if (c.k == 10) hipLaunchKernelGGL((k_inner_resid_acc<10, false>), gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
        else hipLaunchKernelGGL((k_inner_resid_acc<0, false>), gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
      } else if (tu.step_presum == 4 || tu.step_presum == 16)
        hipLaunchKernelGGL(k_inner_resid_t<4>, gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
      else if (tu.step_presum == 2) hipLaunchKernelGGL(k_inner_resid_t<2>, gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
      else hipLaunchKernelGGL(k_inner_resid_t<1>, gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_START_A, 0);
      hipLaunchKernelGGL(k_defl_start_t, gt, dim3(kTSub), 0, stream, c, tile_grp, fl);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_START_B, 0);
      return true;
    }
    return false;
  }

  template <typename S>
  void launch_cycle(const Ctx<S>& c, const ReduceArgs& ra, int nb, bool prof) {
    dim3 gv(p.nchunks, nb), gr(nb);
    auto rec = [&](int j, int kind, int edge) {
      if (prof) (void)hipEventRecord(ev[2 * (3 * j + kind) + edge], stream);
    };
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, stream, c.counter);
    if (!cycle_start_tiled(c, ra, nb)) {
      hipLaunchKernelGGL(k_inner_resid<S>, gv, dim3(kBlock), 0, stream, c);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_START_A, 0);
      hipLaunchKernelGGL(k_defl_start<S>, gv, dim3(kBlock), 0, stream, c);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_START_B, 0);
    }
    for (int j = 0; j < p.mk; ++j) {
      if (c.Z) precond_apply<S>(c, c.V + (size_t)j * p.N, (size_t)c.vdim * p.N, 1, nb);   // Z = P^{-1} V_j
      rec(j, 0, 0);
      step_kernel<S>(0, c, j, nb);
      rec(j, 0, 1);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_STEP_A, j);
      rec(j, 1, 0);
      step_kernel<S>(1, c, j, nb);
      rec(j, 1, 1);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_STEP_B, j);
      if (j + 1 < p.mk) {
        rec(j, 2, 0);
        step_kernel<S>(2, c, j, nb);
        rec(j, 2, 1);
      }
    }
    hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_CYCLE_END, 0);
    if (c.Z) {   // Din += U z + P^{-1} (V y2)
      hipLaunchKernelGGL(k_cycle_vy<S>, gv, dim3(kBlock), 0, stream, c, c.Z);
      precond_apply<S>(c, c.Z, (size_t)p.N, 2, nb);
    }
    hipLaunchKernelGGL(k_cycle_update<S>, gv, dim3(kBlock), 0, stream, c);
  }

  template <typename S>
  hydot_status run_batch(const std::vector<int>& sys_r, const std::vector<int>& sys_l, int buf_rhs_base,
                         void* phi, hydot_dtype phi_dtype, std::vector<int32_t>& iters,
                         std::vector<double>& res) {
    const int nb = (int)sys_r.size();
    const size_t N = (size_t)p.N;
    const double h3 = op->grid.h_mm * op->grid.h_mm * op->grid.h_mm;
    std::vector<SysParam> prm(nb);
    std::vector<SysState> st(nb);
    const int lc_len = p.k * p.k + p.nl;
    std::vector<cd> lcy((size_t)nb * std::max(lc_len, 1), cd{0.0, 0.0});
    for (int i = 0; i < nb; ++i) {
      const int r = sys_r[i], l = sys_l[i];
      SysParam& q = prm[i];
      std::memset(&q, 0, sizeof(q));
      q.sig = op->sigma[l];
      q.sigp_abs = op->sigp[l];
      q.sigp_rel = op->sigp[l] - sigp_mean();
      q.tau_abs = op->has_pert ? op->tau[l] : 0.0;
      q.tau_rel = q.tau_abs - tau_shift();
      q.out_scale = 1.0 / (op->D[l] * h3);
      q.rhs = r - buf_rhs_base;
      q.voxel = (int32_t)rhs_vox[r];
      q.lam = l;
      q.gsys = l * p.R + r;
      std::memset(&st[i], 0, sizeof(SysState));
      st[i].in_sweep = 1;
    }
    // per system: Cholesky factor of G_j and the multi-shift initial-guess coefficients
    const int bad = host_parallel_for(nb, [&](int i) {
      const int r = sys_r[i];
      const SysParam& q = prm[i];
      cd* dst = lcy.data() + (size_t)i * lc_len;
      if (p.k > 0) {
        std::vector<dense::zc> Lf;
        if (!gram_factor(r, q.sig, q.sigp_rel, q.tau_rel, Lf)) return false;
        for (int t = 0; t < p.k * p.k; ++t) dst[t] = cd{Lf[t].real(), Lf[t].imag()};
      }
      if (p.nl > 0) {
        std::vector<dense::zc> y;
        dense::shifted_ls(p.nl, rs[r].Hbar, dense::zc(q.sig.re, q.sig.im), 1.0, y);
        // coefficients of the stored Lanczos vectors (v_l = vs[l] V_l)
        const std::vector<double>& vsc = rs[r].vs;
        for (int t = 0; t < p.nl; ++t) {
          const double sc = t < (int)vsc.size() ? vsc[t] : 1.0;
          dst[p.k * p.k + t] = cd{sc * y[t].real(), sc * y[t].imag()};
        }
      }
      return true;
    });
    if (bad >= 0) return fail(HYDOT_EDEVICE, "solve: per-wavelength deflation Gram matrix is not positive definite");
    HYDOT_HIP(hipMemcpyAsync(at<SysParam>(p.o_prm), prm.data(), nb * sizeof(SysParam), hipMemcpyHostToDevice, stream));
    HYDOT_HIP(hipMemcpyAsync(at<SysState>(p.o_st), st.data(), nb * sizeof(SysState), hipMemcpyHostToDevice, stream));
    if (lc_len > 0) {
      HYDOT_HIP(hipMemcpyAsync(at<cd>(p.o_lcy), lcy.data(), (size_t)nb * lc_len * sizeof(cd), hipMemcpyHostToDevice,
                               stream));
      hipLaunchKernelGGL(k_put_small, dim3((lc_len + 255) / 256, nb), dim3(256), 0, stream, at<cd>(p.o_small),
                         p.sl.total, p.sl.Lc, (const cd*)at<cd>(p.o_lcy), lc_len, nb);
    }
    Ctx<S> c = ctx<S>(p.k, false);
    Ctx<cd> c64 = ctx<cd>(p.k, false);   // FP64 views for residual and output kernels
    // group the wavelengths of one right-hand side when the batch holds whole ones
    tile_grp = 1;
    pair_ok = false;
    const hydot_tuning tg = resolved_tuning(op->tune, &op->gp);
    if (nb % p.L == 0) {
      bool aligned = true;
      for (int i = 0; i < nb && aligned; ++i) aligned = sys_l[i] == i % p.L && sys_r[i] == sys_r[i - i % p.L];
      if (aligned && (tg.step_group == 1 || tg.step_order == 4)) tile_grp = p.L;
      // systems 2i and 2i + 1 share a right-hand side (two-system step kernels)
      pair_ok = aligned && p.L % 2 == 0;
    }
    ReduceArgs ra{};
    ra.tol = o->rel_tol;
    ra.inner_floor = p.prec == HYDOT_PREC_MIXED ? o->inner_tol : 0.0;
    ra.max_iter = o->max_iter;
    ra.max_sweeps = p.prec == HYDOT_PREC_MIXED ? 40 : 20;
    ra.mk = p.mk;
    ra.lanczos = 0;
    ra.cgs_tau = p.prec == HYDOT_PREC_MIXED && !(o->flags & HYDOT_FLAG_FULL_REORTH) ? 1e-4 : 0.0;
    ra.final_res = at<double>(p.o_final);
    dim3 gv(p.nchunks, nb), gr(nb);
    if (p.nl > 0)
      hipLaunchKernelGGL((k_combine_x0<S, typename Store<S>::real>), gv, dim3(kBlock), 0, stream, c,
                         at<typename Store<S>::real>(p.o_VL), p.nl + 1, p.nl);
    else
      hipLaunchKernelGGL(k_zero_x<S>, gv, dim3(kBlock), 0, stream, c);
    HYDOT_HIP(hipGetLastError());

    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int cnt[kCounters] = {0};
    const bool prof = g_prof;
    if (prof) {
      hydot_status ps = prof_events();
      if (ps != HYDOT_OK) return ps;
    }
    const int max_cycles = o->max_iter / std::max(p.mk, 1) + 2;
    hydot_status status = HYDOT_OK;
    for (int sweep = 0; sweep < ra.max_sweeps + 2 && status == HYDOT_OK; ++sweep) {
      hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, stream, c.counter);
      hipLaunchKernelGGL(k_outer_resid<S>, gv, dim3(kBlock), 0, stream, c, 0);
      hipLaunchKernelGGL(k_reduce<S>, gr, dim3(64), 0, stream, c, ra, (int)PH_OUTER, 0);
      HYDOT_HIP(hipGetLastError());
      if ((status = read_counters(cnt)) != HYDOT_OK) break;
      if (cnt[0] == 0) break;
      hipLaunchKernelGGL(k_rhs_in<S>, gv, dim3(kBlock), 0, stream, c);
      for (int cyc = 0; cyc < max_cycles; ++cyc) {
        if (p.graph && !prof) {
          if (!gexec) {
            HYDOT_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            launch_cycle<S>(c, ra, nb, false);
            HYDOT_HIP(hipStreamEndCapture(stream, &graph));
            HYDOT_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
          }
          HYDOT_HIP(hipGraphLaunch(gexec, stream));
        } else {
          ReduceArgs rp = ra;
          rp.count_rhs = prof ? 1 : 0;
          launch_cycle<S>(c, rp, nb, prof);
        }
        HYDOT_HIP(hipGetLastError());
        if ((status = read_counters(cnt)) != HYDOT_OK) break;
        if (prof && (status = prof_collect(cnt, p.k)) != HYDOT_OK) break;
        if (cnt[1] == 0) break;
      }
      hipLaunchKernelGGL(k_outer_update<S>, gv, dim3(kBlock), 0, stream, c);
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (status != HYDOT_OK) return status;
    // output fields and the FP64 residual of the FP64 iterate
    if (phi_dtype == HYDOT_C128)
      hipLaunchKernelGGL((k_output<cd, cd>), gv, dim3(kBlock), 0, stream, c64, (cd*)phi);
    else if (phi_dtype == HYDOT_C64)
      hipLaunchKernelGGL((k_output<cd, cf>), gv, dim3(kBlock), 0, stream, c64, (cf*)phi);
    else
      hipLaunchKernelGGL((k_output<cd, cbf>), gv, dim3(kBlock), 0, stream, c64, (cbf*)phi);
    hipLaunchKernelGGL(k_outer_resid<cd>, gv, dim3(kBlock), 0, stream, c64, 1);
    hipLaunchKernelGGL(k_reduce<cd>, gr, dim3(64), 0, stream, c64, ra, (int)PH_FINAL, 0);
    HYDOT_HIP(hipGetLastError());
    std::vector<SysState> so(nb);
    std::vector<double> fr(nb);
    HYDOT_HIP(hipMemcpyAsync(so.data(), at<SysState>(p.o_st), nb * sizeof(SysState), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipMemcpyAsync(fr.data(), at<double>(p.o_final), nb * sizeof(double), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < nb; ++i) {
      const int g = prm[i].gsys;
      iters[g] = so[i].total_iters;
      res[g] = fr[i];
    }
    (void)N;
    return HYDOT_OK;
  }

  template <typename S>
  hydot_status solve_all(void* phi, hydot_dtype phi_dtype, std::vector<int32_t>& iters, std::vector<double>& res) {
    rs.assign(p.R, RhsSetup());
    if (p.per_system) {
      for (int r = 0; r < p.R; ++r) {
        if (p.recycle) {
          hydot_status s = setup_rhs(r, 1, 0);
          if (s != HYDOT_OK) return s;
        }
        for (int l = 0; l < p.L; ++l) {
          hydot_status s = run_batch<S>({r}, {l}, r, phi, phi_dtype, iters, res);
          if (s != HYDOT_OK) return s;
        }
      }
      return HYDOT_OK;
    }
    if (p.recycle) {
      hydot_status s = setup_rhs(0, p.R, 0);
      if (s != HYDOT_OK) return s;
    }
    // rhs-major system order; batches of nb
    const int total = p.R * p.L;
    for (int s0 = 0; s0 < total; s0 += p.nb) {
      const int nb = std::min(p.nb, total - s0);
      std::vector<int> sr(nb), sl(nb);
      for (int i = 0; i < nb; ++i) {
        sr[i] = (s0 + i) / p.L;
        sl[i] = (s0 + i) % p.L;
      }
      hydot_status s = run_batch<S>(sr, sl, 0, phi, phi_dtype, iters, res);
      if (s != HYDOT_OK) return s;
    }
    return HYDOT_OK;
  }
};

}  // namespace
}  // namespace hydot

using namespace hydot;

extern "C" {

hydot_status hydot_profile_enable(int32_t on) {
  g_prof = on != 0;
  if (g_prof)
    for (auto& r : g_rec) {
      r.launches = 0;
      r.ms = 0.0;
      r.bytes = 0.0;
    }
  return HYDOT_OK;
}

int32_t hydot_profile_read(hydot_kernel_profile* out, int32_t max_records) {
  const int n = 3;
  if (!out) return n;
  const int m = std::min(n, (int)max_records);
  for (int i = 0; i < m; ++i) {
    std::memset(&out[i], 0, sizeof(hydot_kernel_profile));
    std::strncpy(out[i].name, g_rec[i].name, sizeof(out[i].name) - 1);
    out[i].launches = g_rec[i].launches;
    out[i].total_ms = g_rec[i].ms;
    out[i].total_bytes = g_rec[i].bytes;
  }
  return m;
}

hydot_status hydot_solve_inspect(const hydot_operator* op, int32_t n_rhs, const hydot_solve_opts* opts,
                                 const void* workspace, size_t ws_bytes, int32_t what, int32_t index, void* out,
                                 size_t out_bytes, hydot_inspect_info* info, hipStream_t stream) {
  Plan p;
  hydot_status s = make_plan(op, n_rhs, opts, p);
  if (s != HYDOT_OK) return s;
  if (!workspace || ((uintptr_t)workspace & 255u)) return fail(HYDOT_EINVAL, "inspect: workspace must be 256-byte aligned");
  if (ws_bytes < p.total) return fail(HYDOT_ENOMEM, "inspect: workspace smaller than hydot_solve_workspace_bytes");
  if (!info) return fail(HYDOT_EINVAL, "inspect: null info");
  const char* ws = (const char*)workspace;
  const size_t N = (size_t)p.N;
  const int total = p.R * p.L;
  const int last_nb = total - p.nb * ((total - 1) / p.nb);   // systems of the last batch
  std::memset(info, 0, sizeof(*info));
  info->k = p.k;
  if (what == HYDOT_INSPECT_U || what == HYDOT_INSPECT_C) {
    if (!p.recycle || p.k == 0) return fail(HYDOT_EINVAL, "inspect: no deflation space (recycle_k = 0 or NO_RECYCLE)");
    if (index < 0 || index >= p.rl) return fail(HYDOT_EINVAL, "inspect: right-hand side index outside the last Lanczos batch");
    const size_t need = (size_t)p.k * N * sizeof(double);
    info->rhs = p.per_system ? p.R - 1 : index;
    info->lam = -1;
    if (!out) return HYDOT_OK;
    if (out_bytes < need) return fail(HYDOT_ENOMEM, "inspect: output buffer too small");
    const size_t off = (what == HYDOT_INSPECT_U ? p.o_U64 : p.o_C64) + (size_t)index * p.k * N * sizeof(double);
    HYDOT_HIP(hipMemcpyAsync(out, ws + off, need, hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    return HYDOT_OK;
  }
  if (what != HYDOT_INSPECT_CHOL && what != HYDOT_INSPECT_CYCLE) return fail(HYDOT_EINVAL, "inspect: unknown item");
  if (index < 0 || index >= last_nb) return fail(HYDOT_EINVAL, "inspect: system index outside the last batch");
  SysParam prm;
  SysState st;
  HYDOT_HIP(hipMemcpyAsync(&prm, ws + p.o_prm + (size_t)index * sizeof(SysParam), sizeof prm, hipMemcpyDeviceToHost, stream));
  HYDOT_HIP(hipMemcpyAsync(&st, ws + p.o_st + (size_t)index * sizeof(SysState), sizeof st, hipMemcpyDeviceToHost, stream));
  std::vector<cd> sm((size_t)p.sl.total);
  HYDOT_HIP(hipMemcpyAsync(sm.data(), ws + p.o_small + (size_t)index * p.sl.total * sizeof(cd), sm.size() * sizeof(cd),
                           hipMemcpyDeviceToHost, stream));
  HYDOT_HIP(hipStreamSynchronize(stream));
  info->rhs = p.per_system ? p.R - 1 : prm.rhs;
  info->lam = prm.lam;
  info->nsteps = st.nsteps;
  const int k = p.k, m = st.nsteps;
  if (what == HYDOT_INSPECT_CHOL) {
    if (k == 0) return fail(HYDOT_EINVAL, "inspect: no deflation space (recycle_k = 0 or NO_RECYCLE)");
    if (!out) return HYDOT_OK;
    if (out_bytes < (size_t)k * k * sizeof(cd)) return fail(HYDOT_ENOMEM, "inspect: output buffer too small");
    std::memcpy(out, sm.data() + p.sl.Lc, (size_t)k * k * sizeof(cd));
    return HYDOT_OK;
  }
  // last restart cycle: F' [k][m], the Hessenberg matrix with the Givens rotations undone
  // [(m+1) x m, column-major], the scaled basis v_0..v_{m-1} [m][N].  v_m is never formed: the
  // cycle's update needs only the first m vectors, so the last step skips its closing pass.
  const size_t need = ((size_t)k * m + (size_t)(m + 1) * m + (size_t)m * N) * sizeof(cd);
  if (!out) return HYDOT_OK;
  if (out_bytes < need) return fail(HYDOT_ENOMEM, "inspect: output buffer too small");
  cd* o = (cd*)out;
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < k; ++i) o[(size_t)i * m + j] = sm[small_Fp(p.sl, k, i, j)];
  cd* hb = o + (size_t)k * m;
  const double* cs = (const double*)(sm.data() + p.sl.cs);   // cosines in the .re slots
  const cd* sn = sm.data() + p.sl.sn;
  for (int j = 0; j < m; ++j) {
    std::vector<cd> col(m + 1, cd{0.0, 0.0});
    for (int i = 0; i <= j + 1; ++i) col[i] = sm[small_H(p.sl, p.mkmax, i, j)];
    // the rotations applied to column j were 0..j in order; undo them in reverse with the
    // adjoint of [[c, s], [-conj(s), c]]
    for (int i = j; i >= 0; --i) {
      const double c = cs[2 * i];
      const cd si = sn[i];
      const cd a = col[i], b = col[i + 1];
      col[i] = c * a - si * b;
      col[i + 1] = conj(si) * a + c * b;
    }
    for (int i = 0; i <= m; ++i) hb[i + (size_t)(m + 1) * j] = col[i];
  }
  cd* vb = hb + (size_t)(m + 1) * m;
  const char* V = ws + p.o_V + (size_t)index * (p.mk + 1) * N * p.esz;
  const cd* vs = sm.data() + p.sl.vs;
  if (p.prec == HYDOT_PREC_FP64) {
    HYDOT_HIP(hipMemcpyAsync(vb, V, (size_t)m * N * sizeof(cd), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
  } else {
    std::vector<cf> tmp((size_t)m * N);
    HYDOT_HIP(hipMemcpyAsync(tmp.data(), V, tmp.size() * sizeof(cf), hipMemcpyDeviceToHost, stream));
    HYDOT_HIP(hipStreamSynchronize(stream));
    for (size_t e = 0; e < tmp.size(); ++e) vb[e] = cd{(double)tmp[e].re, (double)tmp[e].im};
  }
  for (int l = 0; l < m; ++l) {
    const double sc = vs[l].re;
    for (size_t n = 0; n < N; ++n) vb[(size_t)l * N + n] = sc * vb[(size_t)l * N + n];
  }
  return HYDOT_OK;
}

hydot_status hydot_solve_workspace_bytes(const hydot_operator* op, int32_t n_rhs, const hydot_solve_opts* opts,
                                         size_t* bytes) {
  if (!bytes) return fail(HYDOT_EINVAL, "solve_workspace_bytes: null output");
  Plan p;
  hydot_status s = make_plan(op, n_rhs, opts, p);
  if (s != HYDOT_OK) return s;
  *bytes = p.total;
  return HYDOT_OK;
}

static hydot_status solve_fields_body(hydot_operator* op, int32_t n_rhs, const int64_t* rhs_voxel,
                                      const hydot_solve_opts* opts, void* phi, hydot_dtype phi_dtype,
                                      void* workspace, size_t ws_bytes, int32_t* iters, double* rel_res,
                                      hipStream_t stream) {
  Plan p;
  hydot_status s = make_plan(op, n_rhs, opts, p);
  if (s != HYDOT_OK) return s;
  if (!rhs_voxel || !phi || !workspace) return fail(HYDOT_EINVAL, "solve: null pointer argument");
  if (phi_dtype != HYDOT_C128 && phi_dtype != HYDOT_C64 && phi_dtype != HYDOT_CBF16)
    return fail(HYDOT_EUNSUPPORTED, "solve: phi_dtype must be C128, C64 or CBF16");
  if (((uintptr_t)workspace & 255u) != 0) return fail(HYDOT_EINVAL, "solve: workspace must be 256-byte aligned");
  if (ws_bytes < p.total) return fail(HYDOT_ENOMEM, "solve: workspace smaller than hydot_solve_workspace_bytes");
  for (int r = 0; r < n_rhs; ++r)
    if (rhs_voxel[r] < 0 || rhs_voxel[r] >= (int64_t)p.N) return fail(HYDOT_EINVAL, "solve: rhs voxel out of range");
  hipStream_t st = stream;
  bool own = false;
  if (p.graph && st == nullptr) {  // capture needs a non-legacy stream
    HYDOT_HIP(hipStreamCreate(&st));
    own = true;
  }
  Solver sv;
  sv.op = op;
  sv.p = p;
  sv.ws = (char*)workspace;
  sv.stream = st;
  sv.o = opts;
  sv.rhs_vox = rhs_voxel;
  if (p.precond) {
    s = prec_prepare(op, sv.sigp_mean(), sv.pc);
    if (s != HYDOT_OK) {
      if (own) (void)hipStreamDestroy(st);
      return s;
    }
  }
  std::vector<int32_t> it((size_t)p.R * p.L, 0);
  std::vector<double> rr((size_t)p.R * p.L, 0.0);
  if (p.prec == HYDOT_PREC_FP64)
    s = sv.solve_all<cd>(phi, phi_dtype, it, rr);
  else
    s = sv.solve_all<cf>(phi, phi_dtype, it, rr);
  sv.prof_free();
  if (own) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (s != HYDOT_OK) return s;
  bool all = true;
  for (size_t i = 0; i < rr.size(); ++i)
    if (!(rr[i] <= opts->rel_tol)) all = false;
  if (iters) std::memcpy(iters, it.data(), it.size() * sizeof(int32_t));
  if (rel_res) std::memcpy(rel_res, rr.data(), rr.size() * sizeof(double));
  if (!all) return fail(HYDOT_ENOCONV, "solve: some systems did not reach rel_tol (see rel_res)");
  return HYDOT_OK;
}

hydot_status hydot_solve_fields(hydot_operator* op, int32_t n_rhs, const int64_t* rhs_voxel,
                                const hydot_solve_opts* opts, void* phi, hydot_dtype phi_dtype, void* workspace,
                                size_t ws_bytes, int32_t* iters, double* rel_res, hipStream_t stream) {
  // no C++ exception crosses the C boundary (host set-up allocates)
  try {
    return solve_fields_body(op, n_rhs, rhs_voxel, opts, phi, phi_dtype, workspace, ws_bytes, iters, rel_res,
                             stream);
  } catch (const std::bad_alloc&) {
    return fail(HYDOT_ENOMEM, "solve: host allocation failed");
  } catch (...) {
    return fail(HYDOT_EDEVICE, "solve: unexpected host error");
  }
}

static hydot_status solve_batch_body(int32_t n_problems, hydot_solve_problem* problems, hipStream_t stream) {
  if (n_problems < 1 || n_problems > HYDOT_SOLVE_BATCH_MAX)
    return fail(HYDOT_EINVAL, "solve_batch: n_problems must be in [1, HYDOT_SOLVE_BATCH_MAX]");
  if (!problems) return fail(HYDOT_EINVAL, "solve_batch: null problems");
  for (int i = 0; i < n_problems; ++i) {
    if (!problems[i].op) return fail(HYDOT_EINVAL, "solve_batch: null operator");
    for (int j = 0; j < i; ++j)
      if (problems[j].op == problems[i].op) return fail(HYDOT_EINVAL, "solve_batch: an operator appears twice");
  }
  const int n = n_problems;
  std::vector<hipStream_t> st(n, nullptr);
  std::vector<std::string> msg(n);
  std::vector<std::thread> th;
  std::vector<char> on_thread(n, 0);
  th.reserve(n);
  hipEvent_t fork = nullptr;
  auto release = [&]() {
    for (hipStream_t s : st)
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    if (fork) (void)hipEventDestroy(fork);
  };
  // fork: every problem's stream starts after the work already queued on the caller's stream
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, stream);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    e = hipStreamCreate(&st[i]);   // default priority
    if (e == hipSuccess) e = hipStreamWaitEvent(st[i], fork, 0);
  }
  if (e != hipSuccess) {
    release();
    return hip_check(e, "solve_batch: stream set-up");
  }
  auto run = [&](int i) noexcept {
    hydot_solve_problem& q = problems[i];
    q.status = hydot_solve_fields(q.op, q.n_rhs, q.rhs_voxel, q.opts, q.phi, q.phi_dtype, q.workspace, q.ws_bytes,
                                  q.iters, q.rel_res, st[i]);
    // the fields and residuals of this problem are final once its stream has drained
    const hipError_t se = hipStreamSynchronize(st[i]);
    try {
      if (q.status != HYDOT_OK) msg[i] = hydot_last_error();   // the message is per thread
      if (se != hipSuccess && q.status >= 0) {
        q.status = HYDOT_EDEVICE;
        msg[i] = std::string("stream synchronize: ") + hipGetErrorString(se);
      }
    } catch (...) {   // no memory for the message: the status still reports the failure
      if (se != hipSuccess && q.status >= 0) q.status = HYDOT_EDEVICE;
    }
  };
  // the profiler's counters are process-wide: with it on, the problems run one after another
  if (!g_prof) {
    for (int i = 1; i < n; ++i) {
      try {
        th.emplace_back(run, i);
        on_thread[i] = 1;
      } catch (...) {   // no thread available: that problem runs on the calling thread
      }
    }
  }
  run(0);
  for (int i = 1; i < n; ++i)
    if (!on_thread[i]) run(i);
  for (std::thread& x : th) x.join();
  release();
  int first_err = -1;
  bool noconv = false;
  for (int i = 0; i < n; ++i) {
    if (problems[i].status < 0 && first_err < 0) first_err = i;
    if (problems[i].status == HYDOT_ENOCONV) noconv = true;
  }
  if (first_err >= 0)
    return fail(problems[first_err].status,
                "solve_batch: problem " + std::to_string(first_err) + ": " + msg[first_err]);
  if (noconv) {
    for (int i = 0; i < n; ++i)
      if (problems[i].status == HYDOT_ENOCONV)
        return fail(HYDOT_ENOCONV, "solve_batch: problem " + std::to_string(i) + ": " + msg[i]);
  }
  return HYDOT_OK;
}

hydot_status hydot_solve_fields_batch(int32_t n_problems, hydot_solve_problem* problems, hipStream_t stream) {
  try {   // host allocations before the problems start; every thread is joined before anything else throws
    return solve_batch_body(n_problems, problems, stream);
  } catch (const std::bad_alloc&) {
    return fail(HYDOT_ENOMEM, "solve_batch: host allocation failed");
  } catch (...) {
    return fail(HYDOT_EDEVICE, "solve_batch: unexpected host error");
  }
}

hydot_status hydot_autotune_solve(hydot_operator* op, int32_t n_rhs, const int64_t* rhs_voxel,
                                  const hydot_solve_opts* opts, void* phi, hydot_dtype phi_dtype, void* workspace,
                                  size_t ws_bytes, hydot_tune_trial* trials, int32_t max_trials, int32_t* n_trials,
                                  hipStream_t stream) {
  if (!op || !opts) return fail(HYDOT_EINVAL, "autotune_solve: null argument");
  if (max_trials < 0 || (max_trials > 0 && !trials)) return fail(HYDOT_EINVAL, "autotune_solve: bad trials buffer");
  // each trial is the caller's whole solve: systems converge and drop out over the cycles,
  // which changes which launch shape is fastest (a short sample does not show it)
  const hydot_solve_opts o = *opts;
  const hydot_tuning keep = op->tune;
  const bool prof_keep = g_prof;
  const ProfRec rec_keep[3] = {g_rec[0], g_rec[1], g_rec[2]};
  // candidates in order of preference (library default first); a later candidate replaces the
  // best only when it is more than 1% faster, so timing noise keeps the earlier choice
  const int presums[4] = {16, 4, 2, 4}, vxs[4] = {1, 1, 1, 2};
  int count = 0;
  double best = 1e300;
  hydot_tuning best_t = resolved_tuning(keep, &op->gp);
  hydot_status err = HYDOT_OK;
  // the grid's default block order, then the plain order (the z-slab order where that is 2)
  const int def_order = best_t.step_order;
  const int orders[2] = {def_order, def_order == 2 ? 3 : 2};
  for (int ig = 2; ig >= 1 && err == HYDOT_OK; --ig)
    for (int io = 0; io < 2 && err == HYDOT_OK; ++io)
      for (int ip = 0; ip < 4 && err == HYDOT_OK; ++ip) {
        hydot_tuning t = resolved_tuning(keep, &op->gp);
        t.step_presum = presums[ip];
        t.step_vx = vxs[ip];
        t.step_order = orders[io];
        t.step_group = ig;
        op->tune = t;
        (void)hydot_profile_enable(1);
        hydot_status s = hydot_solve_fields(op, n_rhs, rhs_voxel, &o, phi, phi_dtype, workspace, ws_bytes, nullptr,
                                            nullptr, stream);
        if (s < 0) {
          err = s;
          break;
        }
        double ms = 0.0;
        for (auto& r : g_rec) ms += r.ms;
        if (count < max_trials) trials[count] = hydot_tune_trial{t, ms};
        ++count;
        if (ms < 0.99 * best) {
          best = ms;
          best_t = t;
        }
      }
  g_prof = prof_keep;
  for (int i = 0; i < 3; ++i) g_rec[i] = rec_keep[i];
  if (err != HYDOT_OK) {
    op->tune = keep;
    return err;
  }
  op->tune = best_t;
  if (n_trials) *n_trials = count;
  return HYDOT_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------------
// Separable preconditioner, host side: the eigen-decompositions of the three axis operators of
// K_hat (cached in the operator) and the stand-alone application hydot_apply_preconditioner.
namespace hydot {

namespace {

// T = (1/h^2) (path Laplacian with +2 per Dirichlet end) + (sigp_star / h) (Robin end indicator)
void axis_operator(int n, bool robin_lo, bool robin_hi, double inv_h2, double inv_h, double sigp_star,
                   std::vector<double>& T) {
  T.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double d = 0.0;
    if (i > 0) {
      d += 1.0;
      T[(size_t)i + (size_t)n * (i - 1)] = -inv_h2;
    }
    if (i < n - 1) {
      d += 1.0;
      T[(size_t)i + (size_t)n * (i + 1)] = -inv_h2;
    }
    double e = 0.0;
    if (i == 0) (robin_lo ? e : d) += robin_lo ? 1.0 : 2.0;
    if (i == n - 1) (robin_hi ? e : d) += robin_hi ? 1.0 : 2.0;
    T[(size_t)i * (n + 1)] = d * inv_h2 + e * sigp_star * inv_h;
  }
}

}  // namespace

hydot_status prec_prepare(const hydot_operator* op, double sigp_star, PrecP& pp) {
  const hydot::GridP& g = op->gp;
  const int dims[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a)
    if (dims[a] > kPrecMaxN) return fail(HYDOT_EUNSUPPORTED, "preconditioner: a grid axis is longer than 256");
  int n4[3];
  size_t off[3][3], total = 0;
  for (int a = 0; a < 3; ++a) {
    n4[a] = (dims[a] + 3) & ~3;
    off[a][0] = total;
    total += (size_t)dims[a] * n4[a];
    off[a][1] = total;
    total += (size_t)dims[a] * n4[a];
    off[a][2] = total;
    total += (size_t)n4[a];
  }
  if (!op->pc_valid || op->pc_sigp != sigp_star) {
    std::vector<float> host(total, 0.0f);
    for (int a = 0; a < 3; ++a) {
      const int n = dims[a];
      const bool rlo = (g.robin >> (2 * a)) & 1u, rhi = (g.robin >> (2 * a + 1)) & 1u;
      std::vector<double> T, w, Q;
      axis_operator(n, rlo, rhi, g.inv_h2, g.inv_h, sigp_star, T);
      dense::sym_eig(n, T, w, Q);   // Q column-major: Q[i + n * c] = component i of eigenvector c
      for (int c = 0; c < n; ++c) {
        host[off[a][2] + c] = (float)w[c];
        for (int i = 0; i < n; ++i) {
          const float q = (float)Q[(size_t)i + (size_t)n * c];
          host[off[a][0] + (size_t)i * n4[a] + c] = q;
          host[off[a][1] + (size_t)c * n4[a] + i] = q;
        }
      }
    }
    if (!op->pc_dev) HYDOT_HIP(hipMalloc(&op->pc_dev, total * sizeof(float)));
    HYDOT_HIP(hipMemcpy(op->pc_dev, host.data(), total * sizeof(float), hipMemcpyHostToDevice));
    op->pc_sigp = sigp_star;
    op->pc_valid = true;
  }
  pp.nx = g.nx;
  pp.ny = g.ny;
  pp.nz = g.nz;
  for (int a = 0; a < 3; ++a) {
    pp.ax[a].Qf = op->pc_dev + off[a][0];
    pp.ax[a].Qi = op->pc_dev + off[a][1];
    pp.ax[a].lam = op->pc_dev + off[a][2];
    pp.ax[a].n = dims[a];
    pp.ax[a].n4 = n4[a];
  }
  return HYDOT_OK;
}

}  // namespace hydot

using namespace hydot;

extern "C" {

hydot_status hydot_apply_preconditioner(const hydot_operator* op, uint32_t flags, int32_t lam_index, const void* x,
                                        void* y, int32_t count, hipStream_t stream) {
  if (!op) return fail(HYDOT_EINVAL, "apply_preconditioner: null operator");
  if (!x || !y) return fail(HYDOT_EINVAL, "apply_preconditioner: null vector");
  if (count < 1 || count > 65535) return fail(HYDOT_EINVAL, "apply_preconditioner: count must be in [1, 65535]");
  if (lam_index < 0 || lam_index >= op->L) return fail(HYDOT_EINVAL, "apply_preconditioner: lam_index out of range");
  const uint32_t pc = flags & (HYDOT_FLAG_PRECOND_SEP | HYDOT_FLAG_PRECOND_SEP_FIXED);
  const uint32_t sh = flags & (HYDOT_FLAG_MEAN_SHIFT | HYDOT_FLAG_SHIFT_MIN | HYDOT_FLAG_SHIFT_MAX);
  if (flags & ~(pc | sh)) return fail(HYDOT_EINVAL, "apply_preconditioner: flags other than PRECOND_* and shift flags");
  if (pc == 0 || (pc & (pc - 1))) return fail(HYDOT_EINVAL, "apply_preconditioner: exactly one PRECOND_* flag");
  if (sh & (sh - 1)) return fail(HYDOT_EINVAL, "apply_preconditioner: at most one shift flag");
  const double sigp_star = sh == HYDOT_FLAG_MEAN_SHIFT ? op->sigp_mean
                           : sh == HYDOT_FLAG_SHIFT_MIN ? op->sigp_min
                           : sh == HYDOT_FLAG_SHIFT_MAX ? op->sigp_max : 0.0;
  PrecP pp;
  hydot_status s = prec_prepare(op, sigp_star, pp);
  if (s != HYDOT_OK) return s;
  PrecIO io{};
  io.in = (const cf*)x;
  io.out = (cf*)y;
  io.in_stride = io.out_stride = (size_t)op->gp.N;
  io.st = nullptr;
  io.pred = 0;
  io.prm = nullptr;
  io.fixed = 1;
  io.sig_fixed = pc == HYDOT_FLAG_PRECOND_SEP ? op->sigma[lam_index] : op->sigma_mean;
  prec_apply(pp, io, count, stream);
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

}  // extern "C"
