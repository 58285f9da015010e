// Operator assembly (optical model of Sec. 2.1 and the shift form of
// eq. multipleshifted), error bookkeeping, and the matrix-free application of
// A(lambda) as its own entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "operator.h"
#include "krylov_index.h"

namespace hydot {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

hydot_status fail(hydot_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

hydot_status hip_check(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return HYDOT_EDEVICE;
}

GridP make_gridp(const hydot_grid& g) {
  GridP p;
  p.nx = g.nx;
  p.ny = g.ny;
  p.nz = g.nz;
  p.N = g.nx * g.ny * g.nz;
  p.dx = make_fastdiv((uint32_t)g.nx);
  p.dxy = make_fastdiv((uint32_t)(g.nx * g.ny));
  p.robin = g.robin_faces & 0x3Fu;
  p.inv_h2 = 1.0 / (g.h_mm * g.h_mm);
  p.inv_h = 1.0 / g.h_mm;
  return p;
}

// Per-launch parameters of up to kApplyBatch vectors travel as a kernel argument.
constexpr int kApplyBatch = 64;
struct ApplyParams {
  cd sig[kApplyBatch];
  double sigp[kApplyBatch];
  double scl[kApplyBatch];
  double tau[kApplyBatch];   // absorption perturbation weight (0 without one)
};

// y = scl * A_hat x with A_hat = A(lambda)/(D h^3); scl = D h^3 gives A x.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_apply_op(GridP g, const S* __restrict__ x, S* __restrict__ y,
                                                    ApplyParams prm, const double* __restrict__ mu) {
  const int v = blockIdx.y;
  const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= (uint32_t)g.N) return;
  const S* xv = x + (size_t)v * g.N;
  const VoxelInfo vi = voxel_info(g, n);
  const S a = apply_op<S>(g, xv, n, vi, prm.sig[v], prm.sigp[v], mu ? prm.tau[v] * mu[n] : 0.0);
  y[(size_t)v * g.N + n] = scale(a, prm.scl[v]);
}

hydot_tuning resolved_tuning(const hydot_tuning& t, const GridP* g) {
  hydot_tuning r = t;
  if (r.step_presum == 0) r.step_presum = 16;
  if (r.step_order == 0) r.step_order = g ? default_step_order(g->nx, g->ny) : 3;
  if (r.step_group == 0) r.step_group = 2;
  if (r.born_blocks == 0) r.born_blocks = 4096;
  if (r.step_vx == 0) r.step_vx = 1;
  if (r.step_pair == 0) r.step_pair = 2;
  return r;   // born_stage 0 stays: chosen per call from the LDS footprint
}

}  // namespace hydot

hydot_operator::~hydot_operator() {
  if (mu64) (void)hipFree(mu64);
  if (mu32) (void)hipFree(mu32);
  if (pc_dev) (void)hipFree(pc_dev);
}

using namespace hydot;

extern "C" {

const char* hydot_last_error(void) { return g_last_error.c_str(); }
const char* hydot_version(void) { return "hydot 0.1 (gfx950)"; }

hydot_status hydot_assemble_operator(const hydot_grid* grid, const hydot_optics* optics,
                                     hydot_operator** out) {
  if (!grid || !optics || !out) return fail(HYDOT_EINVAL, "assemble: null argument");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(HYDOT_EINVAL, "assemble: grid dims must be >= 1");
  const int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  if (N >= (int64_t(1) << 31)) return fail(HYDOT_EINVAL, "assemble: nx*ny*nz must be < 2^31");
  if (!(grid->h_mm > 0.0) || !std::isfinite(grid->h_mm)) return fail(HYDOT_EINVAL, "assemble: h_mm must be > 0");
  if (!(grid->A_R > 0.0) || !std::isfinite(grid->A_R)) return fail(HYDOT_EINVAL, "assemble: A_R must be > 0");
  if (grid->robin_faces & ~0x3Fu) return fail(HYDOT_EINVAL, "assemble: robin_faces has bits above 0x3F");
  const int L = optics->n_lambda, ns = optics->n_species;
  if (L < 1) return fail(HYDOT_EINVAL, "assemble: n_lambda must be >= 1");
  if (ns < 1 || ns > 8) return fail(HYDOT_EINVAL, "assemble: n_species must be in [1, 8]");
  if (!optics->mus_prime_per_mm || !optics->extinction || !optics->conc_uM)
    return fail(HYDOT_EINVAL, "assemble: null optics array");
  if (!std::isfinite(optics->omega_over_nu_per_mm) || optics->omega_over_nu_per_mm < 0.0)
    return fail(HYDOT_EINVAL, "assemble: omega_over_nu must be finite and >= 0");
  hydot_operator* op = new (std::nothrow) hydot_operator();
  if (!op) return fail(HYDOT_ENOMEM, "assemble: out of host memory");
  op->grid = *grid;
  op->gp = make_gridp(*grid);
  op->L = L;
  op->nsp = ns;
  op->omega_over_nu = optics->omega_over_nu_per_mm;
  op->ext.assign(optics->extinction, optics->extinction + (size_t)ns * L);
  op->conc.assign(optics->conc_uM, optics->conc_uM + ns);
  op->D.resize(L);
  op->mua.resize(L);
  op->sigma.resize(L);
  op->sigp.resize(L);
  double mean = 0.0;
  for (int l = 0; l < L; ++l) {
    const double mus = optics->mus_prime_per_mm[l];
    if (!(mus > 0.0) || !std::isfinite(mus)) {
      delete op;
      return fail(HYDOT_EINVAL, "assemble: mus_prime must be finite and > 0");
    }
    double mua = 0.0;
    for (int s = 0; s < ns; ++s) mua += op->conc[s] * op->ext[(size_t)s * L + l];
    if (!std::isfinite(mua)) {
      delete op;
      return fail(HYDOT_EINVAL, "assemble: non-finite absorption");
    }
    const double D = 1.0 / (3.0 * mus);            // Sec. 2.1, D = nu/(3 mu_s') with nu divided out
    op->D[l] = D;
    op->mua[l] = mua;                                // eq. perturbation for the background
    op->sigma[l] = cd{mua / D, op->omega_over_nu / D};  // sigma_j of eq. multipleshifted (frequency domain)
    op->sigp[l] = 1.0 / (2.0 * grid->A_R * D);      // sigma'_j of eq. multipleshifted
    mean += op->sigp[l];
  }
  op->sigp_mean = mean / L;                          // mean-shift transform, Sec. 6.1
  op->sigp_min = *std::min_element(op->sigp.begin(), op->sigp.end());
  op->sigp_max = *std::max_element(op->sigp.begin(), op->sigp.end());
  cd sm{0.0, 0.0};
  for (int l = 0; l < L; ++l) sm = cd{sm.re + op->sigma[l].re / L, sm.im + op->sigma[l].im / L};
  op->sigma_mean = sm;                               // one shift for the fixed preconditioner
  *out = op;
  return HYDOT_OK;
}

void hydot_free_operator(hydot_operator* op) { delete op; }

hydot_status hydot_set_absorption_perturbation(hydot_operator* op, const double* shape, const double* scale) {
  if (!op) return hydot::fail(HYDOT_EINVAL, "set_absorption_perturbation: null operator");
  if (!shape) {   // clear
    op->has_pert = false;
    return HYDOT_OK;
  }
  if (!scale) return hydot::fail(HYDOT_EINVAL, "set_absorption_perturbation: null scale");
  const size_t N = (size_t)op->gp.N;
  for (size_t n = 0; n < N; ++n)
    if (!std::isfinite(shape[n])) return hydot::fail(HYDOT_EINVAL, "set_absorption_perturbation: non-finite shape");
  std::vector<double> tau(op->L);
  double mean = 0.0;
  for (int l = 0; l < op->L; ++l) {
    if (!std::isfinite(scale[l])) return hydot::fail(HYDOT_EINVAL, "set_absorption_perturbation: non-finite scale");
    tau[l] = scale[l] / op->D[l];
    mean += tau[l];
  }
  if (!op->mu64) {
    if (hipMalloc(&op->mu64, N * sizeof(double)) != hipSuccess) {
      op->mu64 = nullptr;
      return hydot::fail(HYDOT_EDEVICE, "set_absorption_perturbation: device allocation");
    }
    if (hipMalloc(&op->mu32, N * sizeof(float)) != hipSuccess) {
      op->mu32 = nullptr;
      return hydot::fail(HYDOT_EDEVICE, "set_absorption_perturbation: device allocation");
    }
  }
  std::vector<float> s32(shape, shape + N);
  HYDOT_HIP(hipMemcpy(op->mu64, shape, N * sizeof(double), hipMemcpyHostToDevice));
  HYDOT_HIP(hipMemcpy(op->mu32, s32.data(), N * sizeof(float), hipMemcpyHostToDevice));
  op->tau = tau;
  op->tau_mean = mean / op->L;
  op->has_pert = true;
  return HYDOT_OK;
}

hydot_status hydot_get_tuning(const hydot_operator* op, hydot_tuning* out) {
  if (!op || !out) return hydot::fail(HYDOT_EINVAL, "get_tuning: null argument");
  *out = hydot::resolved_tuning(op->tune, &op->gp);
  return HYDOT_OK;
}

hydot_status hydot_set_tuning(hydot_operator* op, const hydot_tuning* t) {
  if (!op || !t) return hydot::fail(HYDOT_EINVAL, "set_tuning: null argument");
  const bool ok = (t->step_presum == 0 || t->step_presum == 1 || t->step_presum == 2 || t->step_presum == 4 ||
                   t->step_presum == 16) &&
                  (t->step_order >= 0 && t->step_order <= 4) && (t->step_group >= 0 && t->step_group <= 2) &&
                  (t->born_stage == 0 || t->born_stage == 16 || t->born_stage == 32) &&
                  (t->born_blocks == 0 || (t->born_blocks >= 256 && t->born_blocks <= 65536)) &&
                  (t->step_vx >= 0 && t->step_vx <= 2) && !(t->step_vx == 2 && t->step_presum != 4) &&
                  (t->step_pair >= 0 && t->step_pair <= 2);
  if (!ok) return hydot::fail(HYDOT_EINVAL, "set_tuning: field out of range");
  op->tune = *t;
  return HYDOT_OK;
}

hydot_status hydot_operator_optics(const hydot_operator* op, double* D_out, double* mua_out) {
  if (!op) return fail(HYDOT_EINVAL, "operator_optics: null operator");
  for (int l = 0; l < op->L; ++l) {
    if (D_out) D_out[l] = op->D[l];
    if (mua_out) mua_out[l] = op->mua[l];
  }
  return HYDOT_OK;
}

hydot_status hydot_apply_operator(const hydot_operator* op, int32_t n_vec, const int32_t* lam_index,
                                  const void* x, void* y, hydot_dtype dtype, hipStream_t stream) {
  if (!op) return fail(HYDOT_EINVAL, "apply_operator: null operator");
  if (n_vec < 0 || n_vec > 65535) return fail(HYDOT_EINVAL, "apply_operator: n_vec must be in [0, 65535]");
  if (n_vec == 0) return HYDOT_OK;
  if (!lam_index || !x || !y) return fail(HYDOT_EINVAL, "apply_operator: null pointer");
  if (dtype != HYDOT_C128 && dtype != HYDOT_C64) return fail(HYDOT_EUNSUPPORTED, "apply_operator: dtype must be C128 or C64");
  const size_t N = (size_t)op->gp.N;
  const size_t esz = dtype == HYDOT_C128 ? 16 : 8;
  const char* xb = (const char*)x;
  const char* yb = (const char*)y;
  if (xb < yb + (size_t)n_vec * N * esz && yb < xb + (size_t)n_vec * N * esz)
    return fail(HYDOT_EINVAL, "apply_operator: x and y overlap");
  const double h3 = op->grid.h_mm * op->grid.h_mm * op->grid.h_mm;
  for (int v = 0; v < n_vec; ++v)
    if (lam_index[v] < 0 || lam_index[v] >= op->L) return fail(HYDOT_EINVAL, "apply_operator: lam_index out of range");
  for (int v0 = 0; v0 < n_vec; v0 += kApplyBatch) {
    const int nb = std::min(kApplyBatch, n_vec - v0);
    ApplyParams prm;
    for (int v = 0; v < nb; ++v) {
      const int l = lam_index[v0 + v];
      prm.sig[v] = op->sigma[l];
      prm.sigp[v] = op->sigp[l];
      prm.scl[v] = op->D[l] * h3;
      prm.tau[v] = op->has_pert ? op->tau[l] : 0.0;
    }
    dim3 grid((unsigned)((N + kBlock - 1) / kBlock), (unsigned)nb);
    if (dtype == HYDOT_C128)
      hipLaunchKernelGGL(k_apply_op<cd>, grid, dim3(kBlock), 0, stream, op->gp,
                         (const cd*)x + (size_t)v0 * N, (cd*)y + (size_t)v0 * N, prm, (const double*)op->mu64);
    else
      hipLaunchKernelGGL(k_apply_op<cf>, grid, dim3(kBlock), 0, stream, op->gp,
                         (const cf*)x + (size_t)v0 * N, (cf*)y + (size_t)v0 * N, prm, (const double*)op->mu64);
    HYDOT_HIP(hipGetLastError());
  }
  return HYDOT_OK;
}

}  // extern "C"
