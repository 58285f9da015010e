// Parametric level-set shape and data misfit (Sec. 5, eq. pals and
// eq. minimization) with their gradients, for the Born data model of
// eq. measurement with co-located chromophores.
//
// Shape: mu(r) = H_eps(varphi(r) - tau), varphi(r) = sum_b alpha_b psi(beta_b ||r - chi_b||_dag),
// psi the compactly supported radial basis function of Wendland, psi(t) = (1 - t)^4 (4 t + 1) for
// t < 1 and 0 beyond (C^2, support radius 1/beta_b; the paper's choice), or the Gaussian
// psi(t) = exp(-t^2) (beta_b = 1/width), ||x||_dag = sqrt(||x||^2 + nu^2), and the C^1
// smoothed Heaviside
// H_eps(x) = (1 + x/eps + sin(pi x/eps)/pi)/2 on |x| <= eps (0 below, 1 above) whose
// derivative is delta_eps(x) = (1 + cos(pi x/eps))/(2 eps).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "operator.h"

namespace hydot {

constexpr int kMaxBumps = 32;

struct PalsP {
  int nb, basis;   // basis: HYDOT_PALS_WENDLAND or HYDOT_PALS_GAUSSIAN
  double tau, eps, nu, h;
  double alpha[kMaxBumps], beta[kMaxBumps], cx[kMaxBumps], cy[kMaxBumps], cz[kMaxBumps];
};

__device__ inline void voxel_centre(const GridP& g, uint32_t n, double h, double& x, double& y, double& z) {
  const VoxelInfo vi = voxel_info(g, n);
  x = (vi.i + 0.5) * h;
  y = (vi.j + 0.5) * h;
  z = (vi.k + 0.5) * h;
}

__device__ inline double rbf(double t, int basis) {
  if (basis == HYDOT_PALS_GAUSSIAN) return exp(-t * t);
  if (t >= 1.0) return 0.0;
  const double u = 1.0 - t, u2 = u * u;
  return u2 * u2 * (4.0 * t + 1.0);
}

// psi'(t): -20 t (1 - t)^3 on t < 1 (Wendland), -2 t exp(-t^2) (Gaussian).
__device__ inline double rbf_deriv(double t, int basis) {
  if (basis == HYDOT_PALS_GAUSSIAN) return -2.0 * t * exp(-t * t);
  if (t >= 1.0) return 0.0;
  const double u = 1.0 - t;
  return -20.0 * t * u * u * u;
}

__device__ inline double level(const PalsP& p, double x, double y, double z) {
  double phi = 0.0;
  for (int b = 0; b < p.nb; ++b) {
    const double dx = x - p.cx[b], dy = y - p.cy[b], dz = z - p.cz[b];
    const double dist = sqrt(dx * dx + dy * dy + dz * dz + p.nu * p.nu);
    phi += p.alpha[b] * rbf(p.beta[b] * dist, p.basis);
  }
  return phi;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_pals_shape(GridP g, PalsP p, R* mu) {
  const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= (uint32_t)g.N) return;
  double x, y, z;
  voxel_centre(g, n, p.h, x, y, z);
  const double s = level(p, x, y, z) - p.tau;
  double H;
  if (s < -p.eps) H = 0.0;
  else if (s > p.eps) H = 1.0;
  else H = 0.5 * (1.0 + s / p.eps + sin(M_PI * s / p.eps) / M_PI);
  mu[n] = (R)H;
}

// Per-block partial sums of (d mu/d p)^T Re(g), 5*nb values per block.
template <typename G, bool CPLX>
__global__ __launch_bounds__(kBlock) void k_pals_vjp(GridP g, PalsP p, const G* gin, double* part) {
  __shared__ double lds[kWaves][5 * kMaxBumps];
  const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double x = 0, y = 0, z = 0, wgt = 0.0;
  if (n < (uint32_t)g.N) {
    voxel_centre(g, n, p.h, x, y, z);
    const double s = level(p, x, y, z) - p.tau;
    if (s >= -p.eps && s <= p.eps) {
      const double delta = (1.0 + cos(M_PI * s / p.eps)) / (2.0 * p.eps);
      double gv;
      if constexpr (CPLX) gv = (double)gin[2 * (size_t)n];   // real part of interleaved complex
      else gv = (double)gin[n];
      wgt = delta * gv;
    }
  }
  for (int b = 0; b < p.nb; ++b) {
    double da = 0, dbeta = 0, dcx = 0, dcy = 0, dcz = 0;
    if (wgt != 0.0) {
      const double dx = x - p.cx[b], dy = y - p.cy[b], dz = z - p.cz[b];
      const double dist = sqrt(dx * dx + dy * dy + dz * dz + p.nu * p.nu);
      const double t = p.beta[b] * dist;
      const double psi = rbf(t, p.basis);
      const double dpsi = rbf_deriv(t, p.basis);
      da = wgt * psi;
      dbeta = wgt * p.alpha[b] * dpsi * dist;
      const double common = wgt * p.alpha[b] * dpsi * p.beta[b] / dist;
      dcx = -common * dx;
      dcy = -common * dy;
      dcz = -common * dz;
    }
    da = wave_sum(da);
    dbeta = wave_sum(dbeta);
    dcx = wave_sum(dcx);
    dcy = wave_sum(dcy);
    dcz = wave_sum(dcz);
    if (lane == 0) {
      lds[wave][b] = da;
      lds[wave][p.nb + b] = dbeta;
      lds[wave][2 * p.nb + b] = dcx;
      lds[wave][3 * p.nb + b] = dcy;
      lds[wave][4 * p.nb + b] = dcz;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 5 * p.nb; i += kBlock) {
    double a = 0.0;
    for (int w = 0; w < kWaves; ++w) a += lds[w][i];
    part[(size_t)blockIdx.x * 5 * p.nb + i] = a;
  }
}

// Columns of the shape Jacobian: jac[i][n] = d mu_n / d p_i for the 5*nb parameters in the order
// [alpha, beta, chi_x, chi_y, chi_z] (one row of N per parameter: a block of probe vectors).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pals_jacobian(GridP g, PalsP p, R* jac) {
  const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= (uint32_t)g.N) return;
  const size_t N = (size_t)g.N;
  double x, y, z;
  voxel_centre(g, n, p.h, x, y, z);
  const double s = level(p, x, y, z) - p.tau;
  const double delta = (s >= -p.eps && s <= p.eps) ? (1.0 + cos(M_PI * s / p.eps)) / (2.0 * p.eps) : 0.0;
  for (int b = 0; b < p.nb; ++b) {
    double da = 0, dbeta = 0, dcx = 0, dcy = 0, dcz = 0;
    if (delta != 0.0) {
      const double dx = x - p.cx[b], dy = y - p.cy[b], dz = z - p.cz[b];
      const double dist = sqrt(dx * dx + dy * dy + dz * dz + p.nu * p.nu);
      const double t = p.beta[b] * dist;
      const double psi = rbf(t, p.basis);
      const double dpsi = rbf_deriv(t, p.basis);
      da = delta * psi;
      dbeta = delta * p.alpha[b] * dpsi * dist;
      const double common = delta * p.alpha[b] * dpsi * p.beta[b] / dist;
      dcx = -common * dx;
      dcy = -common * dy;
      dcz = -common * dz;
    }
    jac[(size_t)b * N + n] = (R)da;
    jac[(size_t)(p.nb + b) * N + n] = (R)dbeta;
    jac[(size_t)(2 * p.nb + b) * N + n] = (R)dcx;
    jac[(size_t)(3 * p.nb + b) * N + n] = (R)dcy;
    jac[(size_t)(4 * p.nb + b) * N + n] = (R)dcz;
  }
}

__global__ void k_sum_rows(const double* part, int nrows, int ncols, double* out) {
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < nrows; ++r) a += part[(size_t)r * ncols + c];
    out[c] = a;
  }
}

// One block per wavelength: r = ebar*Jmu - y, w_adj = ebar*W^2*r,
// out[l] = (sum W^2 |r|^2 / 2, sum Re(conj(W^2 r) Jmu)).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_misfit(int SD, const double* ebar, const cplx<T>* Jmu, const cplx<T>* yobs,
                                                  const T* wts, cplx<T>* wadj, double* out) {
  __shared__ double lds[2][kWaves];
  const int l = blockIdx.x;
  const double e = ebar[l];
  double fa = 0.0, qa = 0.0;
  for (int i = threadIdx.x; i < SD; i += kBlock) {
    const size_t idx = (size_t)l * SD + i;
    const cplx<T> jm = Jmu[idx], yo = yobs[idx];
    const double w2 = wts ? (double)wts[idx] * (double)wts[idx] : 1.0;
    const double rr = e * jm.re - yo.re, ri = e * jm.im - yo.im;
    fa += 0.5 * w2 * (rr * rr + ri * ri);
    qa += w2 * (rr * jm.re + ri * jm.im);
    wadj[idx] = cplx<T>{(T)(e * w2 * rr), (T)(e * w2 * ri)};
  }
  fa = wave_sum(fa);
  qa = wave_sum(qa);
  if ((threadIdx.x & 63) == 0) {
    lds[0][threadIdx.x >> 6] = fa;
    lds[1][threadIdx.x >> 6] = qa;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int w = 0; w < kWaves; ++w) {
      a += lds[0][w];
      b += lds[1][w];
    }
    out[2 * l] = a;
    out[2 * l + 1] = b;
  }
}

static hydot_status make_pals(const hydot_operator* op, const double* p, int nb, const hydot_pals_opts* po, PalsP& pp) {
  if (!op) return fail(HYDOT_EINVAL, "pals: null operator");
  if (!p || !po) return fail(HYDOT_EINVAL, "pals: null parameters");
  if (nb < 1 || nb > kMaxBumps) return fail(HYDOT_EINVAL, "pals: n_bumps must be in [1, 32]");
  if (!(po->eps > 0.0) || !(po->nu >= 0.0) || !std::isfinite(po->tau) ||
      (po->basis != HYDOT_PALS_WENDLAND && po->basis != HYDOT_PALS_GAUSSIAN))
    return fail(HYDOT_EINVAL, "pals: need eps > 0, nu >= 0, finite tau");
  for (int i = 0; i < 5 * nb; ++i)
    if (!std::isfinite(p[i])) return fail(HYDOT_EINVAL, "pals: non-finite parameter");
  pp.nb = nb;
  pp.basis = po->basis;
  pp.tau = po->tau;
  pp.eps = po->eps;
  pp.nu = po->nu;
  pp.h = op->grid.h_mm;
  for (int b = 0; b < nb; ++b) {
    pp.alpha[b] = p[b];
    pp.beta[b] = p[nb + b];
    pp.cx[b] = p[2 * nb + b];
    pp.cy[b] = p[3 * nb + b];
    pp.cz[b] = p[4 * nb + b];
  }
  return HYDOT_OK;
}

}  // namespace hydot

using namespace hydot;

extern "C" {

hydot_status hydot_pals_shape(const hydot_operator* op, const double* p, int32_t n_bumps, const hydot_pals_opts* popts,
                              void* mu, hydot_dtype mu_dtype, hipStream_t stream) {
  PalsP pp;
  hydot_status s = make_pals(op, p, n_bumps, popts, pp);
  if (s != HYDOT_OK) return s;
  if (!mu) return fail(HYDOT_EINVAL, "pals_shape: null mu");
  const int N = op->gp.N;
  dim3 grid((N + kBlock - 1) / kBlock);
  if (mu_dtype == HYDOT_F64)
    hipLaunchKernelGGL(k_pals_shape<double>, grid, dim3(kBlock), 0, stream, op->gp, pp, (double*)mu);
  else if (mu_dtype == HYDOT_F32)
    hipLaunchKernelGGL(k_pals_shape<float>, grid, dim3(kBlock), 0, stream, op->gp, pp, (float*)mu);
  else
    return fail(HYDOT_EUNSUPPORTED, "pals_shape: mu_dtype must be F64 or F32");
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

hydot_status hydot_pals_shape_jacobian(const hydot_operator* op, const double* p, int32_t n_bumps,
                                       const hydot_pals_opts* popts, void* jac, hydot_dtype jac_dtype,
                                       hipStream_t stream) {
  PalsP pp;
  hydot_status s = make_pals(op, p, n_bumps, popts, pp);
  if (s != HYDOT_OK) return s;
  if (!jac) return fail(HYDOT_EINVAL, "pals_shape_jacobian: null jac");
  const int N = op->gp.N;
  dim3 grid((N + kBlock - 1) / kBlock);
  if (jac_dtype == HYDOT_F64)
    hipLaunchKernelGGL(k_pals_jacobian<double>, grid, dim3(kBlock), 0, stream, op->gp, pp, (double*)jac);
  else if (jac_dtype == HYDOT_F32)
    hipLaunchKernelGGL(k_pals_jacobian<float>, grid, dim3(kBlock), 0, stream, op->gp, pp, (float*)jac);
  else
    return fail(HYDOT_EUNSUPPORTED, "pals_shape_jacobian: jac_dtype must be F64 or F32");
  HYDOT_HIP(hipGetLastError());
  return HYDOT_OK;
}

size_t hydot_pals_workspace_bytes(const hydot_operator* op, int32_t n_bumps) {
  if (!op || n_bumps < 1) return 0;
  const size_t nblk = (op->gp.N + kBlock - 1) / kBlock;
  return (nblk + 1) * 5 * (size_t)n_bumps * sizeof(double);
}

hydot_status hydot_pals_shape_vjp(const hydot_operator* op, const double* p, int32_t n_bumps,
                                  const hydot_pals_opts* popts, const void* g, hydot_dtype g_dtype, double* grad_p,
                                  void* workspace, size_t ws_bytes, hipStream_t stream) {
  PalsP pp;
  hydot_status s = make_pals(op, p, n_bumps, popts, pp);
  if (s != HYDOT_OK) return s;
  if (!g || !grad_p || !workspace) return fail(HYDOT_EINVAL, "pals_vjp: null pointer");
  if (ws_bytes < hydot_pals_workspace_bytes(op, n_bumps)) return fail(HYDOT_ENOMEM, "pals_vjp: workspace too small");
  const int N = op->gp.N;
  const int nblk = (N + kBlock - 1) / kBlock;
  double* part = (double*)workspace;
  double* out = part + (size_t)nblk * 5 * n_bumps;
  switch (g_dtype) {
    case HYDOT_F64: hipLaunchKernelGGL((k_pals_vjp<double, false>), dim3(nblk), dim3(kBlock), 0, stream, op->gp, pp, (const double*)g, part); break;
    case HYDOT_F32: hipLaunchKernelGGL((k_pals_vjp<float, false>), dim3(nblk), dim3(kBlock), 0, stream, op->gp, pp, (const float*)g, part); break;
    case HYDOT_C128: hipLaunchKernelGGL((k_pals_vjp<double, true>), dim3(nblk), dim3(kBlock), 0, stream, op->gp, pp, (const double*)g, part); break;
    case HYDOT_C64: hipLaunchKernelGGL((k_pals_vjp<float, true>), dim3(nblk), dim3(kBlock), 0, stream, op->gp, pp, (const float*)g, part); break;
    default: return fail(HYDOT_EUNSUPPORTED, "pals_vjp: unsupported g_dtype");
  }
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, stream, part, nblk, 5 * n_bumps, out);
  HYDOT_HIP(hipGetLastError());
  HYDOT_HIP(hipMemcpyAsync(grad_p, out, 5 * (size_t)n_bumps * sizeof(double), hipMemcpyDeviceToHost, stream));
  HYDOT_HIP(hipStreamSynchronize(stream));
  return HYDOT_OK;
}

size_t hydot_misfit_workspace_bytes(const hydot_operator* op, int32_t S, int32_t D) {
  (void)S;
  (void)D;
  if (!op) return 0;
  return 3 * (size_t)op->L * sizeof(double);
}

hydot_status hydot_misfit(const hydot_operator* op, int32_t S, int32_t D, const double* dconc, const void* Jmu,
                          const void* y_obs, const void* weights, hydot_dtype dtype, void* w_adj, double* f,
                          double* grad_dconc, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!op) return fail(HYDOT_EINVAL, "misfit: null operator");
  if (S < 1 || D < 1) return fail(HYDOT_EINVAL, "misfit: S and D must be >= 1");
  if (!dconc || !Jmu || !y_obs || !w_adj || !f || !grad_dconc || !workspace)
    return fail(HYDOT_EINVAL, "misfit: null pointer");
  if (dtype != HYDOT_C128 && dtype != HYDOT_C64) return fail(HYDOT_EUNSUPPORTED, "misfit: dtype must be C128 or C64");
  if (ws_bytes < hydot_misfit_workspace_bytes(op, S, D)) return fail(HYDOT_ENOMEM, "misfit: workspace too small");
  const int L = op->L;
  std::vector<double> ebar(L, 0.0);
  for (int l = 0; l < L; ++l)
    for (int sp = 0; sp < op->nsp; ++sp) ebar[l] += op->ext[(size_t)sp * L + l] * dconc[sp];
  double* dbar = (double*)workspace;
  double* dout = dbar + L;
  HYDOT_HIP(hipMemcpyAsync(dbar, ebar.data(), L * sizeof(double), hipMemcpyHostToDevice, stream));
  if (dtype == HYDOT_C128)
    hipLaunchKernelGGL(k_misfit<double>, dim3(L), dim3(kBlock), 0, stream, S * D, dbar, (const cd*)Jmu, (const cd*)y_obs,
                       (const double*)weights, (cd*)w_adj, dout);
  else
    hipLaunchKernelGGL(k_misfit<float>, dim3(L), dim3(kBlock), 0, stream, S * D, dbar, (const cf*)Jmu, (const cf*)y_obs,
                       (const float*)weights, (cf*)w_adj, dout);
  HYDOT_HIP(hipGetLastError());
  std::vector<double> o(2 * (size_t)L);
  HYDOT_HIP(hipMemcpyAsync(o.data(), dout, o.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  HYDOT_HIP(hipStreamSynchronize(stream));
  double fs = 0.0;
  for (int l = 0; l < L; ++l) fs += o[2 * l];
  *f = fs;
  for (int sp = 0; sp < op->nsp; ++sp) {
    double a = 0.0;
    for (int l = 0; l < L; ++l) a += op->ext[(size_t)sp * L + l] * o[2 * l + 1];
    grad_dconc[sp] = a;
  }
  return HYDOT_OK;
}

}  // extern "C"
