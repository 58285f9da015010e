// Internal definition of the opaque operator handle.
#pragma once

#include <vector>

#include "common.h"

struct hydot_operator {
  hydot_grid grid;
  hydot::GridP gp;
  int L = 0;                      // wavelengths
  int nsp = 0;                    // chromophore species
  double omega_over_nu = 0.0;
  std::vector<double> ext;        // [nsp][L] extinction
  std::vector<double> conc;       // [nsp] background concentrations
  std::vector<double> D;          // [L] diffusion coefficient D_lambda = 1/(3 mu_s')
  std::vector<double> mua;        // [L] background absorption
  std::vector<hydot::cd> sigma;   // [L] (mu_a + i omega/nu)/D
  std::vector<double> sigp;       // [L] 1/(2 A_R D)
  double sigp_mean = 0.0;         // mean of sigma' over wavelengths
  double sigp_min = 0.0, sigp_max = 0.0;
  hydot::cd sigma_mean{0.0, 0.0};  // mean of sigma over wavelengths
  // absorption perturbation dmua_l(k) = scale_l * shape(k): tau_l = scale_l / D_l enters the
  // scaled operator as tau_l * diag(shape); device copies of the shape in FP64 and FP32
  bool has_pert = false;
  std::vector<double> tau;        // [L]
  double tau_mean = 0.0;
  double* mu64 = nullptr;         // device [N]
  float* mu32 = nullptr;          // device [N]
  // separable preconditioner data (eigenvectors and eigenvalues of the three axis operators
  // of K_hat), built on first use for the Robin shift sigma*' it was asked with
  mutable float* pc_dev = nullptr;   // device: per axis Qf [n*n4], Qi [n*n4], lam [n4]
  mutable double pc_sigp = 0.0;
  mutable bool pc_valid = false;
  ~hydot_operator();
  hydot_tuning tune{0, 0, 0, 0, 0, 0, 0};  // launch shapes; 0 = library default
};

namespace hydot {
GridP make_gridp(const hydot_grid& g);
// launch shapes with defaults filled in
// (with the grid: the block order default depends on the plane size, default_step_order)
hydot_tuning resolved_tuning(const hydot_tuning& t, const GridP* g = nullptr);
}
