"""Parametric level-set shape, data misfit and gradient, FP64.

Test infrastructure (see the package docstring); never used by the product.

Shape (Sec. 5, eq. pals): chi(r) = H(varphi(r) - tau) with
varphi(r) = sum_k alpha_k psi(beta_k ||r - chi_k||_dagger),
||x||_dagger = sqrt(||x||^2 + nu^2).  The paper names compactly supported radial
basis functions (those of the PaLS method it builds on) and leaves nu, tau and the
smoothed Heaviside open; the readings used here are Wendland's C^2 function
psi(t) = (1 - t)^4 (4t + 1) for t < 1, 0 beyond (basis "wendland", the default; the
Gaussian psi(t) = exp(-t^2) is the alternative basis "gaussian"), nu = 1e-3 mm,
tau = 0.5 and the C^1 smoothed Heaviside

    H_eps(x) = 0 (x < -eps), 1 (x > eps), (1 + x/eps + sin(pi x/eps)/pi)/2 otherwise,
    delta_eps(x) = (1 + cos(pi x/eps))/(2 eps) on |x| <= eps, 0 outside,

with eps = 0.5.  Parameters p = [alpha(n), beta(n), chi_x(n), chi_y(n), chi_z(n)]
(Sec. 5, ordering of p).

Measurement model (Sec. 2.2, eq. measurement, with the chromophores
co-located, eq. perturbation): the absorption change is
sum_l eps_l(lambda) dc_l mu(r), so the predicted data are
yhat[l,s,d] = ebar_l (J_l mu)[s,d], ebar_l = sum_l' eps_l'(lambda_l) dc_l'.
Misfit (eq. minimization): f = 1/2 sum |W (yhat - y)|^2 over complex data,
W diagonal (identity unless weights are given).
"""
from __future__ import annotations

import numpy as np

from . import born, model


def heaviside(x, eps):
    x = np.asarray(x, dtype=np.float64)
    mid = 0.5 * (1.0 + x / eps + np.sin(np.pi * x / eps) / np.pi)
    return np.where(x < -eps, 0.0, np.where(x > eps, 1.0, mid))


def delta(x, eps):
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) <= eps, (1.0 + np.cos(np.pi * x / eps)) / (2.0 * eps), 0.0)


def _split(p):
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0] // 5
    return n, p[:n], p[n:2 * n], np.stack([p[2 * n:3 * n], p[3 * n:4 * n], p[4 * n:5 * n]], axis=1)


def psi(t, basis="wendland"):
    t = np.asarray(t, dtype=np.float64)
    if basis == "gaussian":
        return np.exp(-t ** 2)
    return np.where(t < 1.0, (1.0 - t) ** 4 * (4.0 * t + 1.0), 0.0)


def dpsi(t, basis="wendland"):
    t = np.asarray(t, dtype=np.float64)
    if basis == "gaussian":
        return -2.0 * t * np.exp(-t ** 2)
    return np.where(t < 1.0, -20.0 * t * (1.0 - t) ** 3, 0.0)


def level_function(r, p, nu, basis="wendland"):
    """varphi at points r [P, 3]; also returns per-bump pieces for the derivative."""
    n, alpha, beta, centre = _split(p)
    diff = r[:, None, :] - centre[None, :, :]               # [P, n, 3]
    dist = np.sqrt(np.sum(diff ** 2, axis=2) + nu ** 2)     # [P, n]
    t = beta[None, :] * dist
    ps = psi(t, basis)
    phi = ps @ alpha
    return phi, (diff, dist, t, ps, alpha, beta)


def shape(w, p, tau, eps, nu, basis="wendland"):
    """mu = H_eps(varphi - tau) at every voxel centre, [N]."""
    r = model.voxel_centres(w)
    phi, _ = level_function(r, p, nu, basis)
    return heaviside(phi - tau, eps)


def shape_jacobian(w, p, tau, eps, nu, basis="wendland"):
    """d mu / d p as a dense [N, 5n] matrix (chain rule of the definitions above)."""
    r = model.voxel_centres(w)
    phi, (diff, dist, t, ps, alpha, beta) = level_function(r, p, nu, basis)
    dpsi_dt = dpsi(t, basis)
    d_alpha = ps
    d_beta = alpha[None, :] * dpsi_dt * dist
    # d dist / d centre = -(r - centre)/dist
    common = alpha[None, :] * dpsi_dt * beta[None, :] / dist
    d_cx = -common * diff[:, :, 0]
    d_cy = -common * diff[:, :, 1]
    d_cz = -common * diff[:, :, 2]
    dphi = np.concatenate([d_alpha, d_beta, d_cx, d_cy, d_cz], axis=1)
    return delta(phi - tau, eps)[:, None] * dphi


def ebar(extinction, dconc):
    """Per-wavelength contrast ebar_l = sum_species eps(lambda_l) dc."""
    return np.asarray(dconc, dtype=np.float64) @ np.asarray(extinction, dtype=np.float64)


def misfit(w, phi_s, phi_d, p, dconc, y_obs, tau, eps, nu, weights=None, basis="wendland"):
    """f, df/d(dc) [n_species], df/dp [5n], plus yhat, for the Born data model."""
    mu = shape(w, p, tau, eps, nu, basis)
    Jmu = born.born_apply(phi_s, phi_d, mu[None, :], w.h)[0]         # [L, S, D]
    e = ebar(w.extinction, dconc)
    yhat = e[:, None, None] * Jmu
    W2 = 1.0 if weights is None else np.asarray(weights) ** 2
    r = yhat - y_obs
    f = 0.5 * float(np.sum(W2 * np.abs(r) ** 2))
    wr = W2 * r
    g_dc = np.array([float(np.real(np.sum(np.conj(wr) * w.extinction[l][:, None, None] * Jmu)))
                     for l in range(w.extinction.shape[0])])
    g_mu = np.real(born.born_apply_adjoint(phi_s, phi_d, e[:, None, None] * wr, w.h))
    g_p = shape_jacobian(w, p, tau, eps, nu, basis).T @ g_mu
    return f, g_dc, g_p, yhat
