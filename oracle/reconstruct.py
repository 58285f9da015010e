"""Alg. opt (Sec. 5) on an explicit Born matrix: contrasts by linear least squares, PaLS
parameters by Levenberg-Marquardt, discrepancy-principle stopping.

Test infrastructure (see the package docstring); never used by the product.

Readings (the algorithm box leaves these open or prints them garbled):
* both loop conditions run while the misfit is above the discrepancy target gamma ||W eta||
  (the stopping rule of the text); an outer pass also ends when its LM steps gained less than a
  relative 1e-6 (noise-free data never meet a zero target), and an inner pass after max_inner
  steps or a step that no damping could make descend;
* the LM step is the printed one, (J^T J + nu I) dp = -J^T eps (damping="identity", the
  default), with nu starting at 1e-3 max diag(J^T J); damping="marquardt" takes Marquardt's
  scaling nu diag(J^T J) instead, with nu starting at 1e-3 (the parameters have unrelated units
  -- alpha none, beta 1/mm, centres mm -- and the scaled form is the printed step in parameters
  scaled to unit curvature).  Either way nu is divided by 10 after an accepted step and
  multiplied by 10 after a rejected one (at most 12 tries per step); a step is accepted when it
  lowers the misfit at the current contrasts.  The floor of nu is 1e-12 for nu I and 1e-6 for
  the scaled form: there nu is relative to each curvature entry, so below 1e-6 it no longer
  changes the step, and the 12 tries must still reach a damping far above the curvature (from a
  floor of 1e-12 they reach only nu = 1, too little where voxels cross the band of the smoothed
  Heaviside, and the pass then ends without a step);
* the complex residual and Jacobian are split into real and imaginary parts, so the unknowns
  stay real;
* after the discrepancy stop the contrasts are refitted once more at the final shape.
"""
from __future__ import annotations

import numpy as np

from . import pals


def forward_parts(H, w, p, tau, eps, nu):
    """mu(p) and H mu(p) for the explicit H [L, S, D, N] of the workload w."""
    mu = pals.shape(w, p, tau, eps, nu)
    return mu, np.tensordot(H, mu, axes=([3], [0]))


def lstsq_contrasts(ext, Hmu, y, W):
    A = np.stack([(W * ext[i][:, None, None] * Hmu).ravel() for i in range(ext.shape[0])], axis=1)
    b = (W * y).ravel()
    Ar = np.concatenate([A.real, A.imag], axis=0)
    br = np.concatenate([b.real, b.imag])
    return np.linalg.lstsq(Ar, br, rcond=None)[0]


def lm_jacobian(H, w, p, c, ext, W, tau, eps, nu):
    """d eps / d p = -W ebar H d mu / d p as a real [2M, n_p] matrix."""
    dmu = pals.shape_jacobian(w, p, tau, eps, nu)                   # [N, n_p]
    Hd = np.tensordot(H, dmu, axes=([3], [0]))                      # [L, S, D, n_p]
    ebar = c @ ext
    Jc = -(W * ebar[:, None, None])[..., None] * Hd
    Jc = Jc.reshape(-1, Jc.shape[-1])
    return np.concatenate([Jc.real, Jc.imag], axis=0)


def reconstruct(H, w, ext, y, p0, c0=None, W=1.0, noise_norm=0.0, gamma=1.05, max_outer=20, max_inner=8,
                tau=0.5, eps=0.5, nu=1e-3, fix_c=False, damping="identity"):
    if damping not in ("identity", "marquardt"):
        raise ValueError("damping must be 'identity' or 'marquardt'")
    p = np.array(p0, dtype=float)
    mu, Hmu = forward_parts(H, w, p, tau, eps, nu)
    c = np.array(c0, dtype=float) if c0 is not None else lstsq_contrasts(ext, Hmu, y, W)

    def misfit(cc, HH):
        return np.linalg.norm(W * (y - (cc @ ext)[:, None, None] * HH))

    damp = None
    hist = []
    for _ in range(max_outer):
        if not fix_c:
            c = lstsq_contrasts(ext, Hmu, y, W)
        f = misfit(c, Hmu)
        hist.append(f)
        if f <= gamma * noise_norm:
            break
        f0 = f
        for _ in range(max_inner):
            J = lm_jacobian(H, w, p, c, ext, W, tau, eps, nu)
            r = (W * (y - (c @ ext)[:, None, None] * Hmu)).ravel()
            e = np.concatenate([r.real, r.imag])
            JTJ = J.T @ J
            if damping == "identity":
                scale = np.eye(len(p))
            else:
                scale = np.diag(JTJ.diagonal())
            if damp is None:
                damp = 1e-3 * (JTJ.diagonal().max() if damping == "identity" else 1.0)
            ok = False
            for _ in range(12):
                step = np.linalg.solve(JTJ + damp * scale, -(J.T @ e))
                _, Hm = forward_parts(H, w, p + step, tau, eps, nu)
                ft = misfit(c, Hm)
                if ft < f:
                    p, Hmu, f = p + step, Hm, ft
                    damp = max(damp / 10.0, 1e-12 if damping == "identity" else 1e-6)
                    ok = True
                    break
                damp *= 10.0
            hist.append(f)
            if not ok or f <= gamma * noise_norm:
                break
        if f <= gamma * noise_norm:
            if not fix_c:
                c = lstsq_contrasts(ext, Hmu, y, W)
            break
        if f0 - f <= 1e-6 * f0:
            break
    return c, p, hist
