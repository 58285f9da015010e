"""Reconstruction of chromophore contrasts and PaLS shape parameters from Born data (Sec. 5,
Alg. opt): alternate the linear least-squares solve for the contrasts c with Levenberg-Marquardt
steps for the shape parameters p, stopping by the discrepancy principle.

The LM step is the one Alg. opt prints, (J^T J + nu I) dp = -J^T eps, with nu from
1e-3 max diag(J^T J) (floor 1e-12); damping="marquardt" selects Marquardt's scaling
(J^T J + nu diag(J^T J)) dp = -J^T eps instead, which makes the step independent of the
parameters' units, with nu from 1e-3 (floor 1e-6: nu is relative to each curvature entry there).
Either way nu is divided by 10 after an accepted step and multiplied by 10 after a rejected
one, at most 12 tries per step.

Data model (eq. measurement, eq. minimization): y[l, s, d] = sum_i c_i eps_i(lambda_l) (H mu(p))[l, s, d]
+ noise, residual eps = W (y - D(p) c) with the columns of D(p) = E_i H mu(p).  The LM Jacobian is
J = d eps / d p = -W Ebar H (d mu / d p): the shape Jacobian (hydot_pals_shape_jacobian) is a block
of 5 n_bumps probe vectors and H times it is one Born J v call on the MFMA probe-vector path (or the
low-rank factors of a compressed H).  The small dense problems (the contrast least squares with
n_species unknowns, the LM normal equations with 5 n_bumps unknowns) are solved on the host in FP64.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _binding as B


@dataclass
class BornModel:
    op: B.Operator
    phi_src: torch.Tensor                 # [L, S, N] complex
    phi_det: torch.Tensor                 # [L, D, N]
    extinction: np.ndarray                # [n_species, L]
    weights: np.ndarray | None = None     # [L, S, D] real, or None for W = I
    compressed: object = None             # a CompressedBorn (H ~ U V^H), or None for the full H
    popts: B.PalsOptions = field(default_factory=B.PalsOptions)

    @property
    def shape_LSD(self):
        return (self.op.L, self.phi_src.shape[1], self.phi_det.shape[1])

    def _rdt(self):
        return torch.float64 if self.phi_src.dtype == torch.complex128 else torch.float32

    def H(self, v: torch.Tensor) -> np.ndarray:
        """H v for real v [n, N] -> [n, L, S, D] complex128 (host)."""
        L, S, D = self.shape_LSD
        if self.compressed is None:
            y = B.born_apply(self.op, self.phi_src, self.phi_det, v.to(self._rdt()))
        else:   # compressed rows are source-major (s, l, d)
            y = self.compressed.matvec(v).reshape(v.shape[0], S, L, D).permute(0, 2, 1, 3)
        return y.to(torch.complex128).cpu().numpy()

    def mu(self, p) -> torch.Tensor:
        return B.pals_shape(self.op, p, self.popts, dtype=self._rdt(), device=self.phi_src.device)

    def Hmu(self, p) -> np.ndarray:
        return self.H(self.mu(p)[None])[0]

    def Hjac(self, p) -> np.ndarray:
        jac = B.pals_shape_jacobian(self.op, p, self.popts, dtype=self._rdt(), device=self.phi_src.device)
        out = []
        for j0 in range(0, jac.shape[0], 64):
            out.append(self.H(jac[j0:j0 + 64]))
        return np.concatenate(out, axis=0)                        # [n_p, L, S, D]

    def w(self):
        return 1.0 if self.weights is None else self.weights


def _stack(z: np.ndarray) -> np.ndarray:
    """complex [..] -> real [2*..] (Re then Im) for least squares over real unknowns."""
    z = z.reshape(z.shape[0], -1) if z.ndim > 1 else z
    return np.concatenate([z.real, z.imag], axis=-1)


def contrast_ls(model: BornModel, Hmu: np.ndarray, y: np.ndarray) -> np.ndarray:
    """c = (W D(p))^+ (W y): the columns of D are eps_i(lambda_l) (H mu)."""
    W = model.w()
    cols = [(W * model.extinction[i][:, None, None] * Hmu).reshape(-1) for i in range(model.extinction.shape[0])]
    A = _stack(np.stack(cols, axis=0)).T                          # [2M, n_species]
    b = _stack((W * y).reshape(-1)[None])[0]
    return np.linalg.lstsq(A, b, rcond=None)[0]


def residual(model: BornModel, c, Hmu, y):
    ebar = c @ model.extinction                                    # [L]
    return model.w() * (y - ebar[:, None, None] * Hmu)


def lm_jacobian(model: BornModel, p, c) -> np.ndarray:
    """J = d eps / d p = -W Ebar H dmu/dp as a real [2M, n_p] matrix (real parts of the M
    complex residuals first, then the imaginary parts)."""
    ebar = c @ model.extinction
    Jc = -(model.w() * ebar[:, None, None])[None] * model.Hjac(p)   # [n_p, L, S, D]
    return _stack(Jc).T


@dataclass
class ReconResult:
    c: np.ndarray
    p: np.ndarray
    misfit_history: list
    outer: int
    lm_steps: int
    stopped_by: str
    seconds: float


def reconstruct(model: BornModel, y: np.ndarray, p0: np.ndarray, c0=None, noise_norm: float = 0.0,
                gamma: float = 1.05, max_outer: int = 20, max_inner: int = 8, fix_c: bool = False,
                lm_nu0: float = 1e-3, rtol: float = 1e-6, damping: str = "identity") -> ReconResult:
    """Alg. opt.  y: [L, S, D] complex data; p0: initial PaLS parameters; noise_norm: ||W eta||
    for the discrepancy principle ||eps|| <= gamma ||W eta|| (0: noise-free, stop on stagnation).
    fix_c: keep c = c0 (shape-only reconstruction, the paper's first experiment).
    damping: "identity" (the printed nu I) or "marquardt" (nu diag(J^T J))."""
    if damping not in ("identity", "marquardt"):
        raise ValueError("damping must be 'identity' or 'marquardt'")
    nu_floor = 1e-12 if damping == "identity" else 1e-6
    t0 = time.perf_counter()
    p = np.array(p0, dtype=np.float64)
    Hmu = model.Hmu(p)
    c = np.array(c0, dtype=np.float64) if c0 is not None else contrast_ls(model, Hmu, y)
    target = gamma * noise_norm
    hist = []
    steps = 0
    stopped = "max_outer"
    f = np.linalg.norm(residual(model, c, Hmu, y))
    nu = None
    for outer in range(max_outer):
        if not fix_c:
            c = contrast_ls(model, Hmu, y)
        r = residual(model, c, Hmu, y)
        f = np.linalg.norm(r)
        hist.append(f)
        if f <= target:
            stopped = "discrepancy"
            break
        f_outer = f
        for _ in range(max_inner):
            J = lm_jacobian(model, p, c)                           # [2M, n_p]
            e = _stack(r.reshape(-1)[None])[0]
            JTJ = J.T @ J
            g = J.T @ e
            if damping == "identity":
                scale = np.eye(JTJ.shape[0])
            else:
                scale = np.diag(np.diag(JTJ))                      # Marquardt's scaling
            if nu is None:
                nu = lm_nu0 * (JTJ.diagonal().max() if damping == "identity" else 1.0)
            accepted = False
            for _try in range(12):                                 # Levenberg-Marquardt damping
                dp = np.linalg.solve(JTJ + nu * scale, -g)
                p_try = p + dp
                Hmu_try = model.Hmu(p_try)
                r_try = residual(model, c, Hmu_try, y)
                f_try = np.linalg.norm(r_try)
                if f_try < f:
                    p, Hmu, r, f = p_try, Hmu_try, r_try, f_try
                    nu = max(nu / 10.0, nu_floor)
                    accepted = True
                    break
                nu *= 10.0
            steps += 1
            hist.append(f)
            if not accepted or f <= target:
                break
        if f <= target:
            stopped = "discrepancy"
            if not fix_c:
                c = contrast_ls(model, Hmu, y)
            break
        if f_outer - f <= rtol * f_outer:
            stopped = "stagnation"
            break
    return ReconResult(c=c, p=p, misfit_history=hist, outer=outer + 1, lm_steps=steps, stopped_by=stopped,
                       seconds=time.perf_counter() - t0)


def shape_errors(mu_true: np.ndarray, mu_rec: np.ndarray, level: float = 0.5):
    """Relative L2 error and the Dice coefficient of the shapes (support: mu > level)."""
    l2 = float(np.linalg.norm(mu_true - mu_rec) / np.linalg.norm(mu_true))
    a, b = mu_true > level, mu_rec > level
    denom = a.sum() + b.sum()
    dice = float(2.0 * np.logical_and(a, b).sum() / denom) if denom else 1.0
    return l2, dice
