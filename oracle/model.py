"""Optical model and discrete operator, written out as sparse matrices.

Test infrastructure (see the package docstring); never used by the product.

Discretisation (cell-centred finite volume on a box of nx*ny*nz voxels of
edge h, index n = i + nx*(j + ny*k)):

* K: (K phi)_n = h * sum over face neighbours m inside the grid of (phi_n - phi_m),
  plus 2h*phi_n for each exterior face held at zero (Dirichlet, eq. dirichlet,
  ghost value -phi_n);
* B = diag(h^2 f_n), f_n = number of exterior Robin faces of voxel n; the flux
  through such a face is phi_n h^2/(2 A_R), the first-order form of the Robin
  condition phi + 2 A D dphi/dn = 0 (eq. robin);
* M = h^3 I (lumped mass, Sec. 3.1);
* A(lambda) = D_lambda K + B/(2 A_R) + (mu_a(lambda) + i omega/nu) M.

This is the frequency-domain form of the diffusion equation (eq. diffusion)
with the shifted structure of eq. multipleshifted: after dividing by
D_lambda h^3, A = D h^3 [K/h^3 + sigma' B/h^3 + sigma I] with
sigma = (mu_a + i omega/nu)/D and sigma' = 1/(2 A_R D).

Optical model (Sec. 2.1): D = 1/(3 mu_s'), with nu divided out as in the
diffusion equation after division by nu; mu_a(lambda) = sum_l c_l eps_l(lambda)
(eq. perturbation, here for the homogeneous background).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def optics(w):
    """Per-wavelength D [mm], mu_a [1/mm] and complex absorption s = mu_a + i omega/nu."""
    D = 1.0 / (3.0 * np.asarray(w.mus_prime, dtype=np.float64))
    mua = np.asarray(w.conc_uM, dtype=np.float64) @ np.asarray(w.extinction, dtype=np.float64)
    s = mua + 1j * w.omega_over_nu
    return D, mua, s


def shifts(w):
    """Shift form (Sec. 3.1): sigma_j = s_j/D_j, sigma'_j = 1/(2 A_R D_j)."""
    D, _, s = optics(w)
    return s / D, 1.0 / (2.0 * w.A_R * D)


def _face_bits(robin_faces: int, axis: int):
    lo = (robin_faces >> (2 * axis)) & 1
    hi = (robin_faces >> (2 * axis + 1)) & 1
    return bool(lo), bool(hi)


def path_laplacian(n: int, dirichlet_lo: bool, dirichlet_hi: bool) -> sp.csr_matrix:
    """1-D graph Laplacian of a path of n cells (no flux out), plus 2 per Dirichlet end."""
    main = np.zeros(n)
    if n > 1:
        main[:] = 2.0
        main[0] = 1.0
        main[-1] = 1.0
    if dirichlet_lo:
        main[0] += 2.0
    if dirichlet_hi:
        main[-1] += 2.0
    off = -np.ones(max(n - 1, 0))
    return sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="csr")


def end_indicator(n: int, lo: bool, hi: bool) -> np.ndarray:
    e = np.zeros(n)
    if lo:
        e[0] += 1.0
    if hi:
        e[-1] += 1.0
    return e


def _dims(w):
    return (w.nx, w.ny, w.nz)


def axis_terms(w):
    """Per-axis (path Laplacian incl. Dirichlet ends, Robin end indicator), axes x, y, z."""
    out = []
    for axis, n in enumerate(_dims(w)):
        rlo, rhi = _face_bits(w.robin_faces, axis)
        out.append((path_laplacian(n, not rlo, not rhi), end_indicator(n, rlo, rhi)))
    return out


def _kron_sum(mats_xyz):
    """Sum over axes of I (x) ... (x) M_axis (x) ... with z slowest, x fastest."""
    nx, ny, nz = (m.shape[0] for m in mats_xyz)
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    Mx, My, Mz = mats_xyz
    return (sp.kron(Iz, sp.kron(Iy, Mx)) + sp.kron(Iz, sp.kron(My, Ix))
            + sp.kron(Mz, sp.kron(Iy, Ix))).tocsr()


def assemble_K(w) -> sp.csr_matrix:
    """Stiffness K (face-weight h 7-point Laplacian with Dirichlet end terms)."""
    terms = axis_terms(w)
    return (w.h * _kron_sum([t[0] for t in terms])).tocsr()


def robin_face_count(w) -> np.ndarray:
    """f_n: number of exterior Robin faces of each voxel, flattened with x fastest."""
    terms = axis_terms(w)
    ex, ey, ez = (t[1] for t in terms)
    f = ez[:, None, None] + ey[None, :, None] + ex[None, None, :]
    return f.reshape(-1)


def assemble_B(w) -> sp.csr_matrix:
    return sp.diags(w.h ** 2 * robin_face_count(w), 0, format="csr")


def operator(w, lam_idx: int) -> sp.csr_matrix:
    """A(lambda_j) as a complex sparse matrix."""
    D, _, s = optics(w)
    K = assemble_K(w)
    B = assemble_B(w)
    I = sp.identity(w.N, format="csr")
    return (D[lam_idx] * K + B / (2.0 * w.A_R) + (s[lam_idx] * w.h ** 3) * I).astype(np.complex128).tocsr()


def operator_perturbed(w, lam_idx: int, shape, scale) -> sp.csr_matrix:
    """A(lambda_j) for the heterogeneous absorption mu_a(k) = mu_a(lambda_j) + scale_j * shape(k)
    (Sec. 2.1 diffusion equation with mu_a varying in space; eq. perturbation): the absorption
    term integrated over each voxel adds h^3 * scale_j * shape(k) to the diagonal."""
    extra = w.h ** 3 * float(scale[lam_idx]) * np.asarray(shape, dtype=np.float64)
    return (operator(w, lam_idx) + sp.diags(extra.astype(np.complex128), 0)).tocsr()


def rhs(w, voxel: int) -> np.ndarray:
    """Unit injection into one voxel (S = S0 delta(r - r_s) with S0 = 1)."""
    b = np.zeros(w.N, dtype=np.complex128)
    b[int(voxel)] = 1.0
    return b


def voxel_centres(w) -> np.ndarray:
    """[N, 3] voxel centre coordinates in mm, x fastest."""
    k, j, i = np.meshgrid(np.arange(w.nz), np.arange(w.ny), np.arange(w.nx), indexing="ij")
    return np.stack([(i.reshape(-1) + 0.5) * w.h, (j.reshape(-1) + 0.5) * w.h,
                     (k.reshape(-1) + 0.5) * w.h], axis=1)


def relative_residual(w, lam_idx: int, voxel: int, phi: np.ndarray, pert=None) -> float:
    """||b - A phi||_2 / ||b||_2 of the unscaled system (pert = (shape, scale) for the
    heterogeneous operator)."""
    A = operator(w, lam_idx) if pert is None else operator_perturbed(w, lam_idx, *pert)
    b = rhs(w, voxel)
    return float(np.linalg.norm(b - A @ phi) / np.linalg.norm(b))
