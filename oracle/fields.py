"""Fields phi_{r,lambda} = A(lambda)^-1 b_r for every right-hand side and wavelength.

Test infrastructure (see the package docstring); never used by the product.

The paper's Algorithm 1 (augmented GMRES with a recycled deflation space,
Sec. 3.1) converges to exactly this solution up to its tolerance, so the
oracle uses the plain definition and several independent routes to it:

* ``solve_dense``     - LU of the assembled matrix (small grids);
* ``solve_banded``    - banded LU with the largest axis slowest;
  both also take ``pert = (shape, scale)``, the heterogeneous absorption
  mu_a(k) + scale_j shape(k) of the full (nonlinear) forward model;
* ``solve_separable`` - fast diagonalisation of the homogeneous box
                        (Lynch, Rice and Thomas 1964): exact at any size, and
                        ``separable_at`` evaluates single points cheaply;
* ``gmres``           - textbook restarted GMRES(m) (Saad and Schultz 1986),
                        unrecycled, unpreconditioned, MGS with one
                        re-orthogonalisation, complex Givens rotations;
* ``precond_solve``   - (K_hat + sigma I)^-1 x in the scaled form of eq.
                        multipleshifted: the matrix a preconditioner replacing the
                        paper's ILU of the mean-shifted K (Sec. 6.1) inverts, by
                        sparse LU of the assembled matrix.

Output layout: [L][R][N] complex128 with N contiguous.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import model


def _rhs_list(w, voxels):
    return w.rhs_voxels if voxels is None else np.asarray(voxels, dtype=np.int64)


def _lams(w, lam_idx):
    return range(w.L) if lam_idx is None else list(lam_idx)


def _op(w, j, pert):
    """A(lambda_j), or its heterogeneous-absorption form for pert = (shape, scale)."""
    return model.operator(w, j) if pert is None else model.operator_perturbed(w, j, *pert)


def solve_dense(w, voxels=None, lam_idx=None, pert=None) -> np.ndarray:
    vox = _rhs_list(w, voxels)
    lams = _lams(w, lam_idx)
    out = np.empty((len(lams), len(vox), w.N), dtype=np.complex128)
    Bm = np.zeros((w.N, len(vox)), dtype=np.complex128)
    Bm[vox, np.arange(len(vox))] = 1.0
    for a, j in enumerate(lams):
        A = _op(w, j, pert).toarray()
        out[a] = np.linalg.solve(A, Bm).T
    return out


def _band_permutation(w):
    """Axis order (fastest first) putting the largest dimension slowest."""
    dims = [w.nx, w.ny, w.nz]
    order = sorted(range(3), key=lambda a: dims[a])          # ascending size
    # new index = i_o0 + d_o0*(i_o1 + d_o1*i_o2)
    k, j, i = np.meshgrid(np.arange(w.nz), np.arange(w.ny), np.arange(w.nx), indexing="ij")
    idx = [i.reshape(-1), j.reshape(-1), k.reshape(-1)]
    new = idx[order[0]] + dims[order[0]] * (idx[order[1]] + dims[order[1]] * idx[order[2]])
    bw = dims[order[0]] * dims[order[1]]
    return new, bw


def solve_banded(w, voxels=None, lam_idx=None, pert=None) -> np.ndarray:
    vox = _rhs_list(w, voxels)
    lams = _lams(w, lam_idx)
    new, bw = _band_permutation(w)
    out = np.empty((len(lams), len(vox), w.N), dtype=np.complex128)
    Bm = np.zeros((w.N, len(vox)), dtype=np.complex128)
    Bm[new[vox], np.arange(len(vox))] = 1.0
    for a, j in enumerate(lams):
        A = _op(w, j, pert).tocoo()
        r, c = new[A.row], new[A.col]
        ab = np.zeros((2 * bw + 1, w.N), dtype=np.complex128)
        ab[bw + r - c, c] = A.data
        sol = sla.solve_banded((bw, bw), ab, Bm)
        out[a] = sol[new, :].T
    return out


def _axis_eigs(w, D):
    """Eigen-decomposition of T_axis = D h L_axis + h^2/(2 A_R) E_axis for x, y, z."""
    res = []
    for L1, E1 in model.axis_terms(w):
        T = D * w.h * L1.toarray() + (w.h ** 2 / (2.0 * w.A_R)) * np.diag(E1)
        ev, Q = np.linalg.eigh(T)
        res.append((ev, Q))
    return res


def solve_separable(w, voxels=None, lam_idx=None) -> np.ndarray:
    """A = T_x (+) T_y (+) T_z + s h^3 I on the box, diagonalised axis by axis."""
    vox = _rhs_list(w, voxels)
    lams = _lams(w, lam_idx)
    D, _, s = model.optics(w)
    out = np.empty((len(lams), len(vox), w.N), dtype=np.complex128)
    for a, j in enumerate(lams):
        (ex, Qx), (ey, Qy), (ez, Qz) = _axis_eigs(w, D[j])
        denom = ez[:, None, None] + ey[None, :, None] + ex[None, None, :] + s[j] * w.h ** 3
        for r, v in enumerate(vox):
            i0 = v % w.nx
            j0 = (v // w.nx) % w.ny
            k0 = v // (w.nx * w.ny)
            c = (Qz[k0][:, None, None] * Qy[j0][None, :, None] * Qx[i0][None, None, :]) / denom
            phi = np.einsum("kc,cba->kba", Qz, c)
            phi = np.einsum("jb,kba->kja", Qy, phi)
            phi = np.einsum("ia,kja->kji", Qx, phi)
            out[a, r] = phi.reshape(-1)
    return out


def separable_at(w, lam_idx: int, src_voxel: int, points) -> np.ndarray:
    """phi(points) for one source and wavelength, each point by its own O(N) eigen-sum."""
    D, _, s = model.optics(w)
    (ex, Qx), (ey, Qy), (ez, Qz) = _axis_eigs(w, D[lam_idx])
    denom = ez[:, None, None] + ey[None, :, None] + ex[None, None, :] + s[lam_idx] * w.h ** 3
    i0 = src_voxel % w.nx
    j0 = (src_voxel // w.nx) % w.ny
    k0 = src_voxel // (w.nx * w.ny)
    src = Qz[k0][:, None, None] * Qy[j0][None, :, None] * Qx[i0][None, None, :] / denom
    out = []
    for p in np.asarray(points, dtype=np.int64).reshape(-1):
        i = p % w.nx
        j = (p // w.nx) % w.ny
        k = p // (w.nx * w.ny)
        tgt = Qz[k][:, None, None] * Qy[j][None, :, None] * Qx[i][None, None, :]
        out.append(np.sum(tgt * src))
    return np.asarray(out, dtype=np.complex128)


def gmres(A, b, tol=1e-10, m=30, max_iter=20000, x0=None):
    """Restarted GMRES(m), no preconditioner; stops on ||b - A x||/||b|| <= tol.

    Returns (x, total inner iterations, final true relative residual).
    """
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n, dtype=np.complex128), 0, 0.0
    iters = 0
    r = b - A @ x
    beta = np.linalg.norm(r)
    while beta / bnorm > tol and iters < max_iter:
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            wv = A @ V[j]
            for _ in range(2):                      # MGS, then one re-orthogonalisation
                for i in range(j + 1):
                    hij = np.vdot(V[i], wv)
                    H[i, j] += hij
                    wv = wv - hij * V[i]
            H[j + 1, j] = np.linalg.norm(wv)
            if H[j + 1, j] != 0.0:
                V[j + 1] = wv / H[j + 1, j]
            for i in range(j):                      # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            rr = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / rr
                sn[j] = (a / abs(a)) * np.conj(bb) / rr
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k_used = j + 1
            if abs(g[j + 1]) / bnorm <= tol or iters >= max_iter:
                break
        y = sla.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + V[:k_used].T @ y
        r = b - A @ x
        beta = np.linalg.norm(r)
    return x, iters, float(beta / bnorm)


def solve_gmres(w, voxels=None, lam_idx=None, tol=1e-10, m=30, max_iter=20000):
    """Unrecycled GMRES(m) for every (wavelength, right-hand side); returns (phi, iters, relres)."""
    vox = _rhs_list(w, voxels)
    lams = _lams(w, lam_idx)
    out = np.empty((len(lams), len(vox), w.N), dtype=np.complex128)
    its = np.zeros((len(lams), len(vox)), dtype=np.int64)
    rel = np.zeros((len(lams), len(vox)))
    for a, j in enumerate(lams):
        A = model.operator(w, j)
        for r, v in enumerate(vox):
            x, it, rr = gmres(A, model.rhs(w, v), tol=tol, m=m, max_iter=max_iter)
            out[a, r], its[a, r], rel[a, r] = x, it, rr
    return out, its, rel


def precond_solve(w, x, sigp_star: float, sigma: complex) -> np.ndarray:
    """y = (K / h^3 + sigp_star B / h^3 + sigma I)^-1 x for x [count, N] (the scaled form
    A(lambda_j) / (D_j h^3) = K / h^3 + sigma'_j B / h^3 + sigma_j I with sigma'_j replaced by
    sigp_star; Sec. 3.1 and the mean-shift transform of Sec. 6.1)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    h3 = w.h ** 3
    P = (model.assemble_K(w) / h3 + (sigp_star / h3) * model.assemble_B(w)
         + sigma * sp.identity(w.N, format="csc")).astype(np.complex128).tocsc()
    lu = spl.splu(P)
    x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
    return np.stack([lu.solve(v) for v in x])
