"""Born operator products, FP64.

Test infrastructure (see the package docstring); never used by the product.

Under the Born approximation the scattered field at detector d from source s
is minus the volume integral of phi_d * (absorption change) * phi_s
(Sec. 2.1, integral equation derived with the adjoint field).  On the voxel
grid each voxel contributes its volume h^3, so with v the absorption change
per voxel [1/mm] (the factor nu of the paper is divided out with D):

    J_lambda[s, d, k] = -h^3 phi_{s,lambda}(k) phi_{d,lambda}(k)   (no conjugation)

and this is exactly d phi_s(x_d)/d mu_a(k) of the discrete system, since
dA = h^3 diag(d mu_a) and A is complex symmetric.  The adjoint uses the
Hermitian transpose, (J^H w)_k = sum conj(J[l,s,d,k]) w[l,s,d], summed over
wavelengths.

Layouts: phi_s [L][S][N], phi_d [L][D][N], v [n_v][N] real, y [n_v][L][S][D],
w [L][S][D], g [N].
"""
from __future__ import annotations

import numpy as np


def born_matrix(phi_s, phi_d, h):
    """Explicit J as [L*S*D, N] (small grids only)."""
    L, S, N = phi_s.shape
    D = phi_d.shape[1]
    J = -(h ** 3) * phi_s[:, :, None, :] * phi_d[:, None, :, :]
    return J.reshape(L * S * D, N)


def born_apply(phi_s, phi_d, v, h):
    """y[c, l, s, d] = -h^3 sum_k phi_s[l,s,k] v[c,k] phi_d[l,d,k]."""
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    return -(h ** 3) * np.einsum("lsk,ck,ldk->clsd", phi_s, v, phi_d, optimize=True)


def born_apply_adjoint(phi_s, phi_d, w, h):
    """g[k] = sum_{l,s,d} conj(J[l,s,d,k]) w[l,s,d]."""
    return -(h ** 3) * np.einsum("lsk,lsd,ldk->k", np.conj(phi_s), w, np.conj(phi_d), optimize=True)
