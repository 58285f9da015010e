"""Recursive randomized compression of an explicit Born matrix (Sec. 4, appendix on low-rank
representations), written out on dense numpy arrays.

Test infrastructure (see the package docstring); never used by the product.

* ``split``        - Alg. geom (geometric bisection of the source positions);
* ``randsvd``      - Alg. randsvd (adaptive randomized SVD, Halko, Martinsson and Tropp 2011),
                     with the same test-matrix convention as the library: the leading r + p
                     columns of one Gaussian matrix Omega_1 at rank r, and Omega_2 fixed;
* ``agglomerate``  - blockdiag(U_i) [V_1^H; V_2^H] with the stacked right factors truncated
                     by a full SVD at relative tolerance eps;
* ``recursive``    - Alg. recursive over the tree;
* ``recompress``   - the closing recompression of U V^H (Sec. 4, accuracy of the recursion):
                     thin QR of both factors, SVD of R_U R_V^H, truncation at eps.

Readings shared with the library: "increment r" is r + 1 (the first rank whose error estimate
passes is kept), a leaf of the tree (at most two sources) factors each source's block and then
agglomerates them, and the initial box is the sources' bounding box.
"""
from __future__ import annotations

import numpy as np


def split(points, idx, lo, hi):
    """Tree over the sources idx inside [lo, hi]: a leaf is a list (<= 2 sources), an inner
    node a tuple of its two parts."""
    idx = list(idx)
    if len(idx) <= 2:
        return idx
    lo = np.array(lo, dtype=float)
    hi = np.array(hi, dtype=float)
    widths = hi - lo
    j = int(np.argmax(widths))
    if widths[j] <= 1e-12 * max(1.0, abs(hi[j])):
        return idx
    mid = (lo[j] + hi[j]) / 2.0
    left = [i for i in idx if points[i][j] <= mid]
    right = [i for i in idx if points[i][j] > mid]
    hi_left = hi.copy()
    hi_left[j] = mid
    lo_right = lo.copy()
    lo_right[j] = mid
    if not left:
        return split(points, right, lo_right, hi)
    if not right:
        return split(points, left, lo, hi_left)
    return (split(points, left, lo, hi_left), split(points, right, lo_right, hi))


def randsvd(A, eps, omega1, omega2, p=20):
    """Adaptive randomized SVD of the dense A [m, n]; returns (U S, V, rank history)."""
    m = A.shape[0]
    Z = A @ omega2
    r = 1
    hist = []
    while True:
        Y = A @ omega1[:, :min(r + p, omega1.shape[1])]
        Uy, sy, _ = np.linalg.svd(Y, full_matrices=False)
        rr = min(r, Uy.shape[1])
        Q = Uy[:, :rr]
        err = np.linalg.norm(Z - Q @ (Q.conj().T @ Z), 2)
        hist.append((rr, err, sy[0]))
        if err > eps * sy[0] and rr < min(m, omega1.shape[1] - p):
            r += 1
            continue
        Bm = Q.conj().T @ A
        U1, s, Vh = np.linalg.svd(Bm, full_matrices=False)
        return (Q @ U1) * s[None, :], Vh.conj().T, hist


def agglomerate(parts, eps):
    """parts: list of (U_i, V_i) with block i ~ U_i V_i^H; returns (U, V) for the stacked blocks."""
    if len(parts) == 1:
        return parts[0]
    W = np.concatenate([V.conj().T for _, V in parts], axis=0)     # [sum r_i, n]
    Uw, sw, Vwh = np.linalg.svd(W, full_matrices=False)
    keep = max(1, int(np.sum(sw > eps * sw[0])))
    X = Uw[:, :keep] * sw[None, :keep]
    blocks, off = [], 0
    for U, _ in parts:
        r = U.shape[1]
        blocks.append(U @ X[off:off + r])
        off += r
    return np.concatenate(blocks, axis=0), Vwh[:keep].conj().T


def recursive(blocks, node, eps, omega1, omega2, p=20, ranks=None):
    """Alg. recursive: blocks[s] is the dense row block of source s.  Returns (U, V, sources in
    row order); ranks, if a dict, collects the rank of every node by tree depth."""
    def go(nd, depth):
        if isinstance(nd, list):
            parts = []
            for s in nd:
                U, V, _ = randsvd(blocks[s], eps, omega1, omega2, p)
                parts.append((U, V))
            if ranks is not None and len(parts) > 1:
                ranks.setdefault(depth + 1, []).extend(U.shape[1] for U, _ in parts)
            order = list(nd)
        else:
            res = [go(ch, depth + 1) for ch in nd]
            parts = [(U, V) for U, V, _ in res]
            order = [s for _, _, o in res for s in o]
        U, V = agglomerate(parts, eps)
        if ranks is not None:
            ranks.setdefault(depth, []).append(U.shape[1])
        return U, V, order
    return go(node, 0)


def recompress(U, V, eps):
    """U V^H -> (Q_U U'_r, Q_V V'_r S'_r) keeping the singular values of R_U R_V^H above
    eps times the largest."""
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    Up, sp, Vph = np.linalg.svd(Ru @ Rv.conj().T)
    keep = max(1, int(np.sum(sp > eps * sp[0])))
    return Qu @ Up[:, :keep], (Qv @ Vph[:keep].conj().T) * sp[None, :keep]
