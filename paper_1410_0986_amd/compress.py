"""Randomized recursive low-rank compression of the Born operator H (Sec. 4, with the randomized
SVD of the appendix on low-rank representations).

H has one row per measurement and one column per voxel, H[(s, l, d), k] = J_l[s, d, k]
(source s, wavelength l, detector d; rows source-major).  Its row blocks H_s (one per source,
L*D x N) are never formed: the randomized range finder only needs the products H_s Omega and
H_s^H Q, which are the library's Born products with blocks of probe vectors
(``born_apply`` with n_v columns, ``born_apply_adjoint`` with n_w data vectors) on the fields
of source s.  The small dense steps (QR and SVD of matrices with a few dozen columns) run on the
GPU in FP64 through torch.linalg.

* ``bisection_tree``   - the geometric bisection of the source positions on the plate
  (Alg. geom): split the box across its longest side at the midpoint; a part with more than two
  sources is split again.
* ``randsvd``          - adaptive randomized SVD of one row block (Alg. randsvd): rank r from 1,
  incremented by one until the estimate ||A Omega_2 - Q Q^H A Omega_2|| <= eps * S_r(1, 1),
  oversampling p, k estimator columns.
* ``agglomerate``      - two (or more) children H_i ~ U_i V_i^H combine as
  blockdiag(U_i) [V_1^H; V_2^H]; the stacked right factors are recompressed to tolerance eps
  (a truncated SVD through a thin QR) and the left factor is formed explicitly.
* ``recompress``       - the closing step of Sec. 4 (accuracy of the recursion): thin QR of both
  factors, SVD of R_U R_V^H and truncation, which can lower the rank the local truncations left.
* ``compress``         - RecursiveLowRank over the tree (Alg. recursive) followed by
  ``recompress``, returning H ~ U V^H.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _binding as B


# ------------------------------------------------------------------------- tree
def bisection_tree(xy: np.ndarray, lo, hi, indices=None):
    """Alg. geom on the 2-D source positions xy [S, 2] inside the box [lo, hi].

    Returns a node: a list of source indices (a leaf, at most two sources) or a tuple of
    children.  A split that leaves one side empty is not a node: the non-empty side is split
    again inside its half of the box (the sources are distinct, so this ends)."""
    idx = list(range(len(xy))) if indices is None else list(indices)
    lo = np.asarray(lo, dtype=np.float64).copy()
    hi = np.asarray(hi, dtype=np.float64).copy()
    while True:
        if len(idx) <= 2:
            return idx
        j = int(np.argmax(hi - lo))                  # direction of maximum expanse
        if hi[j] - lo[j] <= 1e-12 * max(1.0, abs(hi[j])):
            return idx                               # coincident positions: one leaf
        gamma = 0.5 * (lo[j] + hi[j])
        t1 = [i for i in idx if xy[i, j] <= gamma]
        t2 = [i for i in idx if xy[i, j] > gamma]
        hi1, lo2 = hi.copy(), lo.copy()
        hi1[j] = gamma
        lo2[j] = gamma
        if t1 and t2:
            return (bisection_tree(xy, lo, hi1, t1), bisection_tree(xy, lo2, hi, t2))
        if t1:
            hi = hi1
        else:
            lo = lo2


def tree_leaves(node) -> list:
    """Sources of a node in the order of its row blocks."""
    return list(node) if isinstance(node, list) else [s for ch in node for s in tree_leaves(ch)]


# -------------------------------------------------------------------- products
@dataclass
class BornBlock:
    """Row block H_tau of the Born operator for the sources tau, products through the library."""
    op: B.Operator
    phi_src: torch.Tensor      # [L, S, N] all sources (complex)
    phi_det: torch.Tensor      # [L, D, N]
    sources: list

    @property
    def m(self) -> int:
        return len(self.sources) * self.op.L * self.phi_det.shape[1]

    def _src(self, s):
        return self.phi_src[:, s:s + 1]

    def matmat(self, omega: torch.Tensor) -> torch.Tensor:
        """H_tau @ omega for real omega [N, c] -> [m, c] complex128 (rows (s, l, d))."""
        rdt = torch.float64 if self.phi_src.dtype == torch.complex128 else torch.float32
        out = []
        for s in self.sources:
            cols = []
            for c0 in range(0, omega.shape[1], 64):
                v = omega[:, c0:c0 + 64].T.to(rdt).contiguous()
                y = B.born_apply(self.op, self._src(s), self.phi_det, v)      # [c, L, 1, D]
                cols.append(y.reshape(v.shape[0], -1).T.to(torch.complex128))
            out.append(torch.cat(cols, dim=1))
        return torch.cat(out, dim=0)

    def rmatmat(self, q: torch.Tensor) -> torch.Tensor:
        """H_tau^H @ q for q [m, c] complex -> [N, c] complex128."""
        L, D = self.op.L, self.phi_det.shape[1]
        cdt = torch.complex128 if self.phi_src.dtype == torch.complex128 else torch.complex64
        acc = None
        for a, s in enumerate(self.sources):
            qs = q[a * L * D:(a + 1) * L * D]                              # rows (l, d) of source s
            w = qs.T.reshape(q.shape[1], L, 1, D).to(cdt).contiguous()
            g = B.born_apply_adjoint(self.op, self._src(s), self.phi_det, w)   # [c, N]
            g = g.T.to(torch.complex128)
            acc = g if acc is None else acc + g
        return acc


# ------------------------------------------------------------- randomized SVD
@dataclass
class LowRank:
    """H_tau ~ U V^H with U [m, r] (singular values folded in) and V [N, r] orthonormal columns."""
    U: torch.Tensor
    V: torch.Tensor
    sources: list
    products: int = 0          # columns of H products spent (both directions)
    history: list = field(default_factory=list)

    @property
    def rank(self) -> int:
        return self.U.shape[1]


def randsvd(A: BornBlock, eps: float, omega1: torch.Tensor, omega2: torch.Tensor, p: int = 20,
            chunk: int = 16) -> LowRank:
    """Alg. randsvd on one row block; omega1 [N, >= r+p] and omega2 [N, k] are the test matrices
    (the leading r+p columns of omega1 are used at rank r).  "Increment r" is r + 1: the first
    rank whose error estimate passes is kept.

    The columns Y = A omega1 are computed in blocks of ``chunk`` Born probe vectors and factored
    once per block, Y = Q_Y R_Y (thin QR).  The leading r+p columns are then Q_Y[:, :t] R_Y[:t, :r+p]
    with t = min(rank of Q_Y, r+p), so their left singular vectors are Q_Y[:, :t] times those of
    the small R block, and the estimate ||Z - Q Q^H Z||_2 (Z = A omega2) splits into parts with
    orthogonal column spaces: inside span Q_Y[:, :t], the rest of span Q_Y and its complement."""
    m = A.m
    Z = A.matmat(omega2)                                             # A Omega_2, [m, k]
    used = omega2.shape[1]
    cmax = omega1.shape[1]
    cap = min(m, cmax - p)
    Y = None
    ncols = 0
    r = 1
    hist = []
    while True:
        need = min(r + p, cmax)
        if ncols < need:
            new = min(cmax, max(need, ncols + chunk))
            Yn = A.matmat(omega1[:, ncols:new])
            used += new - ncols
            Y = Yn if Y is None else torch.cat([Y, Yn], dim=1)
            ncols = new
            Qy, Ry = torch.linalg.qr(Y)                             # [m, K], [K, ncols]
            Zc_d = Qy.conj().T @ Z                                   # [K, k]
            Zp = Z - Qy @ Zc_d
            Gp = (Zp.conj().T @ Zp).cpu().numpy()                    # complement of span Q_Y
            Ry_h = Ry.cpu().numpy()
            Zc = Zc_d.cpu().numpy()
        t = min(Ry_h.shape[0], need)
        Ur, Sr, _ = np.linalg.svd(Ry_h[:t, :need], full_matrices=False)
        rr = min(r, Ur.shape[1])
        Ut = Ur[:, :rr]
        Ein = Zc[:t] - Ut @ (Ut.conj().T @ Zc[:t])
        Eout = Zc[t:]
        G = Ein.conj().T @ Ein + Eout.conj().T @ Eout + Gp
        e = float(np.sqrt(max(np.linalg.eigvalsh(G)[-1], 0.0)))
        hist.append((rr, e, float(Sr[0])))
        if e > eps * Sr[0] and rr < cap:
            r += 1
            continue
        Q = Qy[:, :t] @ torch.from_numpy(np.ascontiguousarray(Ut)).to(Qy.device)
        BH = A.rmatmat(Q)                                            # A^H Q = B^H, [N, r]
        used += rr
        U1, S, Vh = torch.linalg.svd(BH.conj().T, full_matrices=False)
        return LowRank(U=(Q @ U1) * S[None, :], V=Vh.conj().T, sources=list(A.sources), products=used, history=hist)


def agglomerate(parts: list, eps: float) -> LowRank:
    """blockdiag(U_i) [V_1^H; V_2^H; ...] recompressed to relative tolerance eps."""
    if len(parts) == 1:
        return parts[0]
    W_H = torch.cat([pt.V for pt in parts], dim=1)                  # [N, sum r_i] = W^H
    Qw, Rw = torch.linalg.qr(W_H)                                  # W = Rw^H Qw^H
    Us, Sw, Vsh = torch.linalg.svd(Rw.conj().T)
    keep = max(1, int((Sw > eps * Sw[0]).sum().item()))
    X = Us[:, :keep] * Sw[None, :keep]                              # W ~ X (Qw Vs)^H
    V = Qw @ Vsh[:keep].conj().T
    rows, off = [], 0
    for pt in parts:                                               # blockdiag(U_i) @ X
        rows.append(pt.U @ X[off:off + pt.rank])
        off += pt.rank
    return LowRank(U=torch.cat(rows, dim=0), V=V, sources=[s for pt in parts for s in pt.sources],
                   products=sum(pt.products for pt in parts))


def recompress(U: torch.Tensor, V: torch.Tensor, eps: float):
    """U V^H -> (Q_U U'_r, Q_V V'_r S'_r): the singular values of R_U R_V^H above eps times the
    largest are kept (folded into the right factor)."""
    Qu, Ru = torch.linalg.qr(U)
    Qv, Rv = torch.linalg.qr(V)
    Up, sp, Vph = torch.linalg.svd(Ru @ Rv.conj().T)
    keep = max(1, int((sp > eps * sp[0]).sum().item()))
    return Qu @ Up[:, :keep], (Qv @ Vph[:keep].conj().T) * sp[None, :keep].to(V.dtype)


# -------------------------------------------------------------------- driver
@dataclass
class CompressedBorn:
    U: torch.Tensor            # [S*L*D, R], rows source-major (s, l, d) in natural source order
    V: torch.Tensor            # [N, R]
    tree: object
    level_ranks: dict          # tree depth -> ranks of the nodes at that depth
    seconds: float
    products: int
    recursive_rank: int = 0    # rank before the closing recompression
    _vtb: torch.Tensor = field(default=None, repr=False)

    @property
    def rank(self) -> int:
        return self.U.shape[1]

    def _vt_blocks(self) -> torch.Tensor:
        """V^T as [nc, R, N/nc] contiguous blocks (built once): the product V^T v then runs as
        a batched GEMM over nc voxel blocks plus a sum, instead of one GEMM with an N-long
        inner dimension and an R x n_v output (too few output tiles to fill the GPU)."""
        if self._vtb is None:
            N, R = self.V.shape
            nc = 64
            while nc > 1 and N % nc:
                nc //= 2
            self._vtb = self.V.T.reshape(R, nc, N // nc).permute(1, 0, 2).contiguous()
        return self._vtb

    def matvec(self, v: torch.Tensor) -> torch.Tensor:
        """H v for real v [n_v, N] -> [n_v, S*L*D] (rows (s, l, d)).  For real v,
        V^H v = conj(V^T v)."""
        if v.is_complex():
            raise ValueError("matvec takes real probe vectors")
        vtb = self._vt_blocks()
        nc, R, nb = vtb.shape
        vb = v.to(vtb.dtype).reshape(v.shape[0], nc, nb).permute(1, 2, 0).contiguous()   # [nc, nb, n_v]
        x = torch.bmm(vtb, vb).sum(dim=0).conj()                                           # V^H v, [R, n_v]
        return (self.U @ x).T


def compress(op: B.Operator, phi_src: torch.Tensor, phi_det: torch.Tensor, src_xy: np.ndarray, eps: float,
             omega1: np.ndarray, omega2: np.ndarray, box_lo=None, box_hi=None, p: int = 20,
             final_recompress: bool = True) -> CompressedBorn:
    """RecursiveLowRank (Alg. recursive) of H over the bisection tree of the source positions.

    omega1 [N, c1] and omega2 [N, k]: Gaussian test matrices shared by every leaf (c1 bounds the
    leaf rank plus oversampling).  box_lo/box_hi: the plate box (default: the sources' bounding box).
    final_recompress: apply ``recompress`` at eps to the root's factors."""
    t0 = time.perf_counter()
    dev = phi_src.device
    lo = src_xy.min(axis=0) if box_lo is None else box_lo
    hi = src_xy.max(axis=0) if box_hi is None else box_hi
    tree = bisection_tree(np.asarray(src_xy, dtype=np.float64), lo, hi)
    o1 = torch.from_numpy(np.ascontiguousarray(omega1)).to(dev)
    o2 = torch.from_numpy(np.ascontiguousarray(omega2)).to(dev)
    levels: dict = {}

    def rec(node, depth):
        if isinstance(node, list):      # leaf: one randomized SVD per source, then agglomerate
            parts = [randsvd(BornBlock(op, phi_src, phi_det, [s]), eps, o1, o2, p) for s in node]
            if len(parts) > 1:
                levels.setdefault(depth + 1, []).extend(pt.rank for pt in parts)
        else:
            parts = [rec(ch, depth + 1) for ch in node]
        out = agglomerate(parts, eps)
        levels.setdefault(depth, []).append(out.rank)
        return out

    lr = rec(tree, 0)
    # row blocks back to the natural source order
    L, D = op.L, phi_det.shape[1]
    blk = L * D
    pos = {s: a for a, s in enumerate(lr.sources)}
    U = torch.cat([lr.U[pos[s] * blk:(pos[s] + 1) * blk] for s in range(len(src_xy))], dim=0)
    V = lr.V
    if final_recompress:
        U, V = recompress(U, V, eps)
    torch.cuda.synchronize(dev)
    return CompressedBorn(U=U, V=V, tree=tree, level_ranks=levels, seconds=time.perf_counter() - t0,
                          products=lr.products, recursive_rank=lr.rank)


def randsvd_direct(op: B.Operator, phi_src: torch.Tensor, phi_det: torch.Tensor, eps: float, omega1: np.ndarray,
                   omega2: np.ndarray, p: int = 20) -> LowRank:
    """The 'direct' comparison of Sec. 4: one adaptive randomized SVD of the whole H."""
    dev = phi_src.device
    o1 = torch.from_numpy(np.ascontiguousarray(omega1)).to(dev)
    o2 = torch.from_numpy(np.ascontiguousarray(omega2)).to(dev)
    return randsvd(BornBlock(op, phi_src, phi_det, list(range(phi_src.shape[1]))), eps, o1, o2, p)
