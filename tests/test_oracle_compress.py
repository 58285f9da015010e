"""Pins of the oracle's recursive randomized compression (oracle/compress.py): the tree of the
paper's five-source figure, exact recovery of low-rank matrices, agglomeration, and the recursive
factorization of an explicit Born matrix against a textbook SVD."""
import numpy as np
import pytest

import workloads
from oracle import born, compress, fields


def leaves(node):
    return list(node) if isinstance(node, list) else [s for ch in node for s in leaves(ch)]


def test_split_reproduces_the_five_source_figure():
    # sources 1..5 (0-based 0..4) placed so that the bisection gives {1,2} | {3,4,5}, then {3,4} | {5}
    pts = np.array([[0.5, 0.5], [1.5, 1.5], [2.5, 0.5], [2.8, 0.7], [3.5, 1.8]])
    tree = compress.split(pts, range(5), [0.0, 0.0], [4.0, 2.0])
    assert tree == ([0, 1], ([2, 3], [4]))


def test_split_of_a_uniform_array():
    w = workloads.config("medium")
    xy = workloads.optode_xy(w, w.src_voxels)                       # 4 x 4 sources
    tree = compress.split(xy, range(16), xy.min(axis=0), xy.max(axis=0))

    def depth(nd):
        return 0 if isinstance(nd, list) else 1 + max(depth(c) for c in nd)

    assert sorted(leaves(tree)) == list(range(16))
    assert depth(tree) == 3                                         # log2(16) - 1 levels of splits
    stack = [tree]
    while stack:
        nd = stack.pop()
        if isinstance(nd, list):
            assert 1 <= len(nd) <= 2
            # the two sources of a leaf are neighbours on the plate
            if len(nd) == 2:
                assert np.linalg.norm(xy[nd[0]] - xy[nd[1]]) <= 32.0 + 1e-9
        else:
            stack.extend(nd)


def test_randsvd_recovers_exact_low_rank():
    rng = np.random.default_rng(1)
    m, n, r = 60, 300, 5
    A = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) @ rng.standard_normal((r, n))
    om1, om2 = workloads.gaussian_test_matrix(n, 80, seed=7), workloads.gaussian_test_matrix(n, 10, seed=8)
    U, V, hist = compress.randsvd(A, 1e-8, om1, om2)
    assert U.shape[1] == r                                          # the first rank that passes
    assert np.linalg.norm(A - U @ V.conj().T, 2) <= 1e-10 * np.linalg.norm(A, 2)
    assert [h[0] for h in hist] == list(range(1, r + 1))            # r incremented by one
    assert all(h[1] > 1e-8 * h[2] for h in hist[:-1])


def test_randsvd_meets_tolerance_on_decaying_spectrum():
    rng = np.random.default_rng(2)
    m, n = 80, 400
    Qa, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    Qb, _ = np.linalg.qr(rng.standard_normal((n, m)))
    s = 0.5 ** np.arange(m)
    A = (Qa * s) @ Qb.T
    om1, om2 = workloads.gaussian_test_matrix(n, 80, seed=9), workloads.gaussian_test_matrix(n, 10, seed=10)
    for eps in (1e-3, 1e-6):
        U, V, _ = compress.randsvd(A, eps, om1, om2)
        assert np.linalg.norm(A - U @ V.conj().T, 2) <= 10 * eps * s[0]
        # the rank is the epsilon-rank of the block up to the slack of the randomized estimate
        # (a few singular values, each a factor 2 here), not up to a factor 2 of it
        eps_rank = int(np.sum(s > eps * s[0]))
        assert eps_rank - 3 <= U.shape[1] <= eps_rank + 3


def test_agglomerate_two_blocks():
    rng = np.random.default_rng(3)
    n = 200
    base = rng.standard_normal((4, n))                              # shared row space
    A1 = rng.standard_normal((30, 4)) @ base
    A2 = rng.standard_normal((20, 4)) @ base
    p1 = np.linalg.svd(A1, full_matrices=False)
    p2 = np.linalg.svd(A2, full_matrices=False)
    parts = [((p[0][:, :4] * p[1][:4]), p[2][:4].conj().T) for p in (p1, p2)]
    U, V = compress.agglomerate(parts, 1e-10)
    assert U.shape[1] == 4                                          # 4 + 4 columns agglomerate to 4
    A = np.vstack([A1, A2])
    assert np.linalg.norm(A - U @ V.conj().T) <= 1e-10 * np.linalg.norm(A)


def test_recursive_compression_of_born_matrix_against_svd():
    w = workloads.config("tiny", n_lambda=3)
    P = fields.solve_banded(w)
    S = w.S
    J = born.born_matrix(P[:, :S], P[:, S:], w.h).reshape(w.L, S, w.D, w.N)
    blocks = [J[:, s].reshape(w.L * w.D, w.N) for s in range(S)]     # H_s, rows (l, d)
    H = np.concatenate(blocks, axis=0)
    xy = workloads.optode_xy(w, w.src_voxels)
    tree = compress.split(xy, range(S), xy.min(axis=0), xy.max(axis=0))
    om1, om2 = workloads.gaussian_test_matrix(w.N, 40), workloads.gaussian_test_matrix(w.N, 10, seed=5)
    sH = np.linalg.svd(H, compute_uv=False)
    for eps in (1e-2, 1e-4):
        U, V, order = compress.recursive(blocks, tree, eps, om1, om2)
        Hr = np.concatenate([blocks[s] for s in order], axis=0)
        assert np.linalg.norm(Hr - U @ V.conj().T, 2) <= 10 * eps * sH[0]
        eps_rank = int(np.sum(sH > eps * sH[0]))
        assert U.shape[1] <= 2 * eps_rank + 4


def test_recompress_is_the_truncated_svd_of_the_product():
    """The QR-based recompression must give the best rank-k approximation of U V^H, i.e. the
    dense product's own truncated SVD (a textbook routine on the formed matrix)."""
    rng = np.random.default_rng(4)
    m, n, r = 90, 150, 24
    s = 10.0 ** -np.linspace(0, 8, r)
    U = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) * s[None, :]
    V = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    A = U @ V.conj().T
    Ua, sa, Vah = np.linalg.svd(A, full_matrices=False)
    for eps in (1e-3, 1e-6):
        U2, V2 = compress.recompress(U, V, eps)
        k = int(np.sum(sa > eps * sa[0]))
        assert U2.shape[1] == k
        best = (Ua[:, :k] * sa[:k]) @ Vah[:k]
        assert np.linalg.norm(U2 @ V2.conj().T - best) <= 1e-9 * sa[0]
        np.testing.assert_allclose(U2.conj().T @ U2, np.eye(k), atol=1e-12)
        np.testing.assert_allclose(np.linalg.norm(V2, axis=0), sa[:k], rtol=1e-9)
