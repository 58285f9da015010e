"""Recursive randomized compression of H on the GPU (products through the library) against the
oracle's dense implementation with the same Gaussian test matrices: the same tree, the same
ranks, the same low-rank blocks; and the blocked adjoint product it relies on."""
import numpy as np
import pytest
import torch

import workloads
from oracle import born as oborn
from oracle import compress as ocompress
from oracle import fields as ofields

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


@pytest.fixture(scope="module")
def case():
    w = workloads.config("tiny", n_lambda=3)
    return w, ofields.solve_banded(w)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
@pytest.mark.parametrize("n_w", [1, 3, 6])
def test_adjoint_block(hd, case, dtype, tol, n_w):
    w, P = case
    S = w.S
    t = torch.from_numpy(P).to(dtype).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(n_w)
    W = rng.standard_normal((n_w, w.L, S, w.D)) + 1j * rng.standard_normal((n_w, w.L, S, w.D))
    g = hd.born_apply_adjoint(hd_op(hd, w), t[:, :S], t[:, S:], torch.from_numpy(W).to(DEV)).cpu().numpy()
    assert g.shape == (n_w, w.N)
    for c in range(n_w):
        ref = oborn.born_apply_adjoint(Pr[:, :S], Pr[:, S:], W[c], w.h)
        assert np.linalg.norm(g[c] - ref) <= tol * np.linalg.norm(ref)


_ops = {}


def hd_op(hd, w):
    key = (w.nx, w.ny, w.nz, w.L)
    if key not in _ops:
        _ops[key] = hd.Operator.from_workload(w)
    return _ops[key]


def _oracle(w, P, eps, om1, om2):
    S = w.S
    J = oborn.born_matrix(P[:, :S], P[:, S:], w.h).reshape(w.L, S, w.D, w.N)
    blocks = [J[:, s].reshape(w.L * w.D, w.N) for s in range(S)]
    xy = workloads.optode_xy(w, w.src_voxels)
    tree = ocompress.split(xy, range(S), xy.min(axis=0), xy.max(axis=0))
    ranks = {}
    U, V, order = ocompress.recursive(blocks, tree, eps, om1, om2, ranks=ranks)
    H = np.concatenate(blocks, axis=0)
    pos = {s: a for a, s in enumerate(order)}
    blk = w.L * w.D
    Un = np.concatenate([U[pos[s] * blk:(pos[s] + 1) * blk] for s in range(S)], axis=0)
    Ur, Vr = ocompress.recompress(Un, V, eps)
    return tree, ranks, (Un @ V.conj().T, U.shape[1]), (Ur @ Vr.conj().T, Ur.shape[1]), H


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_compression_matches_oracle_fp64(hd, case, eps):
    from paper_1410_0986_amd import compress
    w, P = case
    S = w.S
    om1, om2 = workloads.gaussian_test_matrix(w.N, 40), workloads.gaussian_test_matrix(w.N, 10, seed=5)
    tree, ranks, (UVo, ro), (UVf, rf), H = _oracle(w, P, eps, om1, om2)
    t = torch.from_numpy(P).to(DEV)
    xy = workloads.optode_xy(w, w.src_voxels)
    op = hd_op(hd, w)
    cb = compress.compress(op, t[:, :S], t[:, S:], xy, eps, om1, om2, final_recompress=False)
    assert cb.tree == tree
    assert {k: sorted(v) for k, v in cb.level_ranks.items()} == {k: sorted(v) for k, v in ranks.items()}
    assert cb.rank == ro
    UV = (cb.U @ cb.V.conj().T).cpu().numpy()
    assert np.linalg.norm(UV - UVo) <= 1e-9 * np.linalg.norm(UVo)
    assert np.linalg.norm(H - UV, 2) <= 10 * eps * np.linalg.norm(H, 2)
    cf = compress.compress(op, t[:, :S], t[:, S:], xy, eps, om1, om2)       # with the closing recompression
    assert cf.rank == rf and cf.recursive_rank == ro and rf <= ro
    UV = (cf.U @ cf.V.conj().T).cpu().numpy()
    assert np.linalg.norm(UV - UVf) <= 1e-9 * np.linalg.norm(UVf)
    assert np.linalg.norm(H - UV, 2) <= 10 * eps * np.linalg.norm(H, 2)


def test_compression_fp32_fields_meets_tolerance(hd, case):
    from paper_1410_0986_amd import compress
    w, P = case
    S = w.S
    eps = 1e-4
    om1, om2 = workloads.gaussian_test_matrix(w.N, 40), workloads.gaussian_test_matrix(w.N, 10, seed=5)
    t = torch.from_numpy(P).to(torch.complex64).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    J = oborn.born_matrix(Pr[:, :S], Pr[:, S:], w.h).reshape(w.L, S, w.D, w.N)
    H = np.concatenate([J[:, s].reshape(w.L * w.D, w.N) for s in range(S)], axis=0)
    xy = workloads.optode_xy(w, w.src_voxels)
    cb = compress.compress(hd_op(hd, w), t[:, :S], t[:, S:], xy, eps, om1, om2)
    UV = (cb.U @ cb.V.conj().T).cpu().numpy()
    assert np.linalg.norm(H - UV, 2) <= 10 * eps * np.linalg.norm(H, 2)
    # the compressed operator applied to probe vectors
    v = workloads.born_v(w, n_v=2)
    y = cb.matvec(torch.from_numpy(v).to(DEV)).cpu().numpy()
    assert np.linalg.norm(y - (H @ v.T).T) <= 10 * eps * np.linalg.norm(H @ v.T)
