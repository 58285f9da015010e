"""Host logic of the library's randomized SVD (Alg. randsvd) on a dense stand-in for a Born row
block, against the oracle's literal loop: the same rank sequence (r incremented by one), the
same first passing rank and the same factorization.  Runs on the CPU (torch CPU tensors); the
Born products themselves are covered by the GPU compression tests."""
import numpy as np
import pytest
import torch

import workloads
from oracle import compress as ocompress


class _Dense:
    """A.matmat / A.rmatmat of an explicit complex matrix, the interface of a Born row block."""

    def __init__(self, A):
        self.A = torch.from_numpy(A)
        self.m = A.shape[0]
        self.sources = [0]

    def matmat(self, om):
        return self.A @ om.to(torch.complex128)

    def rmatmat(self, q):
        return self.A.conj().T @ q


def _cases():
    rng = np.random.default_rng(11)
    m, n = 70, 300
    Qa, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    Qb, _ = np.linalg.qr(rng.standard_normal((n, m)))
    yield "decaying", (Qa * 0.6 ** np.arange(m)) @ Qb.T
    r = 6
    yield "rank6", (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) @ rng.standard_normal((r, n))


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_library_randsvd_matches_oracle_loop(eps):
    from paper_1410_0986_amd import compress
    for name, A in _cases():
        n = A.shape[1]
        om1 = workloads.gaussian_test_matrix(n, 90, seed=7)
        om2 = workloads.gaussian_test_matrix(n, 10, seed=8)
        Uo, Vo, hist_o = ocompress.randsvd(A, eps, om1, om2)
        lr = compress.randsvd(_Dense(A), eps, torch.from_numpy(om1), torch.from_numpy(om2), chunk=7)
        assert [h[0] for h in lr.history] == [h[0] for h in hist_o], name
        np.testing.assert_allclose([h[1] for h in lr.history], [h[1] for h in hist_o], rtol=1e-6,
                                   atol=1e-12 * hist_o[0][2])
        assert lr.rank == Uo.shape[1]
        Ml = (lr.U @ lr.V.conj().T).numpy()
        assert np.linalg.norm(Ml - Uo @ Vo.conj().T) <= 1e-9 * np.linalg.norm(A)
