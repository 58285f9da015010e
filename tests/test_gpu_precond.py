"""Separable right preconditioner (a GPU replacement for the ILU of the mean-shifted matrix,
Sec. 6.1): the stand-alone application against the oracle's sparse LU of the same matrix, and
the preconditioned batched solve against the oracle fields (homogeneous and heterogeneous
absorption, every shift variant), with the drop in Arnoldi steps."""
import numpy as np
import pytest
import torch

import workloads
from oracle import fields as ofields
from oracle import model
from oracle import pals as opals

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


def normwise(a, b, axis=-1):
    return np.linalg.norm(a - b, axis=axis) / np.linalg.norm(b, axis=axis)


def opts(hd, flags):
    return hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED,
                           inner_tol=1e-5, flags=flags)


def _sigp_star(hd, sigp, shift):
    return {hd.FLAG_MEAN_SHIFT: sigp.mean(), hd.FLAG_SHIFT_MIN: sigp.min(), hd.FLAG_SHIFT_MAX: sigp.max(),
            0: 0.0}[shift]


# 24 x 20 x 12: tiles of 170 / 204 / 240 lines with 64 / 64 / 128 lines per tile (partial tiles);
# 70 x 6 x 5: an axis longer than 64 and not a multiple of 4 (padded eigenvector rows)
@pytest.mark.parametrize("dims", [(24, 20, 12), (70, 6, 5)])
@pytest.mark.parametrize("shift", ["mean", "min", "none"])
@pytest.mark.parametrize("fixed", [False, True])
def test_apply_preconditioner_matches_oracle(hd, dims, shift, fixed):
    nx, ny, nz = dims
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=4)
    op = hd.Operator.from_workload(w)
    sig, sigp = model.shifts(w)
    sflag = {"mean": hd.FLAG_MEAN_SHIFT, "min": hd.FLAG_SHIFT_MIN, "none": 0}[shift]
    pflag = hd.FLAG_PRECOND_SEP_FIXED if fixed else hd.FLAG_PRECOND_SEP
    rng = np.random.default_rng(11)
    x = (rng.standard_normal((3, w.N)) + 1j * rng.standard_normal((3, w.N))).astype(np.complex64)
    xt = torch.from_numpy(x).to(DEV)
    for lam in (0, 3):
        y = hd.apply_preconditioner(op, lam, xt, sflag | pflag).cpu().numpy()
        sigma = sig.mean() if fixed else sig[lam]
        ref = ofields.precond_solve(w, x.astype(np.complex128), _sigp_star(hd, sigp, sflag), complex(sigma))
        assert normwise(y.astype(np.complex128), ref).max() <= 2e-5
    # in place gives the same result
    xi = xt.clone()
    hd.apply_preconditioner(op, 3, xi, sflag | pflag, out=xi)
    assert torch.equal(xi, hd.apply_preconditioner(op, 3, xt, sflag | pflag))


def test_apply_preconditioner_rejects_bad_flags(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    x = torch.zeros((1, w.N), dtype=torch.complex64, device=DEV)
    for flags in (hd.FLAG_MEAN_SHIFT, hd.FLAG_PRECOND_SEP | hd.FLAG_PRECOND_SEP_FIXED,
                  hd.FLAG_PRECOND_SEP | hd.FLAG_MEAN_SHIFT | hd.FLAG_SHIFT_MIN, hd.FLAG_PRECOND_SEP | hd.FLAG_GRAPH):
        with pytest.raises(hd.HydotError) as e:
            hd.apply_preconditioner(op, 0, x, flags)
        assert e.value.status == hd.EINVAL
    with pytest.raises(hd.HydotError):
        hd.apply_preconditioner(op, w.L, x, hd.FLAG_PRECOND_SEP)


@pytest.fixture(scope="module")
def case():
    w = workloads.config("tiny", nx=24, ny=20, nz=12, n_lambda=4)
    return w, ofields.solve_banded(w)


@pytest.mark.parametrize("pflag_name", ["FLAG_PRECOND_SEP", "FLAG_PRECOND_SEP_FIXED"])
@pytest.mark.parametrize("shift_name", ["FLAG_MEAN_SHIFT", "FLAG_SHIFT_MAX", None])
def test_preconditioned_solve_matches_oracle(hd, case, pflag_name, shift_name):
    w, ref = case
    pflag = getattr(hd, pflag_name)
    sflag = getattr(hd, shift_name) if shift_name else 0
    op = hd.Operator.from_workload(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, opts(hd, sflag | pflag | hd.FLAG_GRAPH),
                                           out_dtype=torch.complex64, device=DEV)
        _, it0, rel0, st0 = hd.solve_fields(op, w.rhs_voxels, opts(hd, sflag | hd.FLAG_GRAPH),
                                            out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    assert st0 == hd.OK and rel0.max() <= 1e-8
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref).max() < 1e-4
    assert it.mean() <= 0.5 * it0.mean()


def test_preconditioned_per_system_mode(hd, case):
    w, ref = case
    op = hd.Operator.from_workload(w)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels[:2],
                                       opts(hd, hd.FLAG_MEAN_SHIFT | hd.FLAG_PRECOND_SEP | hd.FLAG_PER_SYSTEM),
                                       out_dtype=torch.complex64, device=DEV)
    torch.cuda.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref[:, :2]).max() < 1e-4


def test_preconditioned_heterogeneous_solve(hd):
    """The anomaly is not part of the preconditioner: GMRES handles it, still in few steps."""
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=4)
    p, dc = workloads.pals_truth(w)
    shape = opals.shape(w, p, workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU)
    scale = 4.0 * (dc @ w.extinction)
    ref = ofields.solve_banded(w, pert=(shape, scale))
    op = hd.Operator.from_workload(w)
    op.set_absorption_perturbation(shape, scale)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels,
                                       opts(hd, hd.FLAG_MEAN_SHIFT | hd.FLAG_PRECOND_SEP | hd.FLAG_GRAPH),
                                       out_dtype=torch.complex64, device=DEV)
    torch.cuda.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref).max() < 1e-4
