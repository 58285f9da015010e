"""Full (heterogeneous-absorption) forward model on the GPU: the recycled solver with a
per-voxel absorption perturbation mu_a(k) + ebar_l * shape(k), against the oracle's banded LU
of the perturbed operator, and the Born-validity check (the data change of the full model
against the Born prediction)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import born as oborn
from oracle import fields as ofields
from oracle import model as omodel
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


def pals_pert(w, factor=1.0):
    p, dc = workloads.pals_truth(w)
    shape = opals.shape(w, p, workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU)
    return shape, factor * (dc @ w.extinction)


@pytest.fixture(scope="module")
def ragged():
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=4)
    pert = pals_pert(w, 4.0)
    return w, pert, ofields.solve_banded(w, pert=pert)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-6)])
def test_apply_operator_with_perturbation(hd, ragged, dtype, tol):
    w, pert, _ = ragged
    op = hd.Operator.from_workload(w)
    op.set_absorption_perturbation(*pert)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, w.N)) + 1j * rng.standard_normal((2, w.N))
    xt = torch.from_numpy(x).to(dtype).to(DEV)
    y = hd.apply_operator(op, [1, 3], xt).cpu().numpy()
    xr = xt.cpu().numpy().astype(np.complex128)
    for a, l in enumerate((1, 3)):
        ref = omodel.operator_perturbed(w, l, *pert) @ xr[a]
        assert normwise(y[a].astype(np.complex128), ref) < tol
    op.set_absorption_perturbation(None, None)                 # cleared: the plain operator again
    y0 = hd.apply_operator(op, [1], xt[:1]).cpu().numpy()[0]
    assert normwise(y0.astype(np.complex128), omodel.operator(w, 1) @ xr[0]) < tol


@pytest.mark.parametrize("flags", ["mean", "nomean", "norecycle"])
def test_perturbed_solve_fp64(hd, ragged, flags):
    w, pert, ref = ragged
    op = hd.Operator.from_workload(w)
    op.set_absorption_perturbation(*pert)
    fl = {"mean": hd.FLAG_MEAN_SHIFT, "nomean": 0, "norecycle": hd.FLAG_NO_RECYCLE}[flags]
    o = hd.SolveOptions(rel_tol=1e-11, restart_m=18, recycle_k=5 if flags != "norecycle" else 0, lanczos_n=24,
                        flags=fl)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK and rel.max() <= 1e-11
    err = normwise(phi.cpu().numpy(), ref)
    assert err.max() < 1e-8
    # independent FP64 residual of the returned fields for a few systems
    got = phi.cpu().numpy()
    for l, r in ((0, 0), (3, 5)):
        assert omodel.relative_residual(w, l, int(w.rhs_voxels[r]), got[l, r], pert=pert) < 1e-10


def test_perturbed_solve_mixed_graph(hd, ragged):
    w, pert, ref = ragged
    op = hd.Operator.from_workload(w)
    op.set_absorption_perturbation(*pert)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED,
                        inner_tol=1e-5, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref).max() < 1e-4


def test_born_validity_medium(hd):
    """Medium workload with the PaLS anomaly at the true contrast: every perturbed system reaches
    FP64 rel-res 1e-8 (recomputed independently for samples); the detector data change of the full
    model matches the Born prediction to first order (halving the contrast halves the relative
    mismatch)."""
    torch.cuda.empty_cache()
    w = workloads.config("medium")
    S = w.S
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=32, precision=hd.PREC_MIXED,
                        inner_tol=1e-5, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH)
    s = torch.cuda.Stream()
    det = torch.from_numpy(np.asarray(w.det_voxels)).to(DEV)
    with torch.cuda.stream(s):
        phi0, _, rel0, st0 = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex128, device=DEV)
        d0 = phi0[:, :S][:, :, det].clone()
        shape, ebar = pals_pert(w)
        mu = torch.from_numpy(shape).to(DEV)
        y1 = hd.born_apply(op, phi0[:, :S], phi0[:, S:], mu[None])[0]          # J shape, [L, S, D]
        rels = []
        for f in (1.0, 0.5):
            op.set_absorption_perturbation(shape, f * ebar)
            phi, _, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex128, device=DEV)
            assert st == hd.OK and rel.max() <= 1e-8
            if f == 1.0:
                got = phi.cpu().numpy()
                for l, r in ((0, 2), (31, 20)):
                    res = omodel.relative_residual(w, l, int(w.rhs_voxels[r]), got[l, r], pert=(shape, ebar))
                    assert res < 1e-7
            dfull = phi[:, :S][:, :, det] - d0
            pred = f * torch.from_numpy(ebar).to(DEV)[:, None, None] * y1
            rels.append(float(torch.linalg.vector_norm(dfull - pred) / torch.linalg.vector_norm(dfull)))
    s.synchronize()
    assert rels[0] < 0.5                       # the Born model is a fair surrogate at this contrast
    assert 1.6 < rels[0] / rels[1] < 2.4       # its error is second order in the contrast
