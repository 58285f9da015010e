"""Several grids solved as one batch (hydot_solve_fields_batch): every problem's fields, Arnoldi
step counts and residuals are exactly those of its own hydot_solve_fields call, and match the
FP64 oracle at the path's tolerance (1e-8 FP64, 1e-4 mixed)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import fields as ofields
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


def _grids():
    # three grids at the same 8 wavelengths: the tiny box, a ragged box with rows shorter than a
    # wave, and a box with more right-hand sides than the others
    return [workloads.config("tiny"),
            workloads.config("tiny", nx=20, ny=13, nz=7, n_src=2, n_det=4),
            workloads.config("tiny", nx=22, ny=18, nz=10, n_src=8, n_det=8)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_of_grids_matches_single_solves_and_oracle(hd, prec):
    ws = _grids()
    ops = [hd.Operator.from_workload(w) for w in ws]
    if prec == "fp64":
        opts = [hd.SolveOptions(rel_tol=1e-11, restart_m=40, recycle_k=10, lanczos_n=40,
                                flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH)] * 3
        dt, tol_f, tol_r = torch.complex128, 1e-8, 1e-11
    else:
        # the middle problem in two batches of systems, the others in one
        opts = [hd.SolveOptions(rel_tol=1e-8, restart_m=20, recycle_k=5, lanczos_n=40, precision=hd.PREC_MIXED,
                                inner_tol=3e-5, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH, max_batch=mb)
                for mb in (0, 24, 0)]
        dt, tol_f, tol_r = torch.complex64, 1e-4, 1e-8
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = [torch.full((w.L, w.S + w.D, w.N), float("nan"), dtype=dt, device=DEV) for w in ws]
        res = hd.solve_fields_batch([(op, w.rhs_voxels, o, out) for op, w, o, out in zip(ops, ws, opts, outs)])
        singles = [hd.solve_fields(op, w.rhs_voxels, o, out_dtype=dt, device=DEV)
                   for op, w, o in zip(ops, ws, opts)]
    s.synchronize()
    for i, (w, (phi, it, rel, st), (phi1, it1, rel1, st1)) in enumerate(zip(ws, res, singles)):
        assert st == hd.OK and st1 == hd.OK, i
        assert torch.equal(phi, phi1), i
        np.testing.assert_array_equal(it, it1)
        np.testing.assert_array_equal(rel, rel1)
        assert rel.max() <= tol_r, (i, rel.max())
        ref = ofields.solve_banded(w)
        err = normwise(phi.cpu().numpy().astype(np.complex128), ref)
        assert err.max() < tol_f, (i, err.max())


def test_batch_reports_the_failing_problem(hd):
    """A problem that fails its argument checks gets its own status; the others are solved."""
    ws = _grids()[:2]
    ops = [hd.Operator.from_workload(w) for w in ws]
    o = hd.SolveOptions(rel_tol=1e-10, restart_m=40, recycle_k=10, lanczos_n=40)
    bad = ws[1].rhs_voxels.copy()
    bad[1] = ws[1].N            # outside the grid: rejected before anything is launched
    outs = [torch.zeros((w.L, w.S + w.D, w.N), dtype=torch.complex128, device=DEV) for w in ws]
    with pytest.raises(hd.HydotError) as e:
        hd.solve_fields_batch([(ops[0], ws[0].rhs_voxels, o, outs[0]), (ops[1], bad, o, outs[1])])
    assert e.value.status == hd.EINVAL and "problem 1" in str(e.value)
    torch.cuda.synchronize()
    ref = ofields.solve_banded(ws[0])
    assert normwise(outs[0].cpu().numpy(), ref).max() < 1e-8
    assert not outs[1].abs().any()


def test_batch_of_different_solver_paths(hd):
    """Problems of one batch on different paths at once: the separable preconditioner, an
    absorption perturbation on the mixed path, the FP64 per-system loop, and the exact-k
    mixed path; each equal to its own single solve bit for bit and to the oracle."""
    ws = [workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=4),
          workloads.config("tiny", nx=16, ny=16, nz=8, n_lambda=4),
          workloads.config("tiny", nx=12, ny=10, nz=9, n_lambda=4, n_src=2, n_det=2),
          workloads.config("tiny", nx=22, ny=18, nz=10, n_lambda=4)]
    p, dc = workloads.pals_truth(ws[1])
    shape = opals.shape(ws[1], p, workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU)
    scale = 4.0 * (dc @ ws[1].extinction)
    mixed = dict(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED, inner_tol=1e-5)
    opts = [hd.SolveOptions(**mixed, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PRECOND_SEP | hd.FLAG_GRAPH),
            hd.SolveOptions(**mixed, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH),
            hd.SolveOptions(rel_tol=1e-11, restart_m=40, recycle_k=10, lanczos_n=40,
                            flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PER_SYSTEM),
            hd.SolveOptions(**mixed, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH, max_batch=16)]
    dts = [torch.complex64, torch.complex64, torch.complex128, torch.complex64]
    tols = [1e-4, 1e-4, 1e-8, 1e-4]
    def ops():
        o = [hd.Operator.from_workload(w) for w in ws]
        o[1].set_absorption_perturbation(shape, scale)
        return o
    bops, sops = ops(), ops()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = [torch.zeros((w.L, w.S + w.D, w.N), dtype=dt, device=DEV) for w, dt in zip(ws, dts)]
        res = hd.solve_fields_batch([(op, w.rhs_voxels, o, out) for op, w, o, out in zip(bops, ws, opts, outs)])
        singles = [hd.solve_fields(op, w.rhs_voxels, o, out_dtype=dt, device=DEV)
                   for op, w, o, dt in zip(sops, ws, opts, dts)]
    s.synchronize()
    for i, (w, (phi, it, rel, st), (phi1, it1, rel1, st1), tol) in enumerate(zip(ws, res, singles, tols)):
        assert st == hd.OK and st1 == hd.OK, i
        assert torch.equal(phi, phi1), i
        np.testing.assert_array_equal(it, it1)
        np.testing.assert_array_equal(rel, rel1)
        ref = ofields.solve_banded(w, pert=(shape, scale)) if i == 1 else ofields.solve_banded(w)
        err = normwise(phi.cpu().numpy().astype(np.complex128), ref)
        assert err.max() < tol, (i, err.max())
