"""The paper's boundary split (Robin on the top and bottom plates, Dirichlet on the sides) and the
variants of the shift moved into K_hat (mean, minimum, maximum of sigma'_j, or none): every
combination reaches the oracle fields."""
import numpy as np
import pytest
import torch

import workloads
from oracle import fields as ofields

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
TOP_BOTTOM = 0x30   # Robin on -z and +z only


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


def normwise(a, b, axis=-1):
    return np.linalg.norm(a - b, axis=axis) / np.linalg.norm(b, axis=axis)


@pytest.fixture(scope="module", params=[workloads.ALL_ROBIN, TOP_BOTTOM], ids=["all_robin", "top_bottom"])
def case(request):
    w = workloads.config("tiny", nx=18, ny=12, nz=10, n_lambda=4, robin_faces=request.param)
    return w, ofields.solve_banded(w)


@pytest.mark.parametrize("shift", ["none", "mean", "min", "max"])
def test_shift_variants_fp64(hd, case, shift):
    w, ref = case
    op = hd.Operator.from_workload(w)
    fl = {"none": 0, "mean": hd.FLAG_MEAN_SHIFT, "min": hd.FLAG_SHIFT_MIN, "max": hd.FLAG_SHIFT_MAX}[shift]
    o = hd.SolveOptions(rel_tol=1e-11, restart_m=18, recycle_k=5, lanczos_n=24, flags=fl)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK and rel.max() <= 1e-11
    assert normwise(phi.cpu().numpy(), ref).max() < 1e-8


@pytest.mark.parametrize("shift", ["mean", "max", "min", "none"])
def test_shift_variants_mixed(hd, case, shift):
    w, ref = case
    op = hd.Operator.from_workload(w)
    fl = {"mean": hd.FLAG_MEAN_SHIFT, "max": hd.FLAG_SHIFT_MAX, "min": hd.FLAG_SHIFT_MIN, "none": 0}[shift]
    fl |= hd.FLAG_GRAPH
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED,
                        inner_tol=1e-5, flags=fl)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref).max() < 1e-4
