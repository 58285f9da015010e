"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 path 1e-8 and mixed path 1e-4, normwise relative error per
system for fields, over all (lambda, s, d) for J v, over all voxels for J^H w.
"""
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


def oracle_fields(w):
    return ofields.solve_banded(w)


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-14), (torch.complex64, 2e-6)])
@pytest.mark.parametrize("faces", [0x3F, 0x0C])
def test_apply_operator_matches_sparse_matvec(hd, dtype, tol, faces):
    w = workloads.config("tiny", nx=20, ny=13, nz=7)      # ragged: N = 1820
    w.robin_faces = faces
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(1)
    lam = np.array([0, 3, 7, 7, 2])
    x = rng.standard_normal((5, w.N)) + 1j * rng.standard_normal((5, w.N))
    y = hd.apply_operator(op, lam, torch.from_numpy(x).to(dtype).to(DEV)).cpu().numpy()
    for i, l in enumerate(lam):
        ref = omodel.operator(w, int(l)) @ x[i]
        assert normwise(y[i], ref) < tol


# ------------------------------------------------------------------- solves
def _check_fields(w, phi, rel, tol_field, tol_res, ref=None):
    ref = oracle_fields(w) if ref is None else ref
    err = normwise(phi, ref)
    assert err.max() < tol_field, (err.max(), np.unravel_index(err.argmax(), err.shape))
    assert rel.max() <= tol_res
    return ref


def test_solve_tiny_unrecycled_gmres30(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-10, restart_m=30, recycle_k=0, flags=hd.FLAG_NO_RECYCLE, max_iter=5000)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK
    phi = phi.cpu().numpy()
    _check_fields(w, phi, rel, 1e-8, 1e-10)
    # the reported residual is the residual of the returned fields
    for (l, r) in [(0, 0), (5, 6)]:
        rr = omodel.relative_residual(w, l, w.rhs_voxels[r], phi[l, r])
        assert rr <= 1.01e-10
    assert it.min() > 10


@pytest.mark.parametrize("mean_shift", [True, False])
def test_solve_tiny_recycled_fp64(hd, mean_shift):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    flags = hd.FLAG_MEAN_SHIFT if mean_shift else 0
    o = hd.SolveOptions(rel_tol=1e-11, restart_m=40, recycle_k=10, lanczos_n=40, flags=flags)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK
    _check_fields(w, phi.cpu().numpy(), rel, 1e-8, 1e-11)


def test_solve_ragged_grid_mixed_faces_fp64(hd):
    w = workloads.config("tiny", nx=21, ny=11, nz=9, n_lambda=5)   # N = 2079: two chunks, ragged tail
    w.robin_faces = 0x33
    w.src_voxels = np.array([5, 100, 2000], dtype=np.int64)
    w.det_voxels = np.array([2078, 0], dtype=np.int64)
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-11, restart_m=30, recycle_k=6, lanczos_n=24)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK
    _check_fields(w, phi.cpu().numpy(), rel, 1e-8, 1e-11)


def test_solve_mixed_precision(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=40, recycle_k=10, lanczos_n=40, precision=hd.PREC_MIXED,
                        inner_tol=1e-5)
    ref = oracle_fields(w)
    phi32, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex64, device=DEV)
    assert st == hd.OK
    _check_fields(w, phi32.cpu().numpy().astype(np.complex128), rel, 1e-4, 1e-8, ref)
    phi64, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex128, device=DEV)
    _check_fields(w, phi64.cpu().numpy(), rel, 1e-6, 1e-8, ref)


@pytest.mark.parametrize("dims", [(150, 5, 4), (128, 6, 4), (40, 7, 6), (64, 9, 5), (3, 5, 40)])
@pytest.mark.parametrize("k", [5, 6])
def test_solve_mixed_row_lengths(hd, dims, k):
    """The step kernels take x neighbours from the adjacent lanes and, when an x row fits a
    128-voxel sub-tile, the stencil centres from a ring of four sub-tiles in LDS (loaded one
    sub-tile ahead): rows longer than a sub-tile (150, other instances), exactly one (128), rows
    straddling waves (40), one row per wave (64) and many rows per sub-tile (3, whose y
    neighbours cross sub-tiles), with the exact-k (5) and the runtime-k (6) instances."""
    nx, ny, nz = dims
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=k + 13, recycle_k=k, lanczos_n=24, precision=hd.PREC_MIXED,
                        inner_tol=1e-5, flags=hd.FLAG_MEAN_SHIFT)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.complex64, device=DEV)
    assert st == hd.OK and rel.max() <= 1e-8
    ref = oracle_fields(w)
    assert normwise(phi.cpu().numpy().astype(np.complex128), ref).max() < 1e-4


def test_per_system_and_graph_modes_agree(hd):
    w = workloads.config("tiny", n_lambda=3)
    op = hd.Operator.from_workload(w)
    base = dict(rel_tol=1e-11, restart_m=40, recycle_k=8, lanczos_n=32)
    ref = oracle_fields(w)
    for flags in (hd.FLAG_MEAN_SHIFT | hd.FLAG_PER_SYSTEM, hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, hd.SolveOptions(flags=flags, **base), device=DEV)
        assert st == hd.OK
        _check_fields(w, phi.cpu().numpy(), rel, 1e-8, 1e-11, ref)
    # graph capture on a user stream, mixed precision, several batches
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        o = hd.SolveOptions(precision=hd.PREC_MIXED, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH, max_batch=7,
                            rel_tol=1e-8, restart_m=40, recycle_k=8, lanczos_n=32)
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    s.synchronize()
    assert st == hd.OK
    _check_fields(w, phi.cpu().numpy(), rel, 1e-6, 1e-8, ref)


def test_recycling_reduces_iterations(hd):
    w = workloads.config("tiny", nx=32, ny=32, nz=16, n_lambda=6)
    op = hd.Operator.from_workload(w)
    vox = w.rhs_voxels[:2]
    common = dict(rel_tol=1e-8, restart_m=40, lanczos_n=40, flags=hd.FLAG_MEAN_SHIFT)
    _, it0, rel0, _ = hd.solve_fields(op, vox, hd.SolveOptions(recycle_k=0, **common), device=DEV)
    _, it10, rel10, _ = hd.solve_fields(op, vox, hd.SolveOptions(recycle_k=10, **common), device=DEV)
    assert rel0.max() <= 1e-8 and rel10.max() <= 1e-8
    assert it10.sum() < it0.sum()


def test_enoconv_reported_with_fields_written(hd):
    w = workloads.config("tiny", n_lambda=2)
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-12, max_iter=3, restart_m=13, recycle_k=0, flags=hd.FLAG_NO_RECYCLE)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.ENOCONV
    assert np.all(rel > 1e-12) and np.all(np.isfinite(rel))
    assert np.all(it <= 3 + 13)
    assert torch.isfinite(phi).all()


# --------------------------------------------------------------------- Born
def _born_case(w, dtype):
    P = oracle_fields(w)
    Ps, Pd = P[:, :w.S], P[:, w.S:]
    t = torch.from_numpy(P).to(dtype).to(DEV)
    return P, Ps, Pd, t


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_born_apply_matches_oracle(hd, dtype, tol):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    P, Ps, Pd, t = _born_case(w, dtype)
    v = workloads.born_v(w, n_v=3)
    # inputs as the device sees them (FP32 fields are rounded before the product)
    Pr = t.cpu().numpy().astype(np.complex128)
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    vt = torch.from_numpy(v).to(rdt)
    ref = oborn.born_apply(Pr[:, :w.S], Pr[:, w.S:], vt.double().numpy(), w.h)
    y = hd.born_apply(op, t[:, :w.S], t[:, w.S:], vt.to(DEV)).cpu().numpy()
    assert normwise(y.reshape(3, -1), ref.reshape(3, -1)).max() < tol
    # every (probe vector, wavelength, source, detector) entry within tol of the absolute sum of
    # its terms, so small (far-pair) entries are held to the same relative accuracy
    absum = w.h ** 3 * np.einsum("lsk,ck,ldk->clsd", np.abs(Pr[:, :w.S]), np.abs(vt.double().numpy()),
                                 np.abs(Pr[:, w.S:]), optimize=True)
    assert np.all(np.abs(y - ref) <= tol * absum), float((np.abs(y - ref) / absum).max())
    # against the FP64 oracle without input rounding, within the path's tolerance
    ref64 = oborn.born_apply(Ps, Pd, v, w.h)
    assert normwise(y.reshape(-1), ref64.reshape(-1)) < (1e-8 if dtype == torch.complex128 else 1e-4)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_born_adjoint_matches_oracle(hd, dtype, tol):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    P, Ps, Pd, t = _born_case(w, dtype)
    wv = workloads.born_w(w)
    Pr = t.cpu().numpy().astype(np.complex128)
    wt = torch.from_numpy(wv).to(dtype)
    ref = oborn.born_apply_adjoint(Pr[:, :w.S], Pr[:, w.S:], wt.cpu().numpy().astype(np.complex128), w.h)
    g = hd.born_apply_adjoint(op, t[:, :w.S], t[:, w.S:], wt.to(DEV)).cpu().numpy()
    assert normwise(g, ref) < tol
    # every voxel within tol of the absolute sum of its terms
    wr = wt.cpu().numpy().astype(np.complex128)
    absg = w.h ** 3 * np.einsum("lsk,lsd,ldk->k", np.abs(Pr[:, :w.S]), np.abs(wr), np.abs(Pr[:, w.S:]), optimize=True)
    assert np.all(np.abs(g - ref) <= tol * absg), float((np.abs(g - ref) / absg).max())


@pytest.mark.parametrize("grid", [(10, 9, 7), (16, 10, 8)])         # N = 630 (element loads), 1280 (16-byte)
@pytest.mark.parametrize("S,D", [(9, 16), (16, 16), (16, 9), (17, 32), (32, 9), (32, 32), (33, 33)])
def test_born_one_vector_wide_shapes(hd, S, D, grid):
    """One probe vector on FP32 fields with 9..32 sources and detectors (the wide kernel with its
    waves splitting the voxels, one or 2 x 2 tiles per wave) and just above (the row-split
    form): every (wavelength, source, detector) entry within 1e-5 of the absolute sum of its
    terms against the oracle on the same FP32 operands; the same for J^H w of one data vector
    (the wide adjoint's instances with fewer source steps and detector tiles) at every voxel."""
    nx, ny, nz = grid
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(7 * S + D + nx)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = torch.from_numpy(P).to(torch.complex64).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    v = rng.standard_normal((1, w.N)).astype(np.float32)
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.complex128)
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], v.astype(np.float64), w.h)
    absum = w.h ** 3 * np.einsum("lsk,ck,ldk->clsd", np.abs(Pr[:, :S]), np.abs(v.astype(np.float64)),
                                 np.abs(Pr[:, S:]), optimize=True)
    err = np.abs(y - ref)
    assert np.all(err <= 1e-5 * absum), float((err / absum).max())
    W = (rng.standard_normal((w.L, S, D)) + 1j * rng.standard_normal((w.L, S, D))).astype(np.complex64)
    g = hd.born_apply_adjoint(op, t[:, :S], t[:, S:], torch.from_numpy(W).to(DEV)).cpu().numpy()
    Wd = W.astype(np.complex128)
    gref = oborn.born_apply_adjoint(Pr[:, :S], Pr[:, S:], Wd, w.h)
    gabs = w.h ** 3 * np.einsum("lsk,lsd,ldk->k", np.abs(Pr[:, :S]), np.abs(Wd), np.abs(Pr[:, S:]), optimize=True)
    gerr = np.abs(g.astype(np.complex128) - gref)
    assert np.all(gerr <= 1e-5 * gabs), float((gerr / gabs).max())


@pytest.mark.parametrize("S,D", [(3, 5), (9, 2), (24, 24), (64, 64)])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_born_shapes(hd, S, D, dtype, tol):
    """Padding (S, D not multiples of 8), several tiles per wave, the 64 x 64 maximum, ragged N."""
    w = workloads.config("tiny", nx=10, ny=9, nz=7, n_lambda=3)    # N = 630
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(S * 100 + D)
    R = S + D
    P = (rng.standard_normal((w.L, R, w.N)) + 1j * rng.standard_normal((w.L, R, w.N))) * 1e-3
    t = torch.from_numpy(P).to(dtype).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    v = rng.standard_normal((2, w.N))
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    vt = torch.from_numpy(v).to(rdt)
    y = hd.born_apply(op, t[:, :S], t[:, S:], vt.to(DEV)).cpu().numpy()
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], vt.double().numpy(), w.h)
    assert normwise(y.reshape(2, -1), ref.reshape(2, -1)).max() < tol
    wv = rng.standard_normal((w.L, S, D)) + 1j * rng.standard_normal((w.L, S, D))
    wt = torch.from_numpy(wv).to(dtype)
    g = hd.born_apply_adjoint(op, t[:, :S], t[:, S:], wt.to(DEV)).cpu().numpy()
    refg = oborn.born_apply_adjoint(Pr[:, :S], Pr[:, S:], wt.numpy().astype(np.complex128), w.h)
    assert normwise(g, refg) < tol


@pytest.mark.parametrize("S,D", [(3, 5), (9, 2), (24, 24), (64, 64)])
@pytest.mark.parametrize("n_v", [12, 33, 64])
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-5)])
def test_born_probe_blocks(hd, S, D, n_v, dtype, tol):
    """Blocks of 12 or more probe vectors take the pair-product kernel: one to four tiles of 16
    probe vectors (12, 33 and 64 leave partial tiles or none), partial source and detector
    tiles, ragged N split over many blocks."""
    w = workloads.config("tiny", nx=10, ny=9, nz=7, n_lambda=3)    # N = 630
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(S * 1000 + D * 10 + n_v)
    P = (rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))) * 1e-3
    t = torch.from_numpy(P).to(dtype).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    vt = torch.from_numpy(rng.standard_normal((n_v, w.N))).to(rdt)
    y = hd.born_apply(op, t[:, :S], t[:, S:], vt.to(DEV)).cpu().numpy()
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], vt.double().numpy(), w.h)
    assert y.shape == ref.shape == (n_v, w.L, S, D)
    assert normwise(y.reshape(n_v, -1), ref.reshape(n_v, -1)).max() < tol


@pytest.mark.parametrize("S,D", [(33, 47), (64, 40), (64, 64)])
@pytest.mark.parametrize("grid", [(12, 10, 6), (11, 9, 7)])      # N = 720 (a multiple of 4), 693 (odd)
def test_born_many_pairs_entrywise(hd, S, D, grid):
    """More than 32 sources and detectors with complex FP32 fields: the kernels that feed the
    MFMA from registers (16-byte loads when N is a multiple of 4, element loads otherwise),
    partial source and detector tiles, a ragged voxel count, 1 and 3 probe vectors, 1 and 2 data
    vectors.  Every (probe vector, wavelength, source, detector) entry of J v against the FP64
    definition on the same FP32 operands, within 1e-5 of the absolute sum of its terms (FP32
    products accumulated over 128 voxels, FP64 beyond); J^H w entry by entry the same way."""
    nx, ny, nz = grid
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(S * 7 + D + nx)
    P = (rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))) * 1e-3
    t = torch.from_numpy(P).to(torch.complex64).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    Ps, Pd = Pr[:, :S], Pr[:, S:]
    for n_v in (1, 3):
        v = rng.standard_normal((n_v, w.N)).astype(np.float32)
        y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.complex128)
        vd = v.astype(np.float64)
        ref = oborn.born_apply(Ps, Pd, vd, w.h)
        absum = w.h ** 3 * np.einsum("lsk,ck,ldk->clsd", np.abs(Ps), np.abs(vd), np.abs(Pd), optimize=True)
        assert y.shape == ref.shape == (n_v, w.L, S, D)
        assert np.all(np.abs(y - ref) <= 1e-5 * absum), float((np.abs(y - ref) / absum).max())
    for n_w in (1, 2):
        wv = rng.standard_normal((n_w, w.L, S, D)) + 1j * rng.standard_normal((n_w, w.L, S, D))
        wt = torch.from_numpy(wv).to(torch.complex64)
        wr = wt.numpy().astype(np.complex128)
        g = hd.born_apply_adjoint(op, t[:, :S], t[:, S:], wt.to(DEV)).cpu().numpy().astype(np.complex128)
        g = g.reshape(n_w, w.N)
        for c in range(n_w):
            refg = oborn.born_apply_adjoint(Ps, Pd, wr[c], w.h)
            absg = w.h ** 3 * np.einsum("lsk,lsd,ldk->k", np.abs(Ps), np.abs(wr[c]), np.abs(Pd), optimize=True)
            assert np.all(np.abs(g[c] - refg) <= 1e-5 * absg), float((np.abs(g[c] - refg) / absg).max())


@pytest.mark.parametrize("S,D", [(33, 47), (64, 40), (64, 64)])
@pytest.mark.parametrize("grid", [(12, 10, 6), (11, 9, 7)])      # N = 720, 693 (ragged last tile)
def test_born_fp64_many_pairs_entrywise(hd, S, D, grid):
    """J v of one and of three probe vectors and J^H w of one and of two data vectors on complex
    FP64 fields with more than 32 sources and detectors (the FP64-MFMA wide forms): every
    (probe vector, wavelength, source, detector) entry and every voxel against the FP64
    definition within 1e-13 of the absolute sum of its terms, and the dot-product identity
    <w, J v> = <J^H w, v>."""
    nx, ny, nz = grid
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(S * 11 + D + nx)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = torch.from_numpy(P).to(DEV)
    Ps, Pd = P[:, :S], P[:, S:]
    for n_v in (1, 3):
        vv = rng.standard_normal((n_v, w.N))
        y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(vv).to(DEV)).cpu().numpy()
        ref = oborn.born_apply(Ps, Pd, vv, w.h)
        absum = w.h ** 3 * np.einsum("lsk,ck,ldk->clsd", np.abs(Ps), np.abs(vv), np.abs(Pd), optimize=True)
        assert y.shape == ref.shape == (n_v, w.L, S, D)
        assert np.all(np.abs(y - ref) <= 1e-13 * absum), float((np.abs(y - ref) / absum).max())
    for n_w in (1, 2):
        wv = rng.standard_normal((n_w, w.L, S, D)) + 1j * rng.standard_normal((n_w, w.L, S, D))
        g = hd.born_apply_adjoint(op, t[:, :S], t[:, S:], torch.from_numpy(wv).to(DEV)).cpu().numpy()
        g = g.reshape(n_w, w.N)
        for c in range(n_w):
            refg = oborn.born_apply_adjoint(Ps, Pd, wv[c], w.h)
            absg = w.h ** 3 * np.einsum("lsk,lsd,ldk->k", np.abs(Ps), np.abs(wv[c]), np.abs(Pd), optimize=True)
            assert np.all(np.abs(g[c] - refg) <= 1e-13 * absg), float((np.abs(g[c] - refg) / absg).max())
    v = rng.standard_normal((1, w.N))
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy()[0]
    lhs = np.vdot(wv[0].reshape(-1), y.reshape(-1))
    rhs = np.vdot(g[0], v[0])
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(wv[0]) * np.linalg.norm(y)


def test_born_dot_test_on_device(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    P, Ps, Pd, t = _born_case(w, torch.complex128)
    v = workloads.born_v(w)
    wv = workloads.born_w(w)
    y = hd.born_apply(op, t[:, :w.S], t[:, w.S:], torch.from_numpy(v).to(DEV)).cpu().numpy()[0]
    g = hd.born_apply_adjoint(op, t[:, :w.S], t[:, w.S:], torch.from_numpy(wv).to(DEV)).cpu().numpy()
    lhs = np.vdot(wv.reshape(-1), y.reshape(-1))
    rhs = np.vdot(g, v[0])
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(wv) * np.linalg.norm(y)


# ------------------------------------------------------------ differentiation
BASES = [("wendland", 0), ("gaussian", 1)]


@pytest.mark.parametrize("basis,bcode", BASES)
def test_pals_shape_vjp_and_jacobian(hd, basis, bcode):
    w = workloads.config("tiny", nx=24, ny=20, nz=12, n_lambda=3)
    op = hd.Operator.from_workload(w)
    po = hd.PalsOptions(basis=bcode)
    p_true, _ = workloads.pals_truth(w, basis=basis)
    p, _ = workloads.pals_perturbed(w, p_true, np.ones(2))
    tau, eps, nu = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU
    mu = hd.pals_shape(op, p, po, device=DEV).cpu().numpy()
    ref = opals.shape(w, p, tau, eps, nu, basis)
    assert 0 < (ref > 0.5).sum() < w.N
    np.testing.assert_allclose(mu, ref, rtol=1e-12, atol=1e-13)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(w.N)
    gp = hd.pals_shape_vjp(op, p, torch.from_numpy(g).to(DEV), po)
    Jref = opals.shape_jacobian(w, p, tau, eps, nu, basis)
    refp = Jref.T @ g
    np.testing.assert_allclose(gp, refp, rtol=1e-10, atol=1e-10 * np.abs(refp).max())
    jac = hd.pals_shape_jacobian(op, p, po, device=DEV).cpu().numpy()
    assert jac.shape == (p.shape[0], w.N)
    np.testing.assert_allclose(jac, Jref.T, rtol=1e-11, atol=1e-12 * np.abs(Jref).max())
    jac32 = hd.pals_shape_jacobian(op, p, po, dtype=torch.float32, device=DEV).cpu().numpy()
    np.testing.assert_allclose(jac32, Jref.T, rtol=1e-6, atol=1e-6 * np.abs(Jref).max())


def test_pals_rejects_unknown_basis(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    p, _ = workloads.pals_truth(w)
    with pytest.raises(hd.HydotError) as e:
        hd.pals_shape(op, p, hd.PalsOptions(basis=2), device=DEV)
    assert e.value.status == hd.EINVAL


@pytest.mark.parametrize("basis,bcode", BASES)
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-9), (torch.complex64, 1e-4)])
def test_misfit_gradient_matches_oracle(hd, dtype, tol, basis, bcode):
    w = workloads.config("tiny", nx=24, ny=20, nz=12, n_lambda=4)
    op = hd.Operator.from_workload(w)
    P = ofields.solve_separable(w)
    Ps, Pd = P[:, :w.S], P[:, w.S:]
    tau, eps, nu = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU
    p_true, dc_true = workloads.pals_truth(w, basis=basis)
    _, _, _, y_true = opals.misfit(w, Ps, Pd, p_true, dc_true, 0.0, tau, eps, nu, basis=basis)
    y_obs = y_true + workloads.observed_noise(y_true.shape, 0.03 * np.linalg.norm(y_true) / np.sqrt(y_true.size))
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)
    f, gdc, gp, _ = opals.misfit(w, Ps, Pd, p, dc, y_obs, tau, eps, nu, basis=basis)
    t = torch.from_numpy(P).to(dtype).to(DEV)
    dct = torch.tensor(dc, dtype=torch.float64, requires_grad=True)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    yo = torch.from_numpy(y_obs).to(dtype).to(DEV)
    fv = hd.BornMisfit.apply(dct, pt, op, t[:, :w.S], t[:, w.S:], yo, hd.PalsOptions(basis=bcode))
    fv.backward()
    assert abs(fv.item() - f) <= tol * abs(f)
    g_all = np.concatenate([dct.grad.numpy(), pt.grad.numpy()])
    ref_all = np.concatenate([gdc, gp])
    assert np.linalg.norm(g_all - ref_all) <= tol * 10 * np.linalg.norm(ref_all)


def test_misfit_gradient_finite_differences_fp64(hd):
    w = workloads.config("tiny", nx=24, ny=20, nz=12, n_lambda=3)
    op = hd.Operator.from_workload(w)
    P = ofields.solve_separable(w)
    t = torch.from_numpy(P).to(DEV)
    p_true, dc_true = workloads.pals_truth(w)
    rng = np.random.default_rng(9)
    y_obs = torch.from_numpy(rng.standard_normal((w.L, w.S, w.D)) * 1e-7 + 0j).to(DEV)
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)

    def f_of(x):
        return hd.BornMisfit.apply(torch.tensor(x[:2]), torch.tensor(x[2:]), op, t[:, :w.S], t[:, w.S:],
                                   y_obs).item()

    x = np.concatenate([dc, p])
    xt = torch.tensor(x, requires_grad=True)
    fv = hd.BornMisfit.apply(xt[:2], xt[2:], op, t[:, :w.S], t[:, w.S:], y_obs)
    fv.backward()
    g = xt.grad.numpy()
    for i in (0, 1, 2, 10, 18, 26, 34, 41):
        st = 1e-6 * max(1.0, abs(x[i]))
        xu, xd = x.copy(), x.copy()
        xu[i] += st
        xd[i] -= st
        fd = (f_of(xu) - f_of(xd)) / (2 * st)
        assert abs(fd - g[i]) <= 1e-5 * np.abs(g).max() + 1e-6 * abs(g[i])
