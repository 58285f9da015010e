"""Born products from BF16 field storage, split-BF16 products, and blocks of probe vectors.

BF16 operands are checked two ways: against the oracle applied to exactly the operands the
kernel rounds to (phi_src v formed in FP32 then rounded to BF16, phi_det rounded to BF16),
which pins the arithmetic to FP32-accumulation accuracy, and against the unrounded FP64
oracle, which states the variant's error.  Rounding to BF16 on the host uses torch's CPU
conversion (round to nearest even), independent of the library."""
import numpy as np
import pytest
import torch

import workloads
from oracle import born as oborn
from oracle import fields as ofields

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


def normwise(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def to_bf16_pairs(P):
    """complex array -> bfloat16 [..., 2] (re, im), rounded to nearest even from FP32"""
    return torch.view_as_real(torch.from_numpy(np.ascontiguousarray(P)).to(torch.complex64)).to(torch.bfloat16)


def from_bf16_pairs(t):
    return torch.view_as_complex(t.float().contiguous()).numpy().astype(np.complex128)


def bf16_round_real(x32):
    """FP32 array -> the FP64 value of its BF16 rounding"""
    return torch.from_numpy(np.ascontiguousarray(x32, dtype=np.float32)).to(torch.bfloat16).double().numpy()


@pytest.fixture(scope="module")
def tiny():
    w = workloads.config("tiny")
    return w, ofields.solve_banded(w)


def test_solver_writes_bf16_fields(hd, tiny):
    w, ref = tiny
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED,
                        inner_tol=1e-5)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.bfloat16, device=DEV)
    assert st == hd.OK and rel.max() <= 1e-8
    assert tuple(phi.shape) == (w.L, w.S + w.D, w.N, 2)
    got = phi.cpu().float().numpy().astype(np.float64)
    r = np.stack([ref.real, ref.imag], axis=-1)
    # one rounding to BF16 of the FP64 iterate, whose error is normwise (within 1e-5 of each
    # field's 2-norm: residual 1e-8 times the condition number of the tiny operator)
    scale = np.linalg.norm(ref, axis=-1)[..., None, None]
    excess = np.abs(got - r) - (2.0 ** -8 * np.abs(r) + 1e-5 * scale)
    assert excess.max() <= 0, (excess.max(), np.unravel_index(excess.argmax(), excess.shape))
    # round to nearest: almost every element equals the BF16 rounding of the oracle value
    rne = torch.from_numpy(r.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.mean(got == rne) > 0.99, np.mean(got == rne)


def _bf16_expected(Ps, Pd, v, h):
    """oracle J v on the operands the BF16 kernel multiplies: A = bf16(fp32(phi_s) * v), B = bf16(phi_d)"""
    Psr = Ps.real.astype(np.float32), Ps.imag.astype(np.float32)
    A_re = bf16_round_real(Psr[0][None] * v.astype(np.float32)[:, None, None, :])
    A_im = bf16_round_real(Psr[1][None] * v.astype(np.float32)[:, None, None, :])
    B = bf16_round_real(Pd.real.astype(np.float32)) + 1j * bf16_round_real(Pd.imag.astype(np.float32))
    out = []
    for c in range(v.shape[0]):
        A = A_re[c] + 1j * A_im[c]
        out.append(oborn.born_apply(A, B, np.ones((1, v.shape[1])), h)[0])
    return np.stack(out)


@pytest.mark.parametrize("S,D,n_v", [(4, 4, 1), (16, 16, 3), (33, 20, 2), (24, 24, 10)])
def test_born_bf16_fields(hd, S, D, n_v):
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=3)     # N = 1820, ragged stages
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(7 + S + D)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = to_bf16_pairs(P).to(DEV)
    Pr = from_bf16_pairs(t.cpu())                       # the stored operands, exactly
    v = workloads.born_v(w, n_v=n_v, dtype=np.float32)
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.complex128)
    exp = _bf16_expected(Pr[:, :S], Pr[:, S:], v, w.h)
    assert normwise(y, exp) < 2e-6
    # stated error of the variant against the unrounded FP64 products
    ref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)
    assert normwise(y, ref) < 2e-2


def _bf16_pairs_expected(Ps, Pd, v, h):
    """oracle J v on the operands of the pair-product BF16 kernel (12 or more probe vectors):
    P = bf16(fp32(phi_s) * fp32(phi_d)) per pair and voxel, times bf16(v)"""
    a_re, a_im = Ps.real.astype(np.float32), Ps.imag.astype(np.float32)
    b_re, b_im = Pd.real.astype(np.float32), Pd.imag.astype(np.float32)
    # P[l, s, d, k] in FP32, then rounded
    P_re = a_re[:, :, None, :] * b_re[:, None, :, :] - a_im[:, :, None, :] * b_im[:, None, :, :]
    P_im = a_re[:, :, None, :] * b_im[:, None, :, :] + a_im[:, :, None, :] * b_re[:, None, :, :]
    P = bf16_round_real(P_re) + 1j * bf16_round_real(P_im)
    vb = bf16_round_real(v.astype(np.float32))
    return -(h ** 3) * np.einsum("lsdk,ck->clsd", P, vb)


@pytest.mark.parametrize("S,D,n_v", [(4, 4, 12), (16, 16, 33), (33, 20, 64), (9, 64, 16)])
def test_born_bf16_fields_probe_blocks(hd, S, D, n_v):
    """12 or more probe vectors: the pair-product kernel with BF16 MFMA products."""
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=2)     # N = 1820, ragged stages
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(17 + S + D + n_v)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = to_bf16_pairs(P).to(DEV)
    Pr = from_bf16_pairs(t.cpu())
    v = workloads.born_v(w, n_v=n_v, dtype=np.float32)
    assert n_v >= hd.BORN_PAIRS_MIN_NV
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.complex128)
    exp = _bf16_pairs_expected(Pr[:, :S], Pr[:, S:], v, w.h)
    assert normwise(y, exp) < 2e-6
    ref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)
    assert normwise(y, ref) < 2e-2


@pytest.mark.parametrize("S,D,n_v", [(4, 4, 12), (16, 16, 42), (33, 20, 64)])
def test_born_split_bf16_probe_blocks(hd, S, D, n_v):
    """12 or more probe vectors: pair products split into hi + lo BF16 parts (three MFMAs)."""
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=2)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(23 + S + D + n_v)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = torch.from_numpy(P).to(torch.complex64).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    v = workloads.born_v(w, n_v=n_v, dtype=np.float32)
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV), split_bf16=True)
    y = y.cpu().numpy().astype(np.complex128)
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], v.astype(np.float64), w.h)
    assert normwise(y.reshape(n_v, -1), ref.reshape(n_v, -1)).max() < 3e-5


def test_born_bf16_on_solver_fields(hd, tiny):
    w, ref = tiny
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, precision=hd.PREC_MIXED,
                        inner_tol=1e-5)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, out_dtype=torch.bfloat16, device=DEV)
    v = workloads.born_v(w, dtype=np.float32)
    y = hd.born_apply(op, phi[:, :w.S], phi[:, w.S:], torch.from_numpy(v).to(DEV)).cpu().numpy()
    yref = oborn.born_apply(ref[:, :w.S], ref[:, w.S:], v.astype(np.float64), w.h)
    err = normwise(y.astype(np.complex128), yref)
    assert err < 2e-2
    # adjoint from BF16 fields: exact widening, FP32 products
    wv = workloads.born_w(w)
    g = hd.born_apply_adjoint(op, phi[:, :w.S], phi[:, w.S:], torch.from_numpy(wv).to(DEV)).cpu().numpy()
    Pr = from_bf16_pairs(phi.cpu())
    gexp = oborn.born_apply_adjoint(Pr[:, :w.S], Pr[:, w.S:], wv, w.h)
    assert normwise(g.astype(np.complex128), gexp) < 1e-5
    gref = oborn.born_apply_adjoint(ref[:, :w.S], ref[:, w.S:], wv, w.h)
    assert normwise(g.astype(np.complex128), gref) < 2e-2


@pytest.mark.parametrize("S,D,n_v", [(4, 4, 1), (16, 16, 2), (33, 20, 1), (64, 64, 1)])
def test_born_split_bf16(hd, S, D, n_v):
    w = workloads.config("tiny", nx=20, ny=13, nz=7, n_lambda=2)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(11 + S + D)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = torch.from_numpy(P).to(torch.complex64).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    v = workloads.born_v(w, n_v=n_v, dtype=np.float32)
    y = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV), split_bf16=True)
    y = y.cpu().numpy().astype(np.complex128)
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], v.astype(np.float64), w.h)
    assert normwise(y, ref) < 1e-4
    # three BF16 products keep the error far below a single BF16 product
    y1 = hd.born_apply(op, t[:, :S], t[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.complex128)
    assert normwise(y1, ref) < 1e-5


@pytest.mark.parametrize("grid", [(20, 13, 7), (16, 10, 8)])        # N = 1820 (ragged), 1280 (16-byte loads)
@pytest.mark.parametrize("S,D,n_v", [(33, 47, 1), (64, 64, 2), (48, 64, 3)])
@pytest.mark.parametrize("mode", ["bf16", "split"])
def test_born_bf16_wide(hd, mode, S, D, n_v, grid):
    """More than 32 sources and detectors on the BF16 MFMA (fewer than 12 probe vectors): BF16-
    stored fields with BF16 products, and FP32 fields with split-BF16 products.  Every (probe
    vector, wavelength, source, detector) entry against the FP64 products of exactly the operands
    the kernel multiplies (BF16: phi_s v formed in FP32 and rounded, phi_d as stored), within 1e-5
    of the absolute sum of its terms (FP32 sums over 32-voxel steps, FP64 beyond); the split
    within 1e-4 of the absolute sum against the FP32 operands themselves."""
    nx, ny, nz = grid
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(31 + S + D + nx)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    v = workloads.born_v(w, n_v=n_v, dtype=np.float32)
    vt = torch.from_numpy(v).to(DEV)
    if mode == "bf16":
        t = to_bf16_pairs(P).to(DEV)
        Pr = from_bf16_pairs(t.cpu())
        y = hd.born_apply(op, t[:, :S], t[:, S:], vt).cpu().numpy().astype(np.complex128)
        exp = _bf16_expected(Pr[:, :S], Pr[:, S:], v, w.h)
        tol = 1e-5
    else:
        t = torch.from_numpy(P).to(torch.complex64).to(DEV)
        Pr = t.cpu().numpy().astype(np.complex128)
        y = hd.born_apply(op, t[:, :S], t[:, S:], vt, split_bf16=True).cpu().numpy().astype(np.complex128)
        exp = oborn.born_apply(Pr[:, :S], Pr[:, S:], v.astype(np.float64), w.h)
        tol = 1e-4
    assert y.shape == exp.shape == (n_v, w.L, S, D)
    absum = w.h ** 3 * np.einsum("lsk,ck,ldk->clsd", np.abs(Pr[:, :S]), np.abs(v.astype(np.float64)),
                                 np.abs(Pr[:, S:]), optimize=True)
    err = np.abs(y - exp)
    assert np.all(err <= tol * absum), float((err / absum).max())
    # stated error of the variant against the unrounded FP64 products
    ref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)
    assert normwise(y, ref) < (2e-2 if mode == "bf16" else 1e-4)


@pytest.mark.parametrize("grid", [(20, 13, 7), (16, 10, 8)])        # N = 1820 (ragged), 1280 (16-byte loads)
@pytest.mark.parametrize("S,D,n_w", [(33, 47, 1), (64, 64, 2), (48, 64, 1)])
def test_born_adjoint_bf16_wide(hd, S, D, n_w, grid):
    """J^H w from BF16-stored fields with more than 32 sources and detectors (BF16 MFMA, w split
    into BF16 hi + lo): every voxel against the FP64 products of the stored fields and the
    unrounded w, within 2e-5 of the absolute sum of its terms (the split's 2^-18 and FP32 sums
    over the sources); stated error against the unrounded fields."""
    nx, ny, nz = grid
    w = workloads.config("tiny", nx=nx, ny=ny, nz=nz, n_lambda=3)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(71 + S + D + nx)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = to_bf16_pairs(P).to(DEV)
    Pr = from_bf16_pairs(t.cpu())
    W = (rng.standard_normal((n_w, w.L, S, D)) + 1j * rng.standard_normal((n_w, w.L, S, D))).astype(np.complex64)
    g = hd.born_apply_adjoint(op, t[:, :S], t[:, S:], torch.from_numpy(W).to(DEV)).cpu().numpy()
    assert g.shape == (n_w, w.N)
    Wd = W.astype(np.complex128)
    for c in range(n_w):
        exp = oborn.born_apply_adjoint(Pr[:, :S], Pr[:, S:], Wd[c], w.h)
        absum = w.h ** 3 * np.einsum("lsk,lsd,ldk->k", np.abs(Pr[:, :S]), np.abs(Wd[c]), np.abs(Pr[:, S:]),
                                     optimize=True)
        err = np.abs(g[c].astype(np.complex128) - exp)
        assert np.all(err <= 2e-5 * absum), float((err / absum).max())
        ref = oborn.born_apply_adjoint(P[:, :S], P[:, S:], Wd[c], w.h)
        assert normwise(g[c].astype(np.complex128), ref) < 2e-2


def test_split_bf16_rejects_other_fields(hd, tiny):
    w, ref = tiny
    op = hd.Operator.from_workload(w)
    t = torch.from_numpy(ref).to(DEV)
    v = torch.ones(w.N, dtype=torch.float64, device=DEV)
    with pytest.raises(hd.HydotError) as e:
        hd.born_apply(op, t[:, :w.S], t[:, w.S:], v, split_bf16=True)
    assert e.value.status == hd.EUNSUPPORTED


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
@pytest.mark.parametrize("S,D", [(4, 4), (16, 16), (24, 24)])
def test_born_probe_vector_block(hd, tiny, dtype, tol, S, D):
    """42 probe vectors (the Jacobian block of 2 contrasts + 40 shape parameters): groups of up
    to 8 vectors share each staged field tile, with a partial last group."""
    w = workloads.config("tiny", n_lambda=2)
    op = hd.Operator.from_workload(w)
    rng = np.random.default_rng(3 + S)
    P = rng.standard_normal((w.L, S + D, w.N)) + 1j * rng.standard_normal((w.L, S + D, w.N))
    t = torch.from_numpy(P).to(dtype).to(DEV)
    Pr = t.cpu().numpy().astype(np.complex128)
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    v = torch.from_numpy(workloads.born_v(w, n_v=42)).to(rdt)
    y = hd.born_apply(op, t[:, :S], t[:, S:], v.to(DEV)).cpu().numpy().astype(np.complex128)
    ref = oborn.born_apply(Pr[:, :S], Pr[:, S:], v.double().numpy(), w.h)
    for c in range(42):
        assert normwise(y[c], ref[c]) < tol, c
