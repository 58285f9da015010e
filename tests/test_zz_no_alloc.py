"""The allocation-free J v entry point, hydot_born_apply_noalloc, called through the C ABI.

Its products must equal those of hydot_born_apply_ex, which runs the same kernels with a
caller-owned workspace.  Only the voxel split may be lower, so that the FP64 partial sums fit the
static scratch.  That changes only the order of the FP64 sums over voxel ranges: every 32-voxel
stage is formed the same way.  The check runs on two calls in a row, the second smaller, so the
second call runs over what the first left in the shared array.  Each result is also checked
against the plain FP64 definition of J v (Sec. 2.1 integral equation with the adjoint field).  A
call whose partials cannot fit is rejected before any launch.
"""
import ctypes
from ctypes import c_int32, c_int64, c_size_t, c_void_p

import numpy as np
import pytest
import torch

import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
C128, C64 = 0, 1
NATIVE = 0
OK, ENOMEM = 0, -2
SCRATCH_BYTES = 32 << 20   # HYDOT_BORN_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def lib():
    import paper_1410_0986_amd as hd
    L = ctypes.CDLL(hd.library_path())
    L.hydot_born_apply_noalloc.restype = c_int32
    L.hydot_born_apply_noalloc.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32,
                                           c_int32, c_void_p, c_int32, c_void_p, c_void_p]
    L.hydot_born_apply_ex.restype = c_int32
    L.hydot_born_apply_ex.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32, c_int32,
                                      c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]
    L.hydot_born_workspace_bytes.restype = c_int32
    L.hydot_born_workspace_bytes.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32,
                                             ctypes.POINTER(c_size_t)]
    L.hydot_last_error.restype = ctypes.c_char_p
    return hd, L


def _fields(w, S, D, dtype, seed):
    """One [L][S + D][N] array (the solver's output layout): sources are rows [0, S) and
    detectors rows [S, S + D) of each wavelength, so both share lam_stride = S + D."""
    rng = np.random.default_rng(seed)
    shape = (w.L, S + D, w.N)
    P = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return torch.from_numpy(P).to(dtype).to(DEV), P


def _oracle_jv(ps, pd, v, h):
    # y[c, l, s, d] = -h^3 sum_k ps[l, s, k] v[c, k] pd[l, d, k], FP64
    return -(h ** 3) * np.einsum("lsk,ck,ldk->clsd", ps, v, pd, optimize=True)


def _both(hd, L, op, P_t, S, D, v_t, dt):
    stream = c_void_p(torch.cuda.current_stream().cuda_stream)
    n_v = int(v_t.shape[0])
    assert P_t.is_contiguous() and tuple(P_t.shape) == (op.L, S + D, op.N)
    assert tuple(v_t.shape) == (n_v, op.N) and v_t.is_contiguous()
    ls = S + D
    ps = P_t.data_ptr()
    pd = P_t.data_ptr() + S * op.N * P_t.element_size()
    out_dtype = torch.complex128 if dt == C128 else torch.complex64
    y_na = torch.full((n_v, op.L, S, D), complex(7.0, -7.0), dtype=out_dtype, device=DEV)
    y_ws = torch.empty_like(y_na)
    st = L.hydot_born_apply_noalloc(op.handle, ps, S, pd, D, ls, dt, NATIVE, v_t.data_ptr(), n_v, y_na.data_ptr(),
                                    stream)
    assert st == OK, L.hydot_last_error()
    nb = c_size_t()
    assert L.hydot_born_workspace_bytes(op.handle, S, D, dt, NATIVE, n_v, ctypes.byref(nb)) == OK
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=DEV)
    wptr = (ws.data_ptr() + 255) & ~255
    st = L.hydot_born_apply_ex(op.handle, ps, S, pd, D, ls, dt, NATIVE, v_t.data_ptr(), n_v, y_ws.data_ptr(), wptr,
                               nb.value, stream)
    assert st == OK, L.hydot_last_error()
    torch.cuda.synchronize()
    return y_na.cpu().numpy().astype(np.complex128), y_ws.cpu().numpy().astype(np.complex128), nb.value


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_workspace_entry_point_twice(lib):
    hd, L = lib
    # first call: 64x64x32 grid, 32 wavelengths, 16 + 16 optodes, a block of 16 probe vectors on
    # the pair-product kernel in FP32; the tuned split's partials (64 MiB) exceed the scratch, so
    # the entry point lowers the split
    w1 = workloads.config("medium")
    op1 = hd.Operator.from_workload(w1)
    S1, D1, nv1 = w1.S, w1.D, 16
    P1, _ = _fields(w1, S1, D1, torch.complex64, seed=71)
    v1 = np.random.default_rng(72).standard_normal((nv1, w1.N))
    v1_t = torch.from_numpy(v1).to(torch.float32).to(DEV)
    y_na, y_ws, ws_bytes = _both(hd, L, op1, P1, S1, D1, v1_t, C64)
    assert ws_bytes > SCRATCH_BYTES, ws_bytes          # the lowered split is exercised
    # FP32 MFMA within 32-voxel stages, FP64 beyond: the two splits differ only in the FP64 sums
    assert _rel(y_na, y_ws) <= 1e-12
    assert np.array_equal(np.isfinite(y_na), np.ones_like(y_na, dtype=bool))
    # against the plain definition on the rounded operands, one wavelength (FP32 products of
    # unit-variance data over 131072 voxels: normwise 1e-6)
    lam = 5
    P_r = P1[lam:lam + 1].cpu().numpy().astype(np.complex128)
    ref = _oracle_jv(P_r[:, :S1], P_r[:, S1:], v1_t.cpu().numpy().astype(np.float64), w1.h)[:, 0]
    assert _rel(y_na[:, lam], ref) <= 1e-6
    del P1

    # second call, smaller: 16x16x8 grid, 8 wavelengths, 3 sources x 2 detectors, 3 probe vectors
    # on the real-ified kernel in FP64
    w2 = workloads.config("tiny")
    op2 = hd.Operator.from_workload(w2)
    S2, D2, nv2 = 3, 2, 3
    P2, P2_np = _fields(w2, S2, D2, torch.complex128, seed=73)
    v2 = np.random.default_rng(74).standard_normal((nv2, w2.N))
    v2_t = torch.from_numpy(v2).to(DEV)
    y_na2, y_ws2, _ = _both(hd, L, op2, P2, S2, D2, v2_t, C128)
    assert _rel(y_na2, y_ws2) <= 1e-14
    assert _rel(y_na2, _oracle_jv(P2_np[:, :S2], P2_np[:, S2:], v2, w2.h)) <= 1e-13


def test_noalloc_rejects_partials_beyond_the_scratch(lib):
    hd, L = lib
    # 64 probe vectors x 32 wavelengths x 64 x 64 pairs of complex FP64 partials = 128 MiB for
    # a single voxel range: ENOMEM before any launch, y untouched
    w = workloads.config("medium", n_src=64, n_det=64, n_lambda=32)
    op = hd.Operator.from_workload(w)
    S = D = 64
    N = w.N
    # full-size (zero) operands, so every access of the call would stay in bounds even if it ran
    ps = torch.zeros((w.L, S, N), dtype=torch.complex64, device=DEV)
    v = torch.zeros((64, N), dtype=torch.float32, device=DEV)
    y = torch.full((64, w.L, S, D), complex(3.0, 4.0), dtype=torch.complex64, device=DEV)
    torch.cuda.synchronize()
    stream = c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.hydot_born_apply_noalloc(op.handle, ps.data_ptr(), S, ps.data_ptr(), D, S, C64, NATIVE,
                                    v.data_ptr(), 64, y.data_ptr(), stream)
    assert st == ENOMEM
    assert b"static scratch" in L.hydot_last_error()
    torch.cuda.synchronize()
    assert bool((y == complex(3.0, 4.0)).all())
