"""ctypes marshalling for libhydot (see include/hydot.h for the contract of each call)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libhydot.so")

if not os.path.exists(_LIBPATH):
    raise ImportError(f"{_LIBPATH} is not built; run `python paper_1410_0986_amd/build.py` "
                      "(or __graft_entry__.build()) first")
_lib = ctypes.CDLL(_LIBPATH)

OK, ENOCONV, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, 1, -1, -2, -3, -4
C128, C64, CBF16, F64, F32 = 0, 1, 2, 3, 4
BORN_NATIVE, BORN_SPLIT_BF16 = 0, 1
BORN_PAIRS_MIN_NV = 12   # HYDOT_BORN_PAIRS_MIN_NV: native J v of this many probe vectors or more contracts over pairs
PREC_FP64, PREC_MIXED = 0, 1
FLAG_NO_RECYCLE, FLAG_MEAN_SHIFT, FLAG_GRAPH, FLAG_PER_SYSTEM, FLAG_FULL_REORTH = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_SHIFT_MIN, FLAG_SHIFT_MAX = 0x20, 0x40
FLAG_PRECOND_SEP, FLAG_PRECOND_SEP_FIXED = 0x80, 0x100


class HydotError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hydot status {status}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("h_mm", c_double),
                ("A_R", c_double), ("robin_faces", c_uint32)]


class _Optics(ctypes.Structure):
    _fields_ = [("n_lambda", c_int32), ("mus_prime_per_mm", POINTER(c_double)), ("n_species", c_int32),
                ("extinction", POINTER(c_double)), ("conc_uM", POINTER(c_double)),
                ("omega_over_nu_per_mm", c_double)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("rel_tol", c_double), ("max_iter", c_int32), ("restart_m", c_int32),
                ("recycle_k", c_int32), ("lanczos_n", c_int32), ("precision", c_int32),
                ("flags", c_uint32), ("inner_tol", c_double), ("max_batch", c_int32)]


class _PalsOpts(ctypes.Structure):
    _fields_ = [("tau", c_double), ("eps", c_double), ("nu", c_double), ("basis", c_int32)]


def _proto(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_assemble = _proto("hydot_assemble_operator", c_int32, POINTER(_Grid), POINTER(_Optics), POINTER(c_void_p))
_free = _proto("hydot_free_operator", None, c_void_p)
_optics = _proto("hydot_operator_optics", c_int32, c_void_p, POINTER(c_double), POINTER(c_double))
_set_pert = _proto("hydot_set_absorption_perturbation", c_int32, c_void_p, POINTER(c_double), POINTER(c_double))
_apply = _proto("hydot_apply_operator", c_int32, c_void_p, c_int32, POINTER(c_int32), c_void_p, c_void_p,
                c_int32, c_void_p)
_precond = _proto("hydot_apply_preconditioner", c_int32, c_void_p, ctypes.c_uint32, c_int32, c_void_p, c_void_p,
                  c_int32, c_void_p)
_ws_bytes = _proto("hydot_solve_workspace_bytes", c_int32, c_void_p, c_int32, POINTER(_SolveOpts), POINTER(c_size_t))
_solve = _proto("hydot_solve_fields", c_int32, c_void_p, c_int32, POINTER(c_int64), POINTER(_SolveOpts), c_void_p,
                c_int32, c_void_p, c_size_t, POINTER(c_int32), POINTER(c_double), c_void_p)
SOLVE_BATCH_MAX = 16   # HYDOT_SOLVE_BATCH_MAX


class _SolveProblem(ctypes.Structure):
    _fields_ = [("op", c_void_p), ("n_rhs", c_int32), ("rhs_voxel", POINTER(c_int64)),
                ("opts", POINTER(_SolveOpts)), ("phi", c_void_p), ("phi_dtype", c_int32), ("workspace", c_void_p),
                ("ws_bytes", c_size_t), ("iters", POINTER(c_int32)), ("rel_res", POINTER(c_double)),
                ("status", c_int32)]


_solve_batch = _proto("hydot_solve_fields_batch", c_int32, c_int32, POINTER(_SolveProblem), c_void_p)


class _InspectInfo(ctypes.Structure):
    _fields_ = [("rhs", c_int32), ("lam", c_int32), ("k", c_int32), ("nsteps", c_int32)]


_inspect = _proto("hydot_solve_inspect", c_int32, c_void_p, c_int32, POINTER(_SolveOpts), c_void_p, c_size_t, c_int32,
                  c_int32, c_void_p, c_size_t, POINTER(_InspectInfo), c_void_p)
INSPECT_U, INSPECT_C, INSPECT_CHOL, INSPECT_CYCLE = 0, 1, 2, 3
_born = _proto("hydot_born_apply", c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32,
               c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p)
_born_ex = _proto("hydot_born_apply_ex", c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32,
                  c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p)
_born_ws = _proto("hydot_born_workspace_bytes", c_int32, c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32,
                  POINTER(c_size_t))
_born_adj_ex = _proto("hydot_born_apply_adjoint_ex", c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_int32,
                      c_int64, c_int32, c_void_p, c_int32, c_void_p, c_void_p)
_born_adj = _proto("hydot_born_apply_adjoint", c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64,
                   c_int32, c_void_p, c_void_p, c_void_p)
_pals = _proto("hydot_pals_shape", c_int32, c_void_p, POINTER(c_double), c_int32, POINTER(_PalsOpts), c_void_p,
               c_int32, c_void_p)
_pals_ws = _proto("hydot_pals_workspace_bytes", c_size_t, c_void_p, c_int32)
_pals_jac = _proto("hydot_pals_shape_jacobian", c_int32, c_void_p, POINTER(c_double), c_int32, POINTER(_PalsOpts),
                   c_void_p, c_int32, c_void_p)
_pals_vjp = _proto("hydot_pals_shape_vjp", c_int32, c_void_p, POINTER(c_double), c_int32, POINTER(_PalsOpts),
                   c_void_p, c_int32, POINTER(c_double), c_void_p, c_size_t, c_void_p)
_misfit_ws = _proto("hydot_misfit_workspace_bytes", c_size_t, c_void_p, c_int32, c_int32)
_misfit = _proto("hydot_misfit", c_int32, c_void_p, c_int32, c_int32, POINTER(c_double), c_void_p, c_void_p,
                 c_void_p, c_int32, c_void_p, POINTER(c_double), POINTER(c_double), c_void_p, c_size_t, c_void_p)


class _Peaks(ctypes.Structure):
    _fields_ = [("read_GBps", c_double), ("copy_GBps", c_double), ("read10_write1_GBps", c_double),
                ("mfma_f32_TFLOPs", c_double), ("mfma_bf16_TFLOPs", c_double), ("compute_units", c_int32)]


_peaks = _proto("hydot_measure_peaks", c_int32, c_void_p, c_size_t, POINTER(_Peaks), c_void_p)


class _Tuning(ctypes.Structure):
    _fields_ = [("step_presum", c_int32), ("step_order", c_int32), ("step_group", c_int32),
                ("born_stage", c_int32), ("born_blocks", c_int32), ("step_vx", c_int32),
                ("step_pair", c_int32)]


class _Trial(ctypes.Structure):
    _fields_ = [("t", _Tuning), ("ms", c_double)]


_get_tuning = _proto("hydot_get_tuning", c_int32, c_void_p, POINTER(_Tuning))
_set_tuning = _proto("hydot_set_tuning", c_int32, c_void_p, POINTER(_Tuning))
_tune_solve = _proto("hydot_autotune_solve", c_int32, c_void_p, c_int32, POINTER(c_int64), POINTER(_SolveOpts),
                     c_void_p, c_int32, c_void_p, c_size_t, POINTER(_Trial), c_int32, POINTER(c_int32), c_void_p)
_tune_born = _proto("hydot_autotune_born", c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32,
                    c_void_p, c_int32, c_void_p, c_void_p, c_size_t, POINTER(_Trial), c_int32, POINTER(c_int32),
                    c_void_p)
_tune_born_ws = _proto("hydot_autotune_born_workspace_bytes", c_int32, c_void_p, c_int32, c_int32, c_int32, c_int32,
                       POINTER(c_size_t))
_TUNE_FIELDS = ("step_presum", "step_order", "step_group", "born_stage", "born_blocks", "step_vx", "step_pair")


class _KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int64), ("total_ms", c_double),
                ("total_bytes", c_double)]


_prof_enable = _proto("hydot_profile_enable", c_int32, c_int32)
_prof_read = _proto("hydot_profile_read", c_int32, POINTER(_KProf), c_int32)
_last_error = _proto("hydot_last_error", ctypes.c_char_p)
_version = _proto("hydot_version", ctypes.c_char_p)


def library_path() -> str:
    return _LIBPATH


def version() -> str:
    return _version().decode()


def profile_enable(on: bool = True) -> None:
    """Turn on (and reset) or off the event timing of the Arnoldi step kernels."""
    _check(_prof_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel name: (launches, total ms, algorithmic bytes)} accumulated since profile_enable(True)."""
    n = _prof_read(None, 0)
    recs = (_KProf * n)()
    m = _prof_read(recs, n)
    return {recs[i].name.decode(): (int(recs[i].launches), float(recs[i].total_ms), float(recs[i].total_bytes))
            for i in range(m)}


def _check(st: int, allow_noconv: bool = False) -> int:
    if st == OK or (allow_noconv and st == ENOCONV):
        return st
    raise HydotError(st, _last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _stream(device=None) -> c_void_p:
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_cuda(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")


def _ws(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    return buf, (ptr + 255) & ~255


@dataclass
class SolveOptions:
    rel_tol: float = 1e-8
    max_iter: int = 5000
    restart_m: int = 40
    recycle_k: int = 10
    lanczos_n: int = 40
    precision: int = PREC_FP64
    flags: int = FLAG_MEAN_SHIFT
    inner_tol: float = 1e-5
    max_batch: int = 0

    def _c(self) -> _SolveOpts:
        return _SolveOpts(self.rel_tol, self.max_iter, self.restart_m, self.recycle_k, self.lanczos_n,
                          self.precision, self.flags, self.inner_tol, self.max_batch)


PALS_WENDLAND, PALS_GAUSSIAN = 0, 1


@dataclass
class PalsOptions:
    tau: float = 0.5
    eps: float = 0.5
    nu: float = 1e-3
    basis: int = 0          # PALS_WENDLAND (the paper's compactly supported functions) or PALS_GAUSSIAN

    def _c(self) -> _PalsOpts:
        return _PalsOpts(self.tau, self.eps, self.nu, self.basis)


class Operator:
    """A(lambda) on a box grid for every wavelength (hydot_assemble_operator)."""

    def __init__(self, nx, ny, nz, h_mm, A_R, robin_faces, mus_prime, extinction, conc_uM, omega_over_nu):
        self._mus = np.ascontiguousarray(mus_prime, dtype=np.float64)
        self._ext = np.ascontiguousarray(np.atleast_2d(extinction), dtype=np.float64)
        self._conc = np.ascontiguousarray(conc_uM, dtype=np.float64)
        g = _Grid(int(nx), int(ny), int(nz), float(h_mm), float(A_R), int(robin_faces))
        o = _Optics(int(self._mus.shape[0]), _dptr(self._mus), int(self._ext.shape[0]), _dptr(self._ext),
                    _dptr(self._conc), float(omega_over_nu))
        h = c_void_p()
        _check(_assemble(ctypes.byref(g), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h_mm)
        self.N = self.nx * self.ny * self.nz
        self.L = int(self._mus.shape[0])
        self.n_species = int(self._ext.shape[0])
        self.extinction = self._ext

    @classmethod
    def from_workload(cls, w):
        return cls(w.nx, w.ny, w.nz, w.h, w.A_R, w.robin_faces, w.mus_prime, w.extinction, w.conc_uM,
                   w.omega_over_nu)

    @property
    def handle(self):
        return self._h

    def optics(self):
        D = np.empty(self.L)
        mua = np.empty(self.L)
        _check(_optics(self._h, _dptr(D), _dptr(mua)))
        return D, mua

    def set_absorption_perturbation(self, shape, scale) -> None:
        """mu_a(k, lambda_l) += scale[l] * shape[k] in every later solve and operator apply
        (hydot_set_absorption_perturbation); shape=None clears it."""
        if shape is None:
            _check(_set_pert(self.handle, None, None))
            return
        sh = np.ascontiguousarray(shape, dtype=np.float64).reshape(-1)
        sc = np.ascontiguousarray(scale, dtype=np.float64).reshape(-1)
        if sh.shape[0] != self.N or sc.shape[0] != self.L:
            raise ValueError("shape must have N entries and scale n_lambda entries")
        _check(_set_pert(self.handle, _dptr(sh), _dptr(sc)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _free(h)
            self._h = None


def _cdtype(t: torch.Tensor) -> int:
    """Library dtype of a field tensor; complex BF16 fields are bfloat16 tensors whose last
    dimension (size 2) holds (re, im)."""
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.bfloat16 and t.dim() >= 1 and t.shape[-1] == 2:
        return CBF16
    raise ValueError("fields must be complex128, complex64 or bfloat16 [..., 2] (re, im) tensors")


def _field_shape(op, count, dtype):
    return (op.L, count, op.N, 2) if dtype == torch.bfloat16 else (op.L, count, op.N)


def apply_preconditioner(op: Operator, lam_index: int, x: torch.Tensor, flags: int = FLAG_PRECOND_SEP | FLAG_MEAN_SHIFT,
                         out: torch.Tensor | None = None) -> torch.Tensor:
    """y = (K_hat + sigma I)^{-1} x (hydot_apply_preconditioner); x: [count, N] complex64 CUDA tensor.
    out may be x itself (in place)."""
    _need_cuda(x, "x")
    if x.dtype != torch.complex64:
        raise ValueError("x must be complex64")
    x2 = x.reshape(-1, op.N)
    if not x2.is_contiguous():
        raise ValueError("x must be contiguous")
    y = torch.empty_like(x2) if out is None else out.reshape(-1, op.N)
    if y.shape != x2.shape or y.dtype != torch.complex64 or not y.is_contiguous():
        raise ValueError("out must be a contiguous complex64 tensor shaped like x")
    _check(_precond(op.handle, int(flags), int(lam_index), c_void_p(x2.data_ptr()), c_void_p(y.data_ptr()),
                    int(x2.shape[0]), _stream(x.device)))
    return y.reshape(x.shape)


def apply_operator(op: Operator, lam_index, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    """y_v = A(lambda_v) x_v; x: [n_vec, N] complex CUDA tensor."""
    _need_cuda(x, "x")
    x = x.contiguous()
    lam = np.ascontiguousarray(lam_index, dtype=np.int32)
    if x.dim() != 2 or x.shape[1] != op.N or x.shape[0] != lam.shape[0]:
        raise ValueError("x must be [len(lam_index), N]")
    if y is None:
        y = torch.empty_like(x)
    _check(_apply(op.handle, int(lam.shape[0]), lam.ctypes.data_as(POINTER(c_int32)), c_void_p(x.data_ptr()),
                  c_void_p(y.data_ptr()), _cdtype(x), _stream(x.device)))
    return y


def solve_workspace_bytes(op: Operator, n_rhs: int, opts: SolveOptions) -> int:
    n = c_size_t()
    o = opts._c()
    _check(_ws_bytes(op.handle, int(n_rhs), ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


def solve_fields(op: Operator, rhs_voxels, opts: SolveOptions | None = None, out_dtype=torch.complex128,
                 device="cuda", out: torch.Tensor | None = None):
    """Fields phi [L, n_rhs, N] for unit injections at rhs_voxels (hydot_solve_fields).

    Returns (phi, iters [L, n_rhs], rel_res [L, n_rhs], status) with status OK or ENOCONV.
    """
    opts = opts or SolveOptions()
    vox = np.ascontiguousarray(rhs_voxels, dtype=np.int64)
    R = int(vox.shape[0])
    if out is None:
        out = torch.empty(_field_shape(op, R, out_dtype), dtype=out_dtype, device=device)
    _need_cuda(out, "out")
    if not out.is_contiguous() or tuple(out.shape) != _field_shape(op, R, out.dtype):
        raise ValueError("out must be a contiguous [L, n_rhs, N] tensor ([L, n_rhs, N, 2] for bfloat16)")
    o = opts._c()
    nbytes = solve_workspace_bytes(op, R, opts)
    buf, wptr = _ws(nbytes, out.device)
    iters = np.zeros(op.L * R, dtype=np.int32)
    rel = np.zeros(op.L * R, dtype=np.float64)
    st = _solve(op.handle, R, vox.ctypes.data_as(POINTER(c_int64)), ctypes.byref(o), c_void_p(out.data_ptr()),
                _cdtype(out), c_void_p(wptr), c_size_t(nbytes), iters.ctypes.data_as(POINTER(c_int32)),
                _dptr(rel), _stream(out.device))
    _check(st, allow_noconv=True)
    del buf
    return out, iters.reshape(op.L, R), rel.reshape(op.L, R), st


def solve_fields_batch(problems, device="cuda"):
    """Several independent solves as one batch (hydot_solve_fields_batch): the operators' kernels
    run concurrently, each on a stream of its own forked from the current stream.

    problems: sequence of (op, rhs_voxels, opts, out) with out a contiguous [L, n_rhs, N] tensor (or
    None for complex128).  Returns one (phi, iters, rel_res, status) per problem, as solve_fields.
    """
    n = len(problems)
    arr = (_SolveProblem * n)()
    keep = []
    results = []
    dev = None
    for i, (op, rhs_voxels, opts, out) in enumerate(problems):
        opts = opts or SolveOptions()
        vox = np.ascontiguousarray(rhs_voxels, dtype=np.int64)
        R = int(vox.shape[0])
        if out is None:
            out = torch.empty(_field_shape(op, R, torch.complex128), dtype=torch.complex128, device=device)
        _need_cuda(out, "out")
        if not out.is_contiguous() or tuple(out.shape) != _field_shape(op, R, out.dtype):
            raise ValueError("out must be a contiguous [L, n_rhs, N] tensor ([L, n_rhs, N, 2] for bfloat16)")
        if dev is None:
            dev = out.device
        elif out.device != dev:
            raise ValueError("all outputs of a batch must be on one device")
        o = opts._c()
        nbytes = solve_workspace_bytes(op, R, opts)
        buf, wptr = _ws(nbytes, out.device)
        iters = np.zeros(op.L * R, dtype=np.int32)
        rel = np.zeros(op.L * R, dtype=np.float64)
        keep.append((vox, o, buf))
        arr[i] = _SolveProblem(op.handle, R, vox.ctypes.data_as(POINTER(c_int64)), ctypes.pointer(o),
                               out.data_ptr(), _cdtype(out), wptr, nbytes,
                               iters.ctypes.data_as(POINTER(c_int32)), _dptr(rel), 0)
        results.append((out, iters, rel, op.L, R))
    st = _solve_batch(n, arr, _stream(dev))
    _check(st, allow_noconv=True)
    del keep
    return [(out, it.reshape(L, R), rel.reshape(L, R), int(arr[i].status))
            for i, (out, it, rel, L, R) in enumerate(results)]


class SolveSession:
    """A solve whose workspace is kept for reading back the solver's intermediates
    (hydot_solve_inspect): U, C, per-system Cholesky factors, the last restart cycle."""

    def __init__(self, op: Operator, rhs_voxels, opts: SolveOptions, out_dtype=torch.complex128, device="cuda"):
        self.op, self.opts = op, opts
        self.vox = np.ascontiguousarray(rhs_voxels, dtype=np.int64)
        self.R = int(self.vox.shape[0])
        self.nbytes = solve_workspace_bytes(op, self.R, opts)
        self.buf, self.wptr = _ws(self.nbytes, device)
        self.device = device
        self.phi = torch.empty(_field_shape(op, self.R, out_dtype), dtype=out_dtype, device=device)
        o = opts._c()
        self.iters = np.zeros(op.L * self.R, dtype=np.int32)
        self.rel = np.zeros(op.L * self.R, dtype=np.float64)
        st = _solve(op.handle, self.R, self.vox.ctypes.data_as(POINTER(c_int64)), ctypes.byref(o),
                    c_void_p(self.phi.data_ptr()), _cdtype(self.phi), c_void_p(self.wptr), c_size_t(self.nbytes),
                    self.iters.ctypes.data_as(POINTER(c_int32)), _dptr(self.rel), _stream(self.phi.device))
        self.status = _check(st, allow_noconv=True)
        self.iters = self.iters.reshape(op.L, self.R)
        self.rel = self.rel.reshape(op.L, self.R)

    def _call(self, what, index, out):
        o = self.opts._c()
        info = _InspectInfo()
        ptr, nb = (None, 0) if out is None else (out.ctypes.data, out.nbytes)
        _check(_inspect(self.op.handle, self.R, ctypes.byref(o), c_void_p(self.wptr), c_size_t(self.nbytes),
                        int(what), int(index), c_void_p(ptr), c_size_t(nb), ctypes.byref(info),
                        _stream(self.phi.device)))
        return info

    def basis_UC(self, r: int):
        """(U, C) [k, N] real FP64 of right-hand side r."""
        info = self._call(INSPECT_U, r, None)
        U = np.empty((info.k, self.op.N))
        C = np.empty((info.k, self.op.N))
        self._call(INSPECT_U, r, U)
        self._call(INSPECT_C, r, C)
        return U, C

    def chol(self, i: int):
        """(rhs, lam, F [k, k] lower) of system i of the last batch."""
        info = self._call(INSPECT_CHOL, i, None)
        F = np.empty((info.k, info.k), dtype=np.complex128, order="F")
        self._call(INSPECT_CHOL, i, F)
        return info.rhs, info.lam, np.tril(F)

    def cycle(self, i: int):
        """(rhs, lam, F' [k, m], Hbar [m+1, m], V [m, N]) of system i's last restart cycle
        (v_m is not formed by the solver; see hydot_solve_inspect)."""
        info = self._call(INSPECT_CYCLE, i, None)
        k, m, N = info.k, info.nsteps, self.op.N
        buf = np.empty(k * m + (m + 1) * m + m * N, dtype=np.complex128)
        self._call(INSPECT_CYCLE, i, buf)
        Fp = buf[:k * m].reshape(k, m)
        Hb = buf[k * m:k * m + (m + 1) * m].reshape(m, m + 1).T
        V = buf[k * m + (m + 1) * m:].reshape(m, N)
        return info.rhs, info.lam, Fp, Hb, V


def get_tuning(op: Operator) -> dict:
    """Launch shapes the operator uses (hydot_get_tuning), defaults resolved."""
    t = _Tuning()
    _check(_get_tuning(op.handle, ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in _TUNE_FIELDS}


def set_tuning(op: Operator, **fields) -> None:
    """Set launch shapes (hydot_set_tuning); unnamed fields keep their current value."""
    cur = get_tuning(op)
    for f in fields:
        if f not in _TUNE_FIELDS:
            raise ValueError(f"unknown tuning field {f}")
    cur.update(fields)
    t = _Tuning(*(int(cur[f]) for f in _TUNE_FIELDS))
    _check(_set_tuning(op.handle, ctypes.byref(t)))


def _trials(arr, n):
    return [({f: int(getattr(arr[i].t, f)) for f in _TUNE_FIELDS}, float(arr[i].ms)) for i in range(n)]


def autotune_solve(op: Operator, rhs_voxels, opts: SolveOptions | None = None, out_dtype=torch.complex64,
                   device="cuda", out: torch.Tensor | None = None) -> list:
    """Time every Arnoldi step-kernel candidate on this problem (hydot_autotune_solve) and keep the
    fastest in the operator.  Returns [(tuning dict, step-kernel ms), ...]."""
    opts = opts or SolveOptions()
    vox = np.ascontiguousarray(rhs_voxels, dtype=np.int64)
    R = int(vox.shape[0])
    if out is None:
        out = torch.empty((op.L, R, op.N), dtype=out_dtype, device=device)
    _need_cuda(out, "out")
    if not out.is_contiguous() or tuple(out.shape) != (op.L, R, op.N):
        raise ValueError("out must be a contiguous [L, n_rhs, N] tensor")
    o = opts._c()
    nbytes = solve_workspace_bytes(op, R, opts)
    buf, wptr = _ws(nbytes, out.device)
    arr = (_Trial * 64)()
    n = c_int32(0)
    _check(_tune_solve(op.handle, R, vox.ctypes.data_as(POINTER(c_int64)), ctypes.byref(o), c_void_p(out.data_ptr()),
                       _cdtype(out), c_void_p(wptr), c_size_t(nbytes), arr, 64, ctypes.byref(n),
                       _stream(out.device)))
    del buf
    return _trials(arr, n.value)


def autotune_born(op: Operator, phi_src: torch.Tensor, phi_det: torch.Tensor, v: torch.Tensor) -> list:
    """Time every J v candidate on these fields (hydot_autotune_born) and keep the fastest in the
    operator.  Returns [(tuning dict, median ms), ...]."""
    ps, S, ls = _field_view(op, phi_src, "phi_src")
    pd, D, ld = _field_view(op, phi_det, "phi_det")
    if ls != ld or phi_src.dtype != phi_det.dtype:
        raise ValueError("phi_src and phi_det must share the wavelength stride and dtype")
    dt = _cdtype(phi_src)
    rdt = torch.float64 if dt == C128 else torch.float32
    _need_cuda(v, "v")
    v = v.reshape(-1, op.N).to(rdt).contiguous()
    y = torch.empty((v.shape[0], op.L, S, D), dtype=_out_complex(dt), device=phi_src.device)
    nb = c_size_t()
    _check(_tune_born_ws(op.handle, S, D, dt, int(v.shape[0]), ctypes.byref(nb)))
    buf, wptr = _ws(nb.value, phi_src.device)
    arr = (_Trial * 64)()
    n = c_int32(0)
    _check(_tune_born(op.handle, c_void_p(ps), S, c_void_p(pd), D, ls, dt, c_void_p(v.data_ptr()), int(v.shape[0]),
                      c_void_p(y.data_ptr()), c_void_p(wptr), c_size_t(nb.value), arr, 64, ctypes.byref(n),
                      _stream(phi_src.device)))
    del buf
    return _trials(arr, n.value)


def _field_view(op: Operator, t: torch.Tensor, name: str):
    """(pointer, count, wavelength stride in N-vectors) of an [L, count, N] field slice
    (or [L, count, N, 2] bfloat16)."""
    _need_cuda(t, name)
    pair = 2 if t.dtype == torch.bfloat16 else 1
    if t.dim() != (4 if pair == 2 else 3) or t.shape[0] != op.L or t.shape[2] != op.N:
        raise ValueError(f"{name} must be [L, count, N] ([L, count, N, 2] for bfloat16)")
    if pair == 2 and (t.shape[3] != 2 or t.stride(3) != 1):
        raise ValueError(f"{name}: bfloat16 fields need a contiguous (re, im) last dimension")
    vec = op.N * pair
    if t.stride(2) != pair or (t.shape[1] > 1 and t.stride(1) != vec) or t.stride(0) % vec != 0:
        raise ValueError(f"{name} must have N-contiguous rows (a slice of an [L, R, N] field array)")
    return t.data_ptr(), int(t.shape[1]), t.stride(0) // vec


def _out_complex(dt):
    return torch.complex128 if dt == C128 else torch.complex64


def born_apply(op: Operator, phi_src: torch.Tensor, phi_det: torch.Tensor, v: torch.Tensor,
               split_bf16: bool = False) -> torch.Tensor:
    """y[c, l, s, d] = -h^3 sum_k phi_src[l,s,k] v[c,k] phi_det[l,d,k] (hydot_born_apply_ex).

    split_bf16: complex64 fields only; products by split-BF16 MFMA (hi*hi + hi*lo + lo*hi)."""
    ps, S, ls = _field_view(op, phi_src, "phi_src")
    pd, D, ld = _field_view(op, phi_det, "phi_det")
    if ls != ld:
        raise ValueError("phi_src and phi_det must share the wavelength stride")
    if phi_src.dtype != phi_det.dtype:
        raise ValueError("phi_src and phi_det must share a dtype")
    dt = _cdtype(phi_src)
    rdt = torch.float64 if dt == C128 else torch.float32
    _need_cuda(v, "v")
    v = v.reshape(-1, op.N).to(rdt).contiguous()
    y = torch.empty((v.shape[0], op.L, S, D), dtype=_out_complex(dt), device=phi_src.device)
    mode = BORN_SPLIT_BF16 if split_bf16 else BORN_NATIVE
    nbytes = born_workspace_bytes(op, S, D, dt, mode, int(v.shape[0]))
    buf, wptr = _ws(nbytes, phi_src.device)
    _check(_born_ex(op.handle, c_void_p(ps), S, c_void_p(pd), D, ls, dt, mode, c_void_p(v.data_ptr()),
                    int(v.shape[0]), c_void_p(y.data_ptr()), c_void_p(wptr), c_size_t(nbytes),
                    _stream(phi_src.device)))
    del buf
    return y


def born_workspace_bytes(op: Operator, S: int, D: int, field_dtype: int, compute: int = BORN_NATIVE,
                         n_v: int = 1) -> int:
    """Device scratch of one J v call (hydot_born_workspace_bytes) at the operator's launch shapes."""
    n = c_size_t()
    _check(_born_ws(op.handle, int(S), int(D), int(field_dtype), int(compute), int(n_v), ctypes.byref(n)))
    return int(n.value)


def born_apply_adjoint(op: Operator, phi_src: torch.Tensor, phi_det: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """g[k] = sum_{l,s,d} conj(J_l[s,d,k]) w[l,s,d] (hydot_born_apply_adjoint_ex).

    w: [L, S, D] -> g [N]; or a block [n_w, L, S, D] -> g [n_w, N]."""
    ps, S, ls = _field_view(op, phi_src, "phi_src")
    pd, D, ld = _field_view(op, phi_det, "phi_det")
    if ls != ld:
        raise ValueError("phi_src and phi_det must share the wavelength stride")
    dt = _cdtype(phi_src)
    _need_cuda(w, "w")
    w = w.to(_out_complex(dt)).contiguous()
    single = w.dim() == 3
    wb = w[None] if single else w
    if wb.dim() != 4 or tuple(wb.shape[1:]) != (op.L, S, D):
        raise ValueError("w must be [L, S, D] or [n_w, L, S, D]")
    g = torch.empty((wb.shape[0], op.N), dtype=_out_complex(dt), device=phi_src.device)
    _check(_born_adj_ex(op.handle, c_void_p(ps), S, c_void_p(pd), D, ls, dt, c_void_p(wb.data_ptr()),
                        int(wb.shape[0]), c_void_p(g.data_ptr()), _stream(phi_src.device)))
    return g[0] if single else g


def pals_shape(op: Operator, p, popts: PalsOptions | None = None, dtype=torch.float64, device="cuda") -> torch.Tensor:
    popts = popts or PalsOptions()
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1))
    nb = pv.shape[0] // 5
    mu = torch.empty(op.N, dtype=dtype, device=device)
    dt = F64 if dtype == torch.float64 else F32
    o = popts._c()
    _check(_pals(op.handle, _dptr(pv), nb, ctypes.byref(o), c_void_p(mu.data_ptr()), dt, _stream(mu.device)))
    return mu


def pals_shape_jacobian(op: Operator, p, popts: PalsOptions | None = None, dtype=torch.float64,
                        device="cuda") -> torch.Tensor:
    """d mu / d p as a device [5*n_bumps, N] tensor (hydot_pals_shape_jacobian)."""
    popts = popts or PalsOptions()
    pn = np.ascontiguousarray(p, dtype=np.float64)
    nb = pn.shape[0] // 5
    jac = torch.empty((5 * nb, op.N), dtype=dtype, device=device)
    o = popts._c()
    _check(_pals_jac(op.handle, _dptr(pn), nb, ctypes.byref(o), c_void_p(jac.data_ptr()),
                     F64 if dtype == torch.float64 else F32, _stream(jac.device)))
    return jac


def pals_shape_vjp(op: Operator, p, g: torch.Tensor, popts: PalsOptions | None = None) -> np.ndarray:
    popts = popts or PalsOptions()
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1))
    nb = pv.shape[0] // 5
    _need_cuda(g, "g")
    g = g.contiguous()
    dt = {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[g.dtype]
    nbytes = _pals_ws(op.handle, nb)
    buf, wptr = _ws(nbytes, g.device)
    out = np.zeros(5 * nb)
    o = popts._c()
    _check(_pals_vjp(op.handle, _dptr(pv), nb, ctypes.byref(o), c_void_p(g.data_ptr()), dt, _dptr(out),
                     c_void_p(wptr), c_size_t(nbytes), _stream(g.device)))
    del buf
    return out


def misfit(op: Operator, dconc, Jmu: torch.Tensor, y_obs: torch.Tensor, weights: torch.Tensor | None = None):
    """(f, df/d dconc, w_adj) of the Born data model (hydot_misfit); Jmu, y_obs: [L, S, D]."""
    _need_cuda(Jmu, "Jmu")
    Jmu = Jmu.contiguous()
    y_obs = y_obs.to(Jmu.dtype).contiguous()
    L, S, D = Jmu.shape
    dt = _cdtype(Jmu)
    dc = np.ascontiguousarray(np.asarray(dconc, dtype=np.float64).reshape(-1))
    if dc.shape[0] != op.n_species:
        raise ValueError("dconc must have one entry per species")
    wptr_w = None
    if weights is not None:
        rdt = torch.float64 if dt == C128 else torch.float32
        weights = weights.to(rdt).contiguous()
        wptr_w = weights.data_ptr()
    wadj = torch.empty_like(Jmu)
    nbytes = _misfit_ws(op.handle, S, D)
    buf, wsp = _ws(nbytes, Jmu.device)
    f = c_double()
    gdc = np.zeros(op.n_species)
    _check(_misfit(op.handle, S, D, _dptr(dc), c_void_p(Jmu.data_ptr()), c_void_p(y_obs.data_ptr()),
                   c_void_p(wptr_w), dt, c_void_p(wadj.data_ptr()), ctypes.byref(f), _dptr(gdc), c_void_p(wsp),
                   c_size_t(nbytes), _stream(Jmu.device)))
    del buf
    return float(f.value), gdc, wadj


class BornMisfit(torch.autograd.Function):
    """f(dconc, p) = 1/2 ||W (ebar(dconc) J mu(p) - y_obs)||^2 with a hand-written adjoint.

    Forward: PaLS shape -> Born J mu -> misfit.  Backward: Born adjoint J^H (ebar W^2 r)
    -> PaLS vector-Jacobian product; df/d dconc comes from the misfit kernel.
    dconc and p are CPU float64 tensors; the fields stay on the GPU.
    """

    @staticmethod
    def forward(ctx, dconc, p, op, phi_src, phi_det, y_obs, popts=None, weights=None):
        popts = popts or PalsOptions()
        rdt = torch.float64 if phi_src.dtype == torch.complex128 else torch.float32
        pn = p.detach().cpu().numpy().astype(np.float64)
        mu = pals_shape(op, pn, popts, dtype=rdt, device=phi_src.device)
        Jmu = born_apply(op, phi_src, phi_det, mu[None])[0]
        f, gdc, wadj = misfit(op, dconc.detach().cpu().numpy(), Jmu, y_obs, weights)
        ctx.op, ctx.popts = op, popts
        ctx.fields = (phi_src, phi_det)
        ctx.wadj, ctx.pn, ctx.gdc = wadj, pn, gdc
        return torch.tensor(f, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gf):
        phi_src, phi_det = ctx.fields
        g = born_apply_adjoint(ctx.op, phi_src, phi_det, ctx.wadj)
        gp = pals_shape_vjp(ctx.op, ctx.pn, g, ctx.popts)
        s = float(gf)
        return (torch.from_numpy(s * ctx.gdc), torch.from_numpy(s * gp), None, None, None, None, None, None)


def measure_peaks(device="cuda", gib: float = 8.0) -> dict:
    """Achievable peaks of the GPU from the library's probe kernels (hydot_measure_peaks), on a
    scratch buffer of `gib` GiB."""
    nbytes = int(gib * (1 << 30))
    buf, ptr = _ws(nbytes, device)
    out = _Peaks()
    _check(_peaks(c_void_p(ptr), c_size_t(nbytes), ctypes.byref(out), _stream(device)))
    del buf
    return {f: getattr(out, f) for f, _ in _Peaks._fields_}
