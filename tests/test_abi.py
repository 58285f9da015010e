"""C-ABI tests that need no GPU: the library loads, exports every declared symbol,
validates its arguments before any launch, and its host-side optical model agrees
with the oracle's independent one."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from oracle import model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hydot.h")


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hydot_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("hydot_assemble_operator", "hydot_solve_fields", "hydot_born_apply", "hydot_born_apply_adjoint"):
        assert name in syms


def test_library_exports_every_declared_symbol(hd):
    lib = ctypes.CDLL(hd.library_path())
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert "gfx950" in hd.version()


def _op(hd, w):
    return hd.Operator.from_workload(w)


def test_optical_model_matches_oracle(hd):
    w = workloads.config("medium")
    op = _op(hd, w)
    D, mua = op.optics()
    Do, muao, _ = model.optics(w)
    np.testing.assert_allclose(D, Do, rtol=1e-15)
    np.testing.assert_allclose(mua, muao, rtol=1e-14)


@pytest.mark.parametrize("field,value", [("nx", 0), ("h", 0.0), ("h", -1.0), ("A_R", 0.0),
                                         ("robin_faces", 0x40)])
def test_assemble_rejects_bad_grid(hd, field, value):
    w = workloads.config("tiny")
    setattr(w, field, value)
    with pytest.raises(hd.HydotError) as e:
        _op(hd, w)
    assert e.value.status == hd.EINVAL


def test_assemble_rejects_bad_optics(hd):
    w = workloads.config("tiny")
    w.mus_prime = w.mus_prime.copy()
    w.mus_prime[3] = float("nan")
    with pytest.raises(hd.HydotError) as e:
        _op(hd, w)
    assert e.value.status == hd.EINVAL
    w = workloads.config("tiny")
    with pytest.raises(hd.HydotError):
        hd.Operator(4, 4, 4, 2.0, 2.5, 0x3F, w.mus_prime, np.zeros((9, w.L)), np.zeros(9), w.omega_over_nu)


def test_workspace_size_grows_with_batch_and_precision(hd):
    w = workloads.config("tiny")
    op = _op(hd, w)
    o64 = hd.SolveOptions(restart_m=40, recycle_k=10, lanczos_n=40)
    o32 = hd.SolveOptions(restart_m=40, recycle_k=10, lanczos_n=40, precision=hd.PREC_MIXED)
    b64 = hd.solve_workspace_bytes(op, 8, o64)
    b32 = hd.solve_workspace_bytes(op, 8, o32)
    assert b64 > 0 and b32 > 0
    # the Krylov basis alone: systems x (m-k+1) x N x 16 bytes
    assert b64 >= 8 * w.L * 31 * w.N * 16
    assert b32 < b64
    per = hd.solve_workspace_bytes(op, 8, hd.SolveOptions(flags=hd.FLAG_PER_SYSTEM | hd.FLAG_MEAN_SHIFT))
    assert per < b64


@pytest.mark.parametrize("kw", [dict(recycle_k=40), dict(recycle_k=10, lanczos_n=10), dict(restart_m=5, recycle_k=10),
                                dict(rel_tol=0.0), dict(max_iter=0), dict(precision=7), dict(flags=0x200),
                                dict(precision=1, inner_tol=0.0), dict(restart_m=400, recycle_k=0)])
def test_solve_options_validated(hd, kw):
    w = workloads.config("tiny")
    op = _op(hd, w)
    with pytest.raises(hd.HydotError) as e:
        hd.solve_workspace_bytes(op, 8, hd.SolveOptions(**kw))
    assert e.value.status == hd.EINVAL


def _raw(hd):
    return ctypes.CDLL(hd.library_path())


def test_solve_fields_validates_before_launch(hd):
    from paper_1410_0986_amd._binding import _SolveOpts
    lib = _raw(hd)
    w = workloads.config("tiny")
    op = _op(hd, w)
    o = _SolveOpts(1e-8, 100, 40, 10, 40, 0, 0, 1e-5, 0)
    need = hd.solve_workspace_bytes(op, 8, hd.SolveOptions())
    vox = np.ascontiguousarray(w.rhs_voxels)
    vp = vox.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    f = lib.hydot_solve_fields
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(0x7F0000000000)      # never dereferenced: validation fails first
    # null phi
    assert f(op.handle, 8, vp, ctypes.byref(o), None, 0, fake, need, None, None, None) == hd.EINVAL
    # misaligned workspace
    assert f(op.handle, 8, vp, ctypes.byref(o), fake, 0, ctypes.c_void_p(0x7F0000000010), need, None, None,
             None) == hd.EINVAL
    # workspace too small
    assert f(op.handle, 8, vp, ctypes.byref(o), fake, 0, fake, need - 1, None, None, None) == hd.ENOMEM
    # voxel out of range
    bad = vox.copy()
    bad[2] = w.N
    assert f(op.handle, 8, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(o), fake, 0, fake, need,
             None, None, None) == hd.EINVAL
    # unsupported output dtype
    assert f(op.handle, 8, vp, ctypes.byref(o), fake, 3, fake, need, None, None, None) == hd.EUNSUPPORTED
    assert "dtype" in hd._binding._last_error().decode()


def test_solve_batch_validates_before_launch(hd):
    from paper_1410_0986_amd._binding import _SolveProblem
    lib = _raw(hd)
    f = lib.hydot_solve_fields_batch
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    w = workloads.config("tiny")
    a, b = _op(hd, w), _op(hd, w)
    arr = (_SolveProblem * (hd.SOLVE_BATCH_MAX + 1))()
    for i in range(hd.SOLVE_BATCH_MAX + 1):
        arr[i].op = a.handle if i == 0 else b.handle
        arr[i].status = 77
    assert f(0, arr, None) == hd.EINVAL
    assert f(hd.SOLVE_BATCH_MAX + 1, arr, None) == hd.EINVAL
    assert f(1, None, None) == hd.EINVAL
    assert f(3, arr, None) == hd.EINVAL                        # operator b twice
    assert "twice" in hd._binding._last_error().decode()
    arr[1].op = None
    assert f(2, arr, None) == hd.EINVAL                        # null operator
    assert all(arr[i].status == 77 for i in range(3))          # nothing ran


def test_born_validates_before_launch(hd):
    lib = _raw(hd)
    w = workloads.config("tiny")
    op = _op(hd, w)
    f = lib.hydot_born_apply
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                  ctypes.c_void_p]
    fake = ctypes.c_void_p(0x7F0000000000)
    big = 1 << 40
    assert f(op.handle, fake, 0, fake, 4, 8, 0, fake, 1, fake, fake, big, None) == hd.EINVAL        # S = 0
    assert f(op.handle, fake, 65, fake, 4, 80, 0, fake, 1, fake, fake, big, None) == hd.EINVAL      # S > 64
    assert f(op.handle, fake, 4, fake, 4, 3, 0, fake, 1, fake, fake, big, None) == hd.EINVAL        # lam_stride < S
    assert f(op.handle, fake, 4, fake, 4, 8, 0, fake, 0, fake, fake, big, None) == hd.EINVAL        # n_v = 0
    assert f(op.handle, fake, 4, fake, 4, 8, 4, fake, 1, fake, fake, big, None) == hd.EUNSUPPORTED  # real dtype
    # caller-owned scratch: the query, then a missing, misaligned or short workspace
    for dt in (hd.C128, hd.C64, hd.CBF16):
        for nv in (1, 3, 12, 42):
            need = hd._binding.born_workspace_bytes(op, 4, 4, dt, hd.BORN_NATIVE, nv)
            assert need > 0 and need % 8 == 0
            assert f(op.handle, fake, 4, fake, 4, 8, dt, fake, nv, fake, fake, need - 8, None) == hd.ENOMEM
            assert "workspace" in hd._binding._last_error().decode()
    assert f(op.handle, fake, 4, fake, 4, 8, 1, fake, 1, fake, None, big, None) == hd.EINVAL        # no workspace
    assert f(op.handle, fake, 4, fake, 4, 8, 1, fake, 1, fake, ctypes.c_void_p(0x7F0000000008), big,
             None) == hd.EINVAL                                                                     # misaligned
    # the split partials grow with the requested grid size, and the plan is the same for the query
    # and the call: a workspace of exactly the queried size passes validation
    need1 = hd._binding.born_workspace_bytes(op, 4, 4, hd.C64, hd.BORN_NATIVE, 1)
    hd.set_tuning(op, born_blocks=256)
    need2 = hd._binding.born_workspace_bytes(op, 4, 4, hd.C64, hd.BORN_NATIVE, 1)
    assert need2 < need1
    with pytest.raises(hd.HydotError):
        hd._binding.born_workspace_bytes(op, 4, 4, hd.C64, hd.BORN_SPLIT_BF16 + 5, 1)
    g = lib.hydot_born_apply_adjoint
    g.restype = ctypes.c_int32
    g.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert g(op.handle, None, 4, fake, 4, 8, 0, fake, fake, None) == hd.EINVAL


def test_pals_and_misfit_validate(hd):
    w = workloads.config("tiny")
    op = _op(hd, w)
    lib = _raw(hd)
    from paper_1410_0986_amd._binding import _PalsOpts
    f = lib.hydot_pals_shape
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int32, ctypes.c_void_p]
    p = np.zeros(5 * 40)
    pp = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    po = _PalsOpts(0.5, 0.5, 1e-3)
    fake = ctypes.c_void_p(0x7F0000000000)
    assert f(op.handle, pp, 40, ctypes.byref(po), fake, 3, None) == hd.EINVAL   # too many bumps
    po_bad = _PalsOpts(0.5, 0.0, 1e-3)
    assert f(op.handle, pp, 8, ctypes.byref(po_bad), fake, 3, None) == hd.EINVAL  # eps = 0
    assert f(op.handle, pp, 8, ctypes.byref(po), fake, 0, None) == hd.EUNSUPPORTED  # complex mu
    assert lib.hydot_misfit_workspace_bytes(op.handle, 4, 4) > 0


def test_tuning_defaults_and_validation(hd):
    op = _op(hd, workloads.config("tiny"))
    t = hd.get_tuning(op)
    assert t == {"step_presum": 16, "step_order": 3, "step_group": 2, "born_stage": 0, "born_blocks": 4096,
                 "step_vx": 1, "step_pair": 2}
    hd.set_tuning(op, step_presum=4, step_order=1, born_stage=16, born_blocks=1024)
    t = hd.get_tuning(op)
    assert (t["step_presum"], t["step_order"], t["born_stage"], t["born_blocks"]) == (4, 1, 16, 1024)
    for bad in (dict(step_presum=3), dict(step_order=5), dict(step_group=-1), dict(born_stage=64),
                dict(born_blocks=100), dict(born_blocks=1 << 17), dict(step_vx=3), dict(step_vx=2, step_presum=2),
                dict(step_pair=3), dict(step_pair=-1)):
        with pytest.raises(hd.HydotError) as e:
            hd.set_tuning(op, **bad)
        assert e.value.status == hd.EINVAL
    assert hd.get_tuning(op)["step_order"] == 1   # a rejected call changes nothing
    hd.set_tuning(op, step_presum=1, step_order=0, born_stage=0, born_blocks=0)
    assert hd.get_tuning(op)["step_presum"] == 1 and hd.get_tuning(op)["step_order"] == 3
    hd.set_tuning(op, step_presum=0)
    assert hd.get_tuning(op)["step_presum"] == 16
    hd.set_tuning(op, step_presum=16, step_vx=1)
    with pytest.raises(hd.HydotError):
        hd.set_tuning(op, step_presum=16, step_vx=2)


def test_shift_flags_are_exclusive(hd):
    op = _op(hd, workloads.config("tiny"))
    for fl in (hd.FLAG_MEAN_SHIFT | hd.FLAG_SHIFT_MIN, hd.FLAG_SHIFT_MIN | hd.FLAG_SHIFT_MAX):
        with pytest.raises(hd.HydotError) as e:
            hd.solve_workspace_bytes(op, 4, hd.SolveOptions(flags=fl))
        assert e.value.status == hd.EINVAL
    assert hd.solve_workspace_bytes(op, 4, hd.SolveOptions(flags=hd.FLAG_SHIFT_MAX)) > 0


def test_preconditioner_flag_validation(hd):
    w = workloads.config("tiny")
    op = hd.Operator.from_workload(w)
    R = w.S + w.D
    base = dict(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, inner_tol=1e-5)
    ok = hd.SolveOptions(precision=hd.PREC_MIXED, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PRECOND_SEP, **base)
    plain = hd.SolveOptions(precision=hd.PREC_MIXED, flags=hd.FLAG_MEAN_SHIFT, **base)
    # the preconditioned plan holds one more vector per system
    assert hd.solve_workspace_bytes(op, R, ok) >= hd.solve_workspace_bytes(op, R, plain) + R * w.L * w.N * 8
    cases = [(dict(precision=hd.PREC_MIXED, flags=hd.FLAG_PRECOND_SEP | hd.FLAG_PRECOND_SEP_FIXED), hd.EINVAL),
             (dict(precision=hd.PREC_FP64, flags=hd.FLAG_PRECOND_SEP), hd.EUNSUPPORTED)]
    for kw, status in cases:
        with pytest.raises(hd.HydotError) as e:
            hd.solve_workspace_bytes(op, R, hd.SolveOptions(**{**base, **kw}))
        assert e.value.status == status
    big = dict(base, restart_m=45, recycle_k=5)
    with pytest.raises(hd.HydotError) as e:
        hd.solve_workspace_bytes(op, R, hd.SolveOptions(precision=hd.PREC_MIXED, flags=hd.FLAG_PRECOND_SEP, **big))
    assert e.value.status == hd.EUNSUPPORTED


def test_binding_constants_mirror_header(hd):
    text = open(HEADER).read()
    m = re.search(r"#define\s+HYDOT_BORN_PAIRS_MIN_NV\s+(\d+)", text)
    assert m and int(m.group(1)) == hd.BORN_PAIRS_MIN_NV


def test_solve_rejects_basis_beyond_buffer_range(hd):
    """The FP32 step kernels address a system's Krylov basis through 32-bit byte offsets: a
    512 x 512 x 256 grid with restart_m - recycle_k = 4 needs 5 x 2^26 x 8 B > 2 GiB per system."""
    w = workloads.config("tiny", nx=512, ny=512, nz=256, n_lambda=2)
    op = _op(hd, w)
    mixed = hd.SolveOptions(restart_m=8, recycle_k=4, lanczos_n=8, precision=hd.PREC_MIXED)
    with pytest.raises(hd.HydotError) as e:
        hd.solve_workspace_bytes(op, 2, mixed)
    assert e.value.status == hd.EUNSUPPORTED
    # the FP64 path has no such limit
    assert hd.solve_workspace_bytes(op, 2, hd.SolveOptions(restart_m=8, recycle_k=4, lanczos_n=8,
                                                           precision=hd.PREC_FP64)) > 0


def test_solve_inspect_validates(hd):
    """hydot_solve_inspect checks the item, the index and the buffers before any copy."""
    from paper_1410_0986_amd import _binding as B
    w = workloads.config("tiny")
    op = _op(hd, w)
    opts = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24)
    need = hd.solve_workspace_bytes(op, 8, opts)
    o = opts._c()
    info = B._InspectInfo()
    fake = ctypes.c_void_p(0x7F0000000000)
    f = B._inspect
    assert f(op.handle, 8, ctypes.byref(o), fake, need - 256, 0, 0, None, 0, ctypes.byref(info), None) == hd.ENOMEM
    assert f(op.handle, 8, ctypes.byref(o), fake, need, 7, 0, None, 0, ctypes.byref(info), None) == hd.EINVAL
    assert f(op.handle, 8, ctypes.byref(o), fake, need, B.INSPECT_U, 8, None, 0, ctypes.byref(info), None) == hd.EINVAL
    assert f(op.handle, 8, ctypes.byref(o), fake, need, B.INSPECT_U, 3, None, 0, ctypes.byref(info), None) == hd.OK
    assert info.k == 5 and info.rhs == 3
    out = np.empty(10)
    assert f(op.handle, 8, ctypes.byref(o), fake, need, B.INSPECT_C, 3, ctypes.c_void_p(out.ctypes.data), out.nbytes,
             ctypes.byref(info), None) == hd.ENOMEM
    assert f(op.handle, 8, ctypes.byref(o), ctypes.c_void_p(0x7F0000000008), need, B.INSPECT_U, 3, None, 0,
             ctypes.byref(info), None) == hd.EINVAL
    nr = hd.SolveOptions(rel_tol=1e-8, restart_m=18, recycle_k=5, lanczos_n=24, flags=hd.FLAG_NO_RECYCLE)
    o2 = nr._c()
    need2 = hd.solve_workspace_bytes(op, 8, nr)
    assert f(op.handle, 8, ctypes.byref(o2), fake, need2, B.INSPECT_U, 0, None, 0, ctypes.byref(info), None) == hd.EINVAL


def test_measure_peaks_validates_before_launch(hd):
    lib = _raw(hd)
    f = lib.hydot_measure_peaks
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    out = hd._binding._Peaks()
    fake = ctypes.c_void_p(0x7F0000000000)
    assert f(None, 1 << 31, ctypes.byref(out), None) == hd.EINVAL                         # null buffer
    assert f(fake, 1 << 31, None, None) == hd.EINVAL                                      # null output
    assert f(ctypes.c_void_p(0x7F0000000010), 1 << 31, ctypes.byref(out), None) == hd.EINVAL   # misaligned
    assert f(fake, (1 << 30) - 256, ctypes.byref(out), None) == hd.EINVAL                 # under 1 GiB


# ctypes structures of the binding and the C types they marshal
_STRUCTS = {"_Grid": "hydot_grid", "_Optics": "hydot_optics", "_SolveOpts": "hydot_solve_opts",
            "_PalsOpts": "hydot_pals_opts", "_SolveProblem": "hydot_solve_problem", "_InspectInfo": "hydot_inspect_info",
            "_Peaks": "hydot_peaks", "_Tuning": "hydot_tuning", "_Trial": "hydot_tune_trial",
            "_KProf": "hydot_kernel_profile"}


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs a host C++ compiler and the HIP headers")
def test_binding_structs_match_the_header(hd, tmp_path):
    """Every structure the binding passes through the C ABI has the size and field offsets the
    header gives it (compiled with the host compiler)."""
    from paper_1410_0986_amd import _binding as b
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "hydot.h"', 'int main() {']
    expect = []
    for py, c in _STRUCTS.items():
        cls = getattr(b, py)
        lines.append(f'  std::printf("%zu\\n", sizeof({c}));')
        expect.append(ctypes.sizeof(cls))
        for name, *_ in cls._fields_:
            lines.append(f'  std::printf("%zu\\n", offsetof({c}, {name}));')
            expect.append(getattr(cls, name).offset)
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect
