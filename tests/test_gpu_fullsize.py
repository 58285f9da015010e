"""Full-size parity: the workloads at their real shapes, in the launch configuration
bench.py times, checked on outputs the oracle computes one by one (whole fields of
sampled systems by fast diagonalisation, Born products at sampled wavelengths and
voxels) and on properties that hold at any size (every FP64 residual, the adjoint
identity, finite differences of the misfit)."""
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


def bench_opts(hd, **kw):
    import bench
    base = dict(rel_tol=1e-8, restart_m=bench.RESTART_M, recycle_k=bench.RECYCLE_K, lanczos_n=bench.LANCZOS_N,
                precision=hd.PREC_MIXED, inner_tol=bench.INNER_TOL,
                flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH, max_iter=5000)
    base.update(kw)
    return hd.SolveOptions(**base)


def normwise(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def medium(hd):
    w = workloads.config("medium")
    op = hd.Operator.from_workload(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, bench_opts(hd), out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    return w, op, phi, it, rel, st


def test_medium_every_system_meets_tolerance(hd, medium):
    w, op, phi, it, rel, st = medium
    assert st == hd.OK
    assert rel.shape == (w.L, w.S + w.D)
    assert rel.max() <= 1e-8
    assert np.all(it > 0)


@pytest.mark.parametrize("lam,r", [(0, 0), (31, 31), (7, 16), (19, 5), (24, 27)])
def test_medium_sampled_fields(hd, medium, lam, r):
    w, op, phi, it, rel, st = medium
    ref = ofields.solve_separable(w, voxels=[w.rhs_voxels[r]], lam_idx=[lam])[0, 0]
    got = phi[lam, r].cpu().numpy().astype(np.complex128)
    assert normwise(got, ref) < 1e-4


def test_medium_born_sampled(hd, medium):
    w, op, phi, it, rel, st = medium
    S = w.S
    v = workloads.born_v(w, dtype=np.float32)
    y = hd.born_apply(op, phi[:, :S], phi[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy()[0]
    for lam in (3, 29):
        P = ofields.solve_separable(w, lam_idx=[lam])
        yref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)[0, 0]
        assert normwise(y[lam].astype(np.complex128), yref) < 1e-4
        # the kernel entry by entry against the exact products of the stored fields (far pairs
        # depend on field values far below the solve's normwise tolerance, so the fields are
        # held to the oracle separately)
        _born_entrywise(w, phi, v, y, lam)
    # J^H w at sampled voxels: every (lambda, rhs) field evaluated there one by one
    wv = workloads.born_w(w)
    g = hd.born_apply_adjoint(op, phi[:, :S], phi[:, S:], torch.from_numpy(wv).to(torch.complex64).to(DEV))
    g = g.cpu().numpy().astype(np.complex128)
    pts = np.array([w.src_voxels[5], w.det_voxels[9], w.N // 2 + 17, w.N // 3])
    F = np.empty((w.L, w.S + w.D, len(pts)), dtype=np.complex128)
    for lam in range(w.L):
        for r, vox in enumerate(w.rhs_voxels):
            F[lam, r] = ofields.separable_at(w, lam, int(vox), pts)
    gref = oborn.born_apply_adjoint(F[:, :S], F[:, S:], wv, w.h)
    assert np.abs(g[pts] - gref).max() <= 1e-4 * np.abs(gref).max()
    # adjoint identity over the whole grid (both products from the device)
    lhs = np.vdot(wv.reshape(-1), y.reshape(-1).astype(np.complex128))
    rhs = np.vdot(g, v[0].astype(np.float64))
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def _born_entrywise(w, phi, v, y, lam, tol=1e-5):
    """J v of one probe vector at wavelength lam (y: [L][S][D]) against the FP64 products of the
    device's own FP32 fields, every (source, detector) entry within tol of the absolute sum of its
    terms."""
    S = w.S
    F = phi[lam].cpu().numpy().astype(np.complex128)
    vd = v[0].astype(np.float64)
    ref = oborn.born_apply(F[None, :S], F[None, S:], vd[None], w.h)[0, 0]
    absum = w.h ** 3 * np.einsum("sk,k,dk->sd", np.abs(F[:S]), np.abs(vd), np.abs(F[S:]), optimize=True)
    err = np.abs(y[lam].astype(np.complex128) - ref)
    assert np.all(err <= tol * absum), float((err / absum).max())


def test_medium_born_jacobian_block_sampled(hd, medium):
    """The 42-column block (2 contrasts + 40 PaLS parameters) takes the pair-product kernel at
    the full medium shape: sampled wavelengths against the oracle's fields."""
    w, op, phi, it, rel, st = medium
    S = w.S
    v = workloads.born_v(w, n_v=42, seed=2024, dtype=np.float32)
    assert v.shape[0] >= hd.BORN_PAIRS_MIN_NV
    y = hd.born_apply(op, phi[:, :S], phi[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy()
    for lam in (0, 17):
        P = ofields.solve_separable(w, lam_idx=[lam])
        yref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)[:, 0]
        got = y[:, lam].astype(np.complex128)
        assert np.max(np.linalg.norm((got - yref).reshape(42, -1), axis=1)
                      / np.linalg.norm(yref.reshape(42, -1), axis=1)) < 1e-4


def test_medium_plain_fp64_subset(hd):
    """The plain per-system FP64 path at full grid size: one source at 4 wavelengths, 1e-8 field parity."""
    w = workloads.subset_lambdas(workloads.config("medium"), [0, 10, 20, 31])
    w.src_voxels = w.src_voxels[3:4]
    w.det_voxels = w.det_voxels[:0]
    op = hd.Operator.from_workload(w)
    o = hd.SolveOptions(rel_tol=1e-11, restart_m=40, recycle_k=10, lanczos_n=40,
                        flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PER_SYSTEM)
    phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, o, device=DEV)
    assert st == hd.OK and rel.max() <= 1e-11
    ref = ofields.solve_separable(w)
    got = phi.cpu().numpy()
    for lam in range(w.L):
        assert normwise(got[lam, 0], ref[lam, 0]) < 1e-8


def test_batch_config_sampled(hd):
    """64 right-hand sides x 64 wavelengths in one batched launch."""
    torch.cuda.empty_cache()
    w = workloads.config("batch")
    op = hd.Operator.from_workload(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, bench_opts(hd), out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    for lam, r in [(0, 63), (40, 2), (63, 31)]:
        ref = ofields.solve_separable(w, voxels=[w.rhs_voxels[r]], lam_idx=[lam])[0, 0]
        assert normwise(phi[lam, r].cpu().numpy().astype(np.complex128), ref) < 1e-4
    S = w.S
    v = workloads.born_v(w, dtype=np.float32)
    y = hd.born_apply(op, phi[:, :S], phi[:, S:], torch.from_numpy(v).to(DEV)).cpu().numpy()[0]
    for lam in (0, 21, 50, 63):
        P = ofields.solve_separable(w, lam_idx=[lam])
        yref = oborn.born_apply(P[:, :S], P[:, S:], v.astype(np.float64), w.h)[0, 0]
        assert normwise(y[lam].astype(np.complex128), yref) < 1e-4, lam
    for lam in (21, 63):
        _born_entrywise(w, phi, v, y, lam)


def _large_shards(w, n_shards=8):
    return [workloads.subset_lambdas(w, np.arange(i * w.L // n_shards, (i + 1) * w.L // n_shards))
            for i in range(n_shards)]


@pytest.mark.timeout(1100)
def test_large_config_sampled(hd):
    """128x128x64 grid (1048576 voxels), 64 + 64 right-hand sides, 128 wavelengths 650-1000 nm,
    with its three companion grids (32x32x16, 48x48x24, 80x80x40) in one batch per wavelength
    shard, in the launch configuration bench.py times: eight shards of 16 wavelengths (2048
    main-grid systems each, batches of 512; 2304 companion-grid systems) into complex FP32
    fields.  Every one of the 16384 main-grid and 18432 companion-grid systems meets rel-res
    1e-8; sampled fields of every grid against the oracle's fast diagonalisation at the
    mixed-path tolerance 1e-4; on the first shard, every grid's output of the batch equals its
    own single solve exactly; on one shard, FP32 and split-BF16 J v at near source-detector
    pairs against the oracle's fields entrywise, and J^H w at sampled voxels against the
    oracle's point evaluations."""
    torch.cuda.empty_cache()
    w = workloads.config("large")
    shards = _large_shards(w)
    comp = [workloads.config(c) for c in ("large_g32", "large_g48", "large_g80")]
    comp_shards = [_large_shards(cw) for cw in comp]
    S, R, N = w.S, w.S + w.D, w.N
    Ls = shards[0].L
    s = torch.cuda.Stream()
    opts = bench_opts(hd, max_batch=512)
    copts = bench_opts(hd, max_batch=1024)
    samples = {0: [(0, 0)], 4: [(13, 100)], 7: [(15, 63)]}      # shard: (wavelength in shard, rhs)
    comp_samples = {2: (3, 0), 6: (12, -1)}                     # shard: (wavelength in shard, rhs)
    jv_shard = 5
    with torch.cuda.stream(s):
        phi = torch.empty((Ls, R, N), dtype=torch.complex64, device=DEV)
        cphi = [torch.empty((Ls, cw.S + cw.D, cw.N), dtype=torch.complex64, device=DEV) for cw in comp]
    for i, ws in enumerate(shards):
        op = hd.Operator.from_workload(ws)
        cws = [cs[i] for cs in comp_shards]
        cops = [hd.Operator.from_workload(c) for c in cws]
        with torch.cuda.stream(s):
            res = hd.solve_fields_batch([(op, ws.rhs_voxels, opts, phi)] +
                                        [(co, c.rhs_voxels, copts, cp) for co, c, cp in zip(cops, cws, cphi)])
        s.synchronize()
        for g, (_, it, rel, st) in enumerate(res):
            assert st == hd.OK and rel.max() <= 1e-8, (i, g, rel.max())
        it, rel = res[0][1], res[0][2]
        assert rel.shape == (Ls, R)
        print(f"large shard {i}: {Ls * R} + {sum(r[2].size for r in res[1:])} systems in one batch, max rel-res "
              f"{max(r[2].max() for r in res):.2e}, mean iters {it.mean():.1f}", flush=True)
        for lam, r in samples.get(i, []):
            ref = ofields.solve_separable(ws, voxels=[ws.rhs_voxels[r]], lam_idx=[lam])[0, 0]
            assert normwise(phi[lam, r].cpu().numpy().astype(np.complex128), ref) < 1e-4, (i, lam, r)
        if i in comp_samples:
            lam, r = comp_samples[i]
            for c, cp in zip(cws, cphi):
                ref = ofields.solve_separable(c, voxels=[c.rhs_voxels[r]], lam_idx=[lam])[0, 0]
                assert normwise(cp[lam, r].cpu().numpy().astype(np.complex128), ref) < 1e-4, (i, c.nx, lam, r)
        if i == 0:
            # the batch changes no problem's arithmetic: each grid alone gives the same bits
            for g, (o_, c_, o2, p_) in enumerate([(op, ws, opts, phi)] +
                                                 [(co, c, copts, cp) for co, c, cp in zip(cops, cws, cphi)]):
                with torch.cuda.stream(s):
                    p1, it1, rel1, st1 = hd.solve_fields(o_, c_.rhs_voxels, o2, out_dtype=torch.complex64,
                                                         device=DEV)
                s.synchronize()
                assert st1 == hd.OK and torch.equal(p1, p_), g
                np.testing.assert_array_equal(it1, res[g][1])
                np.testing.assert_array_equal(rel1, res[g][2])
                del p1
            torch.cuda.empty_cache()
        if i == jv_shard:
            _large_born_checks(hd, ws, op, phi, s)
    del phi, cphi
    torch.cuda.empty_cache()


def _large_born_checks(hd, ws, op, phi, s):
    S, N, h = ws.S, ws.N, ws.h
    lam = 9
    v = workloads.born_v(ws, dtype=np.float32)
    vt = torch.from_numpy(v).to(DEV)
    with torch.cuda.stream(s):
        y32 = hd.born_apply(op, phi[:, :S], phi[:, S:], vt)
        ysp = hd.born_apply(op, phi[:, :S], phi[:, S:], vt, split_bf16=True)
    s.synchronize()
    # near pairs: source (a, b) and detector (a, b) of the same cell of the 8 x 8 optode arrays
    # (22.6 mm apart); their sums are dominated by voxels where both fields are resolved
    pairs = [0, 9, 27, 36, 54, 63]
    P = ofields.solve_separable(ws, voxels=[ws.src_voxels[q] for q in pairs] + [ws.det_voxels[q] for q in pairs],
                                lam_idx=[lam])[0]
    Ps, Pd = P[:len(pairs)], P[len(pairs):]
    yref = -(h ** 3) * np.einsum("pk,k,pk->p", Ps, v[0].astype(np.float64), Pd)
    absum = h ** 3 * np.einsum("pk,k,pk->p", np.abs(Ps), np.abs(v[0].astype(np.float64)), np.abs(Pd))
    print("large J v near pairs: oracle fields done", flush=True)
    for name, y in (("fp32", y32), ("split_bf16", ysp)):
        got = y.cpu().numpy()[0, lam][pairs, pairs].astype(np.complex128)
        print(f"  {name}: max entry error / absolute sum {(np.abs(got - yref) / absum).max():.2e}, "
              f"normwise {normwise(got, yref):.2e}", flush=True)
        assert np.all(np.abs(got - yref) <= 1e-4 * absum), (name, (np.abs(got - yref) / absum).max())
        assert normwise(got, yref) < 1e-4, name
    # J^H w at sampled voxels: every (wavelength, rhs) field of the shard evaluated there one by one
    wv = workloads.born_w(ws)
    with torch.cuda.stream(s):
        g = hd.born_apply_adjoint(op, phi[:, :S], phi[:, S:], torch.from_numpy(wv).to(torch.complex64).to(DEV))
    s.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    pts = np.array([ws.src_voxels[20] - ws.nx * ws.ny * 2, ws.det_voxels[41], N // 2 + 33, N - 1 - 517])
    F = np.empty((ws.L, ws.S + ws.D, len(pts)), dtype=np.complex128)
    for l in range(ws.L):
        for r, vox in enumerate(ws.rhs_voxels):
            F[l, r] = ofields.separable_at(ws, l, int(vox), pts)
    gref = oborn.born_apply_adjoint(F[:, :S], F[:, S:], wv, h)
    print(f"large J^H w at sampled voxels: max error / max |g| {np.abs(g[pts] - gref).max() / np.abs(gref).max():.2e}",
          flush=True)
    assert np.abs(g[pts] - gref).max() <= 1e-4 * np.abs(gref).max()
    # BF16-stored fields of this shard, solved by the library into BF16: within one BF16 rounding
    # of the FP32 fields plus the solve error, and BF16 J v at the near pairs against the exact
    # products of the operands the kernel multiplies (bf16(phi_s v), stored phi_d), within the
    # FP32 accumulation of 32-voxel stages
    with torch.cuda.stream(s):
        phb, _, relb, stb = hd.solve_fields(op, ws.rhs_voxels, bench_opts(hd, max_batch=512), out_dtype=torch.bfloat16,
                                           device=DEV)
        yb = hd.born_apply(op, phb[:, :S], phb[:, S:], vt)
    s.synchronize()
    assert stb == hd.OK and relb.max() <= 1e-8

    def fieldb(r):
        return torch.view_as_complex(phb[lam, r].float().contiguous()).cpu().numpy().astype(np.complex128)

    src = [pairs[1], pairs[4]]
    gotb = yb.cpu().numpy()[0, lam][src, src].astype(np.complex128)
    for q, sidx in enumerate(src):
        fs = torch.from_numpy(fieldb(sidx))
        vb = torch.from_numpy(v[0])
        A = (fs.real.float() * vb).to(torch.bfloat16).double().numpy() + \
            1j * (fs.imag.float() * vb).to(torch.bfloat16).double().numpy()
        Bd = fieldb(S + sidx)
        exp = -(h ** 3) * np.sum(A * Bd)
        bound = h ** 3 * np.sum(np.abs(A) * np.abs(Bd))
        assert abs(gotb[q] - exp) <= 1e-5 * bound
        ref = Ps[pairs.index(sidx)]
        assert normwise(fieldb(sidx), ref) < 4e-3
    del phb


@pytest.mark.parametrize("name", ["large_g32", "large_g48", "large_g80"])
def test_large_companion_grids(hd, name):
    """The three smaller grids of the large workload (128 wavelengths 650-1000 nm), each a
    separate operator solved in full by the batched path (complex FP32 output; at most 2048
    systems per batch: the 80^3-class grid's 8192 systems would need a 333 GB workspace)."""
    torch.cuda.empty_cache()
    w = workloads.config(name)
    op = hd.Operator.from_workload(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, bench_opts(hd, max_batch=2048),
                                           out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.shape == (w.L, w.S + w.D) and rel.max() <= 1e-8
    R = w.S + w.D
    for lam, r in [(0, R - 1), (100, 1)]:
        ref = ofields.solve_separable(w, voxels=[w.rhs_voxels[r]], lam_idx=[lam])[0, 0]
        assert normwise(phi[lam, r].cpu().numpy().astype(np.complex128), ref) < 1e-4
    del phi


def test_diff_config_fields_and_gradient(hd):
    """96x96x48 grid, 24+24 optodes, 48 wavelengths in two batches; misfit gradient by the
    adjoint kernels against central finite differences of the device misfit (FP64 fields)."""
    torch.cuda.empty_cache()
    w = workloads.config("diff")
    op = hd.Operator.from_workload(w)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi, it, rel, st = hd.solve_fields(op, w.rhs_voxels, bench_opts(hd, max_batch=w.L * 24),
                                           out_dtype=torch.complex64, device=DEV)
    s.synchronize()
    assert st == hd.OK and rel.max() <= 1e-8
    for lam, r in [(0, 0), (47, 47), (23, 30)]:
        ref = ofields.solve_separable(w, voxels=[w.rhs_voxels[r]], lam_idx=[lam])[0, 0]
        assert normwise(phi[lam, r].cpu().numpy().astype(np.complex128), ref) < 1e-4
    S = w.S
    # the differentiation workload's anomaly: 8 Gaussian bumps, widths 3-8 mm
    po = hd.PalsOptions(basis=hd.PALS_GAUSSIAN)
    p_true, dc_true = workloads.pals_truth(w, basis="gaussian")
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)
    ph = phi.to(torch.complex128)
    mu_t = hd.pals_shape(op, p_true, po, device=DEV)
    Jmu = hd.born_apply(op, ph[:, :S], ph[:, S:], mu_t[None])[0]
    ebar = torch.from_numpy(dc_true @ w.extinction).to(DEV)
    y_obs = ebar[:, None, None] * Jmu
    x = np.concatenate([dc, p])
    xt = torch.tensor(x, requires_grad=True)
    f = hd.BornMisfit.apply(xt[:2], xt[2:], op, ph[:, :S], ph[:, S:], y_obs, po)
    f.backward()
    g = xt.grad.numpy()
    assert f.item() > 0

    def f_of(xx):
        return hd.BornMisfit.apply(torch.tensor(xx[:2]), torch.tensor(xx[2:]), op, ph[:, :S], ph[:, S:],
                                   y_obs, po).item()

    for i in (0, 1, 2, 9, 17, 25, 33, 41):
        st_ = 1e-6 * max(1.0, abs(x[i]))
        xu, xd = x.copy(), x.copy()
        xu[i] += st_
        xd[i] -= st_
        fd = (f_of(xu) - f_of(xd)) / (2 * st_)
        assert abs(fd - g[i]) <= 1e-5 * np.abs(g).max() + 1e-5 * abs(g[i])
    # zero gradient at the truth (noise-free data)
    xt0 = torch.tensor(np.concatenate([dc_true, p_true]), requires_grad=True)
    f0 = hd.BornMisfit.apply(xt0[:2], xt0[2:], op, ph[:, :S], ph[:, S:], y_obs, po)
    f0.backward()
    assert f0.item() <= 1e-12 * f.item()
    assert np.abs(xt0.grad.numpy()).max() <= 1e-6 * np.abs(g).max()
