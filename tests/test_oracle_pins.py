"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: an
independent loop-built matrix, the exact lattice Green's function, the
continuum point-source solution, a 1-D closed form, reciprocity, finite
differences of direct solves, the adjoint identity, and the PaLS chain rule.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.special as ss

import workloads
from oracle import born, fields, model, pals


def custom_workload(nx, ny, nz, h, D, mua, robin_faces=workloads.ALL_ROBIN, A_R=2.5, n_lambda=1):
    """Workload with prescribed D and mu_a (single chromophore of unit concentration)."""
    lam = np.full(n_lambda, 700.0)
    return workloads.Workload(
        name="custom", nx=nx, ny=ny, nz=nz, h=h, A_R=A_R, robin_faces=robin_faces,
        lambdas_nm=lam, mus_prime=np.full(n_lambda, 1.0 / (3.0 * D)),
        extinction=np.full((1, n_lambda), mua), conc_uM=np.array([1.0]),
        omega_over_nu=workloads.omega_over_nu(),
        src_voxels=np.array([0], dtype=np.int64), det_voxels=np.array([nx * ny * nz - 1], dtype=np.int64))


def loop_built_operator(w, lam_idx):
    """A(lambda) assembled voxel by voxel and face by face (independent of the Kronecker form)."""
    D = 1.0 / (3.0 * w.mus_prime[lam_idx])
    mua = float(np.dot(w.conc_uM, w.extinction[:, lam_idx]))
    s = mua + 1j * w.omega_over_nu
    A = np.zeros((w.N, w.N), dtype=np.complex128)
    dims = (w.nx, w.ny, w.nz)
    for k in range(w.nz):
        for j in range(w.ny):
            for i in range(w.nx):
                n = i + w.nx * (j + w.ny * k)
                A[n, n] += s * w.h ** 3
                idx = [i, j, k]
                for axis in range(3):
                    for side, step in ((0, -1), (1, +1)):
                        q = list(idx)
                        q[axis] += step
                        if 0 <= q[axis] < dims[axis]:
                            m = q[0] + w.nx * (q[1] + w.ny * q[2])
                            A[n, n] += D * w.h
                            A[n, m] -= D * w.h
                        elif (w.robin_faces >> (2 * axis + side)) & 1:
                            A[n, n] += w.h ** 2 / (2.0 * w.A_R)
                        else:
                            A[n, n] += 2.0 * D * w.h
    return A


@pytest.mark.parametrize("faces", [workloads.ALL_ROBIN, 0x30, 0x0F, 0x2D])
def test_assembly_matches_loop_builder(faces):
    w = workloads.config("tiny", nx=5, ny=4, nz=3)
    w.robin_faces = faces
    for j in (0, 3):
        A_loop = loop_built_operator(w, j)
        A_kron = model.operator(w, j).toarray()
        np.testing.assert_allclose(A_kron, A_loop, rtol=1e-15, atol=1e-14)


def test_all_solvers_agree_with_brute_force():
    w = workloads.config("tiny", nx=6, ny=5, nz=4)
    w.robin_faces = 0x33   # Robin on x and z faces, Dirichlet on y faces
    w.src_voxels = np.array([3, 17], dtype=np.int64)
    w.det_voxels = np.array([100, 119], dtype=np.int64)
    lams = [0, 7]
    ref = np.empty((2, w.S + w.D, w.N), dtype=np.complex128)
    for a, j in enumerate(lams):
        A = loop_built_operator(w, j)
        Bm = np.zeros((w.N, w.S + w.D))
        Bm[w.rhs_voxels, np.arange(w.S + w.D)] = 1.0
        ref[a] = np.linalg.solve(A, Bm).T
    for route in (fields.solve_dense(w, lam_idx=lams), fields.solve_banded(w, lam_idx=lams),
                  fields.solve_separable(w, lam_idx=lams),
                  fields.solve_gmres(w, lam_idx=lams, tol=1e-14)[0]):
        err = np.linalg.norm(route - ref, axis=2) / np.linalg.norm(ref, axis=2)
        assert err.max() < 1e-11


def test_separable_point_evaluation():
    w = workloads.config("tiny")
    full = fields.solve_separable(w, lam_idx=[2])[0]
    pts = np.array([0, 5, 77, 1023, 2047, int(w.det_voxels[1])])
    for r, v in enumerate(w.rhs_voxels):
        got = fields.separable_at(w, 2, int(v), pts)
        np.testing.assert_allclose(got, full[r, pts], rtol=1e-10, atol=1e-12 * np.abs(full[r]).max())


def _lattice_green(a, n):
    """G_a(n) = int_0^inf exp(-a t) prod_i exp(-2t) I_{n_i}(2t) dt: (L_lattice + a) G = delta on Z^3."""
    n = [abs(int(x)) for x in n]

    def f(t):
        return np.exp(-a * t) * ss.ive(n[0], 2 * t) * ss.ive(n[1], 2 * t) * ss.ive(n[2], 2 * t)

    re = si.quad(lambda t: f(t).real, 0, np.inf, limit=4000, epsabs=0, epsrel=1e-13)[0]
    im = si.quad(lambda t: f(t).imag, 0, np.inf, limit=4000, epsabs=0, epsrel=1e-13)[0]
    return re + 1j * im


def test_interior_field_is_lattice_green_function():
    """Deep inside a large box the discrete field equals the exact lattice Green's function / (D h)."""
    D, mua, h, n = 0.5, 0.03, 2.0, 96
    w = custom_workload(n, n, n, h, D, mua)
    s = mua + 1j * w.omega_over_nu
    a = s * h ** 3 / (D * h)
    c = n // 2
    src = c + n * (c + n * c)
    offsets = [(0, 0, 0), (1, 0, 0), (2, 1, 0), (3, 3, 3), (5, 2, 1), (8, 0, 0), (10, 5, 3), (15, 0, 0)]
    pts = [(c + o[0]) + n * ((c + o[1]) + n * (c + o[2])) for o in offsets]
    got = fields.separable_at(w, 0, src, pts)
    for o, g in zip(offsets, got):
        exact = _lattice_green(a, o) / (D * h)
        assert abs(g - exact) / abs(exact) < 1e-8, (o, g, exact)


def test_continuum_green_function_second_order():
    """phi -> exp(-k r)/(4 pi D r) at fixed r with error O(h^2) (infinite-medium solution)."""
    D, mua = 0.5, 0.03
    s = mua + 1j * workloads.omega_over_nu()
    k = np.sqrt(s / D)
    radii = np.array([8.0, 12.0, 16.0])
    errs = []
    for h, n in ((2.0, 41), (1.0, 81), (0.5, 161)):
        w = custom_workload(n, n, n, h, D, mua)
        c = (n - 1) // 2
        src = c + n * (c + n * c)
        pts = [(c + int(round(r / h))) + n * (c + n * c) for r in radii]
        got = fields.separable_at(w, 0, src, pts)
        exact = np.exp(-k * radii) / (4 * np.pi * D * radii)
        errs.append(np.abs(got - exact) / np.abs(exact))
    errs = np.array(errs)
    assert errs[0].max() < 0.15
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.0) and np.all(ratios < 5.5), ratios


def test_one_dimensional_chain_closed_form():
    """nx = ny = 1: a chain whose lateral Robin faces add 4 h^2/(2 A_R) per voxel; the far-from-end
    field is rho^|n| / (D h (1/rho - rho)) with rho + 1/rho = 2 + a."""
    D, mua, h, nz = 0.6, 0.02, 2.0, 801
    w = custom_workload(1, 1, nz, h, D, mua, A_R=50.0)
    s = mua + 1j * w.omega_over_nu
    a = (4 * h ** 2 / (2 * w.A_R) + s * h ** 3) / (D * h)
    rho = ((2 + a) - np.sqrt((2 + a) ** 2 - 4)) / 2
    if abs(rho) > 1:
        rho = 1 / rho
    c = nz // 2
    pts = np.arange(c - 20, c + 21)
    got = fields.separable_at(w, 0, c, pts)
    exact = rho ** np.abs(pts - c) / (D * h * (1 / rho - rho))
    np.testing.assert_allclose(got, exact, rtol=1e-10, atol=1e-13 * abs(exact).max())


def test_reciprocity_of_fields():
    w = workloads.config("tiny")
    for route in (fields.solve_banded(w, lam_idx=[1, 6]), fields.solve_gmres(w, lam_idx=[1, 6], tol=1e-13)[0]):
        for a in range(2):
            Ps, Pd = route[a, :w.S], route[a, w.S:]
            sd = Ps[:, w.det_voxels]               # phi_s(x_d)
            ds = Pd[:, w.src_voxels].T             # phi_d(x_s)
            np.testing.assert_allclose(sd, ds, rtol=1e-11, atol=1e-10 * np.abs(sd).max())


def test_gmres_meets_tolerance():
    w = workloads.config("tiny")
    _, its, rel = fields.solve_gmres(w, lam_idx=[0], tol=1e-10)
    assert rel.max() <= 1e-10
    assert its.min() > 10


def _tiny_fields(lams=(0, 4)):
    w = workloads.config("tiny", nx=8, ny=8, nz=4, n_lambda=5)
    P = fields.solve_banded(w, lam_idx=list(lams))
    return w, P[:, :w.S], P[:, w.S:]


def test_born_is_derivative_of_direct_solves():
    """J[s,d,k] = d phi_s(x_d) / d mu_a(k): central differences of two sparse direct solves."""
    w, Ps, Pd = _tiny_fields((2,))
    J = born.born_matrix(Ps, Pd, w.h).reshape(1, w.S, w.D, w.N)
    A0 = model.operator(w, 2).tocsc()
    delta = 1e-4
    for k in (0, 37, 129, 200):
        E = sp.csc_matrix(([w.h ** 3], ([k], [k])), shape=(w.N, w.N))
        for s_i, sv in enumerate(w.src_voxels):
            b = model.rhs(w, sv)
            up = spla.spsolve(A0 + delta * E, b)
            dn = spla.spsolve(A0 - delta * E, b)
            fd = (up[w.det_voxels] - dn[w.det_voxels]) / (2 * delta)
            np.testing.assert_allclose(fd, J[0, s_i, :, k], rtol=1e-5)


def test_born_explicit_matrix_and_dot_test():
    w, Ps, Pd = _tiny_fields()
    v = workloads.born_v(w, n_v=2)
    wv = workloads.born_w(workloads.config("tiny", nx=8, ny=8, nz=4, n_lambda=2))
    J = born.born_matrix(Ps, Pd, w.h)
    y = born.born_apply(Ps, Pd, v, w.h)
    for c in range(2):
        np.testing.assert_allclose(y[c].reshape(-1), J @ v[c], rtol=1e-13, atol=1e-30)
    g = born.born_apply_adjoint(Ps, Pd, wv, w.h)
    np.testing.assert_allclose(g, J.conj().T @ wv.reshape(-1), rtol=1e-12, atol=1e-30)
    lhs = np.vdot(wv.reshape(-1), y[0].reshape(-1))
    rhs = np.vdot(g, v[0])
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(wv) * np.linalg.norm(y[0])


def test_born_linearisation_is_second_order():
    """phi(mu_a + t dmu) - phi(mu_a) - t J dmu = O(t^2) for a local absorption change."""
    w, Ps, Pd = _tiny_fields((1,))
    rng = np.random.default_rng(5)
    dmu = np.zeros(w.N)
    dmu[rng.choice(w.N, 20, replace=False)] = rng.uniform(0.0, 1.0, 20)
    y = born.born_apply(Ps, Pd, dmu, w.h)[0, 0]                 # [S, D] -> source 0
    A0 = model.operator(w, 1).tocsc()
    b = model.rhs(w, w.src_voxels[0])
    base = spla.spsolve(A0, b)[w.det_voxels]
    rem = []
    for t in (1e-3, 5e-4):
        pert = spla.spsolve(A0 + sp.diags(t * w.h ** 3 * dmu), b)[w.det_voxels]
        rem.append(np.abs(pert - base - t * y[0]).max())
    assert 3.5 < rem[0] / rem[1] < 4.5


def test_heaviside_and_delta():
    eps = 0.5
    x = np.linspace(-1, 1, 20001)
    H = pals.heaviside(x, eps)
    assert pals.heaviside(0.0, eps) == pytest.approx(0.5)
    assert pals.heaviside(-eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert pals.heaviside(eps, eps) == pytest.approx(1.0)
    assert np.all(np.diff(H) >= -1e-15)
    d = pals.delta(x, eps)
    assert np.trapezoid(d, x) == pytest.approx(1.0, rel=1e-6)
    fd = (pals.heaviside(x[1:-1] + 1e-6, eps) - pals.heaviside(x[1:-1] - 1e-6, eps)) / 2e-6
    np.testing.assert_allclose(fd, d[1:-1], atol=1e-5)


def _pals_case(basis):
    w = workloads.config("tiny", nx=12, ny=12, nz=8, n_lambda=3)
    p_true, dc_true = workloads.pals_truth(w, basis=basis)
    return w, p_true, dc_true


@pytest.mark.parametrize("basis", ["wendland", "gaussian"])
def test_shape_jacobian_matches_finite_differences(basis):
    # the two radial functions of the PaLS basis, pinned to their closed forms at a few points
    t = np.array([0.0, 0.25, 0.5, 0.99, 1.0, 1.5])
    if basis == "wendland":
        np.testing.assert_allclose(pals.psi(t), [1.0, 0.75 ** 4 * 2.0, 0.0625 * 3.0, 1e-8 * 4.96, 0.0, 0.0],
                                   rtol=1e-12, atol=1e-20)
    else:
        np.testing.assert_allclose(pals.psi(t, basis), np.exp(-t * t), rtol=1e-15)
    fdp = (pals.psi(t[1:4] + 1e-7, basis) - pals.psi(t[1:4] - 1e-7, basis)) / 2e-7
    np.testing.assert_allclose(pals.dpsi(t[1:4], basis), fdp, rtol=1e-6, atol=1e-12)
    w, p_true, _ = _pals_case(basis)
    p, _ = workloads.pals_perturbed(w, p_true, np.ones(2))
    tau, eps, nu = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU
    Jp = pals.shape_jacobian(w, p, tau, eps, nu, basis)
    assert np.abs(Jp).max() > 0
    for i in range(p.shape[0]):
        st = 1e-6 * max(1.0, abs(p[i]))
        pu, pd = p.copy(), p.copy()
        pu[i] += st
        pd[i] -= st
        fd = (pals.shape(w, pu, tau, eps, nu, basis) - pals.shape(w, pd, tau, eps, nu, basis)) / (2 * st)
        np.testing.assert_allclose(fd, Jp[:, i], atol=2e-6 * max(1.0, np.abs(Jp[:, i]).max()))


@pytest.mark.parametrize("basis", ["wendland", "gaussian"])
def test_misfit_gradient_matches_finite_differences_and_vanishes_at_truth(basis):
    w, p_true, dc_true = _pals_case(basis)
    P = fields.solve_separable(w)
    Ps, Pd = P[:, :w.S], P[:, w.S:]
    tau, eps, nu = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU
    _, _, _, y_obs = pals.misfit(w, Ps, Pd, p_true, dc_true, 0.0, tau, eps, nu, basis=basis)
    f0, gdc0, gp0, _ = pals.misfit(w, Ps, Pd, p_true, dc_true, y_obs, tau, eps, nu, basis=basis)
    assert f0 == 0.0
    assert np.abs(gp0).max() == 0.0 and np.abs(gdc0).max() == 0.0
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)
    f, gdc, gp, _ = pals.misfit(w, Ps, Pd, p, dc, y_obs, tau, eps, nu, basis=basis)
    assert f > 0
    x = np.concatenate([dc, p])
    g = np.concatenate([gdc, gp])
    fd = np.empty_like(x)
    for i in range(x.shape[0]):
        st = 1e-6 * max(1.0, abs(x[i]))
        xu, xd = x.copy(), x.copy()
        xu[i] += st
        xd[i] -= st
        fu = pals.misfit(w, Ps, Pd, xu[2:], xu[:2], y_obs, tau, eps, nu, basis=basis)[0]
        fdn = pals.misfit(w, Ps, Pd, xd[2:], xd[:2], y_obs, tau, eps, nu, basis=basis)[0]
        fd[i] = (fu - fdn) / (2 * st)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(g).max())


def test_spectra_are_seeded_and_in_range():
    w1 = workloads.config("large")
    w2 = workloads.config("large")
    np.testing.assert_array_equal(w1.extinction, w2.extinction)
    D, mua, _ = model.optics(w1)
    assert 0.003 < mua.min() and mua.max() < 0.05
    assert 0.4 < D.min() and D.max() < 0.8
    assert w1.src_voxels.shape == (64,) and w1.det_voxels.shape == (64,)
    assert np.all(w1.src_voxels // (w1.nx * w1.ny) == w1.nz - 1)


def test_operator_is_complex_symmetric_with_spd_real_part():
    w = workloads.config("tiny", nx=6, ny=5, nz=4)
    A = model.operator(w, 3)
    assert abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.real.toarray())
    assert ev.min() > 0


def test_uniform_perturbation_equals_raised_background():
    """shape = 1 with scale s_l is a homogeneous medium with mu_a + s_l: the perturbed operator's
    banded LU must match fast diagonalisation of a workload whose background absorption carries an
    extra chromophore with extinction s_l (two independent routes)."""
    w = workloads.config("tiny", n_lambda=3)
    s = np.array([0.004, 0.011, 0.02])
    got = fields.solve_banded(w, pert=(np.ones(w.N), s))
    w2 = workloads.config("tiny", n_lambda=3)
    w2.extinction = np.vstack([w2.extinction, s[None, :]])
    w2.conc_uM = np.concatenate([w2.conc_uM, [1.0]])
    ref = fields.solve_separable(w2)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    # and the perturbation really changes the fields
    base = fields.solve_banded(w)
    assert np.abs(got - base).max() > 1e-3 * np.abs(base).max()


def test_perturbed_fields_reciprocity_and_born_limit():
    """The heterogeneous operator stays complex symmetric (reciprocity between optodes), and
    phi(mu_a + t*s*shape) - phi(mu_a) - t * s_l * J shape = O(t^2) (the Born approximation is the
    first-order term of the full forward model)."""
    w = workloads.config("tiny", n_lambda=2)
    p, _ = workloads.pals_truth(w)
    shape = pals.shape(w, p, workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU)
    s = np.array([0.01, 0.02])
    P = fields.solve_banded(w, pert=(shape, s))
    S = w.S
    for a in range(S):
        for b in range(w.D):
            np.testing.assert_allclose(P[:, a, w.det_voxels[b]], P[:, S + b, w.src_voxels[a]], rtol=1e-9)
    base = fields.solve_banded(w)
    y = born.born_apply(base[:, :S], base[:, S:], shape[None], w.h)[0]      # [L, S, D]
    rem = []
    for t in (0.2, 0.1):
        Pt = fields.solve_banded(w, pert=(shape, t * s))
        diff = Pt[:, :S][:, :, w.det_voxels] - base[:, :S][:, :, w.det_voxels]
        rem.append(np.abs(diff - t * s[:, None, None] * y).max())
    assert 3.5 < rem[0] / rem[1] < 4.5


def test_precond_solve_is_the_scaled_solve_for_one_wavelength():
    """With a single wavelength the mean sigma' is that wavelength's, so (K_hat + sigma_0 I) is
    exactly A(lambda_0) / (D_0 h^3): its solve must equal D_0 h^3 phi from the banded LU of the
    unscaled operator (two independent routes)."""
    w = workloads.config("tiny", nx=9, ny=7, nz=5, n_lambda=1)
    sig, sigp = model.shifts(w)
    D, _, _ = model.optics(w)
    vox = [int(w.src_voxels[0]), 17, w.N - 1]
    y = fields.precond_solve(w, np.eye(w.N)[vox], float(sigp.mean()), complex(sig[0]))
    phi = fields.solve_banded(w, voxels=vox)[0]
    np.testing.assert_allclose(y, D[0] * w.h ** 3 * phi, rtol=1e-10, atol=1e-12 * np.abs(y).max())
    # with a different sigma'* the result changes only through the Robin faces
    y2 = fields.precond_solve(w, np.eye(w.N)[vox], float(sigp.mean()) * 1.5, complex(sig[0]))
    assert np.abs(y2 - y).max() > 1e-6 * np.abs(y).max()
