"""Pins of the oracle's Alg. opt (oracle/reconstruct.py).

* the LM Jacobian -W Ebar H dmu/dp matches central differences of the residual;
* with H a (complex multiple of the) identity, Alg. opt is a plain nonlinear least-squares fit of
  the PaLS shape to an image of it, which is well posed: from the perturbed start it must reach
  the truth (contrasts and parameters) to high accuracy, with a monotone misfit, with either
  damping form of the LM step;
* one LM step solves the normal equations of its damping form (the printed nu I, or
  Marquardt's nu diag(J^T J));
* at the truth the contrast least squares returns the true contrasts and the loop stops at once;
* with noise on the Born data of the tiny workload the loop stops at the first iterate whose
  misfit is within gamma ||eta|| (discrepancy principle).
"""
import numpy as np
import pytest

import workloads
from oracle import born, fields, pals
from oracle import reconstruct as orec

TAU, EPS, NU = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU


def _born_case(n_bumps):
    w = workloads.config("tiny", n_lambda=6)
    P = fields.solve_banded(w)
    S = w.S
    H = born.born_matrix(P[:, :S], P[:, S:], w.h).reshape(w.L, S, w.D, w.N)
    p_true, dc_true = workloads.pals_truth(w, n_bumps=n_bumps)
    mu_true = pals.shape(w, p_true, TAU, EPS, NU)
    y = (dc_true @ w.extinction)[:, None, None] * np.tensordot(H, mu_true, axes=([3], [0]))
    return w, H, p_true, dc_true, y


def test_lm_jacobian_matches_finite_differences():
    w, H, p_true, dc_true, y = _born_case(3)
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)
    Wt = np.random.default_rng(5).uniform(0.5, 2.0, size=y.shape)
    J = orec.lm_jacobian(H, w, p, dc, w.extinction, Wt, TAU, EPS, NU)

    def res(pp):
        _, Hm = orec.forward_parts(H, w, pp, TAU, EPS, NU)
        r = (Wt * (y - (dc @ w.extinction)[:, None, None] * Hm)).ravel()
        return np.concatenate([r.real, r.imag])

    for i in range(p.shape[0]):
        d = 1e-6 * max(1.0, abs(p[i]))
        pu, pd = p.copy(), p.copy()
        pu[i] += d
        pd[i] -= d
        fd = (res(pu) - res(pd)) / (2 * d)
        assert np.linalg.norm(fd - J[:, i]) <= 1e-5 * np.linalg.norm(J[:, i]) + 1e-14


@pytest.mark.parametrize("damping", ["identity", "marquardt"])
def test_identity_operator_fit_reaches_truth(damping):
    """Both damping forms of the LM step (the printed nu I and Marquardt's nu diag(J^T J)) solve
    this well-posed fit to the truth from the perturbed start."""
    w = workloads.config("tiny", nx=10, ny=10, nz=6, n_lambda=3)
    H = np.broadcast_to(np.eye(w.N)[None, None], (w.L, 1, w.N, w.N)) * (1.0 + 0.5j)
    p_true, dc_true = workloads.pals_truth(w, n_bumps=3)
    dc_true = np.array([6.0, 9.0])
    mu_true = pals.shape(w, p_true, TAU, EPS, NU)
    y = (dc_true @ w.extinction)[:, None, None] * np.tensordot(H, mu_true, axes=([3], [0]))
    p0, _ = workloads.pals_perturbed(w, p_true, dc_true)
    c, p, hist = orec.reconstruct(H, w, w.extinction, y, p0, max_outer=60, damping=damping)
    assert np.all(np.diff(hist) <= 0.0)
    assert hist[-1] <= 1e-8 * hist[0]
    np.testing.assert_allclose(c, dc_true, rtol=1e-8)
    np.testing.assert_allclose(p, p_true, rtol=0, atol=1e-6)


def test_damping_forms_take_the_printed_and_the_scaled_step():
    """One LM step from the same point: the default solves (J^T J + nu I) dp = -J^T e with
    nu = 1e-3 max diag(J^T J); the scaled form (J^T J + nu diag(J^T J)) dp = -J^T e with
    nu = 1e-3.  Checked against those normal equations through a single inner step."""
    w, H, p_true, dc_true, y = _born_case(1)
    p0, _ = workloads.pals_perturbed(w, p_true, dc_true)
    J = orec.lm_jacobian(H, w, p0, dc_true, w.extinction, 1.0, TAU, EPS, NU)
    _, Hmu = orec.forward_parts(H, w, p0, TAU, EPS, NU)
    r = (y - (dc_true @ w.extinction)[:, None, None] * Hmu).ravel()
    e = np.concatenate([r.real, r.imag])
    JTJ = J.T @ J
    for damping, M in (("identity", 1e-3 * JTJ.diagonal().max() * np.eye(len(p0))),
                       ("marquardt", 1e-3 * np.diag(JTJ.diagonal()))):
        _, p1, hist = orec.reconstruct(H, w, w.extinction, y, p0, c0=dc_true, fix_c=True, max_outer=1,
                                       max_inner=1, damping=damping)
        step = p1 - p0
        assert hist[1] < hist[0]      # the first try descends here, so the step is the undamped-retry one
        np.testing.assert_allclose((JTJ + M) @ step, -(J.T @ e), rtol=1e-8, atol=1e-10 * np.abs(J.T @ e).max())


def test_truth_is_a_fixed_point():
    w, H, p_true, dc_true, y = _born_case(3)
    _, Hmu = orec.forward_parts(H, w, p_true, TAU, EPS, NU)
    np.testing.assert_allclose(orec.lstsq_contrasts(w.extinction, Hmu, y, 1.0), dc_true, rtol=1e-10)
    c, p, hist = orec.reconstruct(H, w, w.extinction, y, p_true, noise_norm=1e-9 * np.linalg.norm(y))
    assert len(hist) == 1 and hist[0] <= 1e-12 * np.linalg.norm(y)
    np.testing.assert_array_equal(p, p_true)


@pytest.mark.parametrize("n_bumps", [1, 3])
def test_noisy_reconstruction_stops_at_discrepancy(n_bumps):
    w, H, p_true, dc_true, y = _born_case(n_bumps)
    eta = workloads.observed_noise(y.shape, 10 ** (-30 / 20) * np.linalg.norm(y) / np.sqrt(y.size))
    p0, _ = workloads.pals_perturbed(w, p_true, dc_true)
    gamma = 1.05
    target = gamma * np.linalg.norm(eta)
    c, p, hist = orec.reconstruct(H, w, w.extinction, y + eta, p0, noise_norm=np.linalg.norm(eta), gamma=gamma,
                                  max_outer=60)
    assert hist[-1] <= target
    assert np.all(np.asarray(hist[:-1]) > target)
    assert np.all(np.diff(hist) <= 0.0)
