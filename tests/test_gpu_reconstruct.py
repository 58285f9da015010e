"""Alg. opt on the GPU (Born products, shape and shape Jacobian through the library) against the
oracle's dense implementation on the same fields, data and start: the LM Jacobian, the contrast
least squares and the whole iteration (misfit history, contrasts, parameters); and the Exp. 1
analogue: the compressed operator gives the reconstruction of the full one."""
import numpy as np
import pytest
import torch

import workloads
from oracle import born as oborn
from oracle import fields as ofields
from oracle import pals as opals
from oracle import reconstruct as orec

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
TAU, EPS, NU = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU


@pytest.fixture(scope="module")
def hd():
    import paper_1410_0986_amd as hd
    return hd


@pytest.fixture(scope="module")
def case(hd):
    w = workloads.config("tiny", n_lambda=6)
    P = ofields.solve_banded(w)
    S = w.S
    H = oborn.born_matrix(P[:, :S], P[:, S:], w.h).reshape(w.L, S, w.D, w.N)
    op = hd.Operator.from_workload(w)
    t = torch.from_numpy(P).to(DEV)
    return w, P, H, op, t


def _data(w, H, n_bumps, snr_db):
    p_true, dc_true = workloads.pals_truth(w, n_bumps=n_bumps)
    mu_true = opals.shape(w, p_true, TAU, EPS, NU)
    y = (dc_true @ w.extinction)[:, None, None] * np.tensordot(H, mu_true, axes=([3], [0]))
    eta = np.zeros_like(y) if snr_db is None else \
        workloads.observed_noise(y.shape, 10 ** (-snr_db / 20) * np.linalg.norm(y) / np.sqrt(y.size))
    return p_true, dc_true, mu_true, y + eta, float(np.linalg.norm(eta))


def _model(hd, w, op, t, weights=None, compressed=None):
    from paper_1410_0986_amd import reconstruct as rec
    return rec.BornModel(op, t[:, :w.S], t[:, w.S:], w.extinction, weights=weights, compressed=compressed)


def test_lm_jacobian_and_contrasts_match_oracle(hd, case):
    from paper_1410_0986_amd import reconstruct as rec
    w, P, H, op, t = case
    p_true, dc_true, _, y, _ = _data(w, H, 3, None)
    p, dc = workloads.pals_perturbed(w, p_true, dc_true)
    Wt = np.random.default_rng(5).uniform(0.5, 2.0, size=y.shape)
    m = _model(hd, w, op, t, weights=Wt)
    J = rec.lm_jacobian(m, p, dc)
    Jo = orec.lm_jacobian(H, w, p, dc, w.extinction, Wt, TAU, EPS, NU)
    assert J.shape == Jo.shape
    assert np.linalg.norm(J - Jo) <= 1e-10 * np.linalg.norm(Jo)
    Hmu = m.Hmu(p)
    _, Hmu_o = orec.forward_parts(H, w, p, TAU, EPS, NU)
    assert np.linalg.norm(Hmu - Hmu_o) <= 1e-12 * np.linalg.norm(Hmu_o)
    np.testing.assert_allclose(rec.contrast_ls(m, Hmu, y), orec.lstsq_contrasts(w.extinction, Hmu_o, y, Wt),
                               rtol=1e-9)


@pytest.mark.parametrize("damping", ["identity", "marquardt"])
@pytest.mark.parametrize("n_bumps,snr_db,fix_c", [(3, 30.0, False), (1, 30.0, False), (3, 33.0, True)])
def test_reconstruction_matches_oracle(hd, case, n_bumps, snr_db, fix_c, damping):
    from paper_1410_0986_amd import reconstruct as rec
    w, P, H, op, t = case
    p_true, dc_true, mu_true, y, nn = _data(w, H, n_bumps, snr_db)
    p0, _ = workloads.pals_perturbed(w, p_true, dc_true)
    c0 = dc_true if fix_c else None
    r = rec.reconstruct(_model(hd, w, op, t), y, p0, c0=c0, noise_norm=nn, max_outer=60, fix_c=fix_c,
                        damping=damping)
    c_o, p_o, hist_o = orec.reconstruct(H, w, w.extinction, y, p0, c0=c0, noise_norm=nn, max_outer=60,
                                        fix_c=fix_c, damping=damping)
    assert r.stopped_by == "discrepancy"
    assert len(r.misfit_history) == len(hist_o)
    np.testing.assert_allclose(r.misfit_history, hist_o, rtol=1e-8)
    np.testing.assert_allclose(r.c, c_o, rtol=1e-8)
    np.testing.assert_allclose(r.p, p_o, rtol=1e-7, atol=1e-9)
    if fix_c:
        np.testing.assert_array_equal(r.c, dc_true)


def test_shape_errors(hd):
    from paper_1410_0986_amd import reconstruct as rec
    a = np.zeros(100)
    a[:40] = 1.0
    b = np.zeros(100)
    b[20:50] = 1.0
    l2, dice = rec.shape_errors(a, b)
    assert dice == pytest.approx(2 * 20 / 70)
    assert l2 == pytest.approx(np.sqrt(30) / np.sqrt(40))
    assert rec.shape_errors(a, a) == (0.0, 1.0)


def test_compressed_operator_reconstruction(hd, case):
    """Exp. 1 analogue: shape-only reconstruction (known contrasts, 33 dB) with the compressed H at
    a tight tolerance reproduces the full-H reconstruction, and a loose tolerance keeps the shape
    error close to it."""
    from paper_1410_0986_amd import compress, reconstruct as rec
    w, P, H, op, t = case
    p_true, dc_true, mu_true, y, nn = _data(w, H, 3, 33.0)
    p0, _ = workloads.pals_perturbed(w, p_true, dc_true)
    full = rec.reconstruct(_model(hd, w, op, t), y, p0, c0=dc_true, noise_norm=nn, fix_c=True, max_outer=60)
    xy = workloads.optode_xy(w, w.src_voxels)
    om1 = workloads.gaussian_test_matrix(w.N, 80)
    om2 = workloads.gaussian_test_matrix(w.N, 10, seed=workloads.COMPRESS_SEED + 1)
    mu_full = opals.shape(w, full.p, TAU, EPS, NU)
    e_full = rec.shape_errors(mu_true, mu_full)
    for eps, close in ((1e-9, 1e-4), (1e-3, 0.05)):
        cb = compress.compress(op, t[:, :w.S], t[:, w.S:], xy, eps, om1, om2)
        r = rec.reconstruct(_model(hd, w, op, t, compressed=cb), y, p0, c0=dc_true, noise_norm=nn, fix_c=True,
                            max_outer=60)
        assert r.stopped_by == "discrepancy"
        mu = opals.shape(w, r.p, TAU, EPS, NU)
        e = rec.shape_errors(mu_true, mu)
        assert abs(e[0] - e_full[0]) <= close and abs(e[1] - e_full[1]) <= max(close, 0.02)
        if eps < 1e-6:
            assert np.linalg.norm(mu - mu_full) <= 1e-4 * np.linalg.norm(mu_full)
