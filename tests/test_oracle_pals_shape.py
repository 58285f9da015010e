"""Pins of the oracle's PaLS shape (Sec. 5, eq. pals) that do not go through its own formulas.

A single bump alpha psi(beta ||r - chi||_dag) centred on a voxel centre is a ball of the
lattice: its level set varphi = tau is the sphere of radius R with beta sqrt(R^2 + nu^2) = t_tau,
where t_tau is the root of psi(t) = tau, found here by bisection on the basis function as the
paper's readings define it (Wendland's (1 - t)^4 (4t + 1), or exp(-t^2) with the closed form
t_tau = sqrt(ln 2) at tau = 1/2).  So, whatever the smoothed Heaviside:
* the voxel at the centre sees varphi = psi(beta nu), about 1, and mu = 1;
* every voxel at distance exactly R sees varphi = tau and mu = 1/2 (H(0) = 1/2), and all six
  axis neighbours at the same distance agree (a half-voxel offset of the voxel centres breaks
  this, and a wrong beta * distance scaling moves the level set off R);
* outside the Wendland support (beta ||.|| >= 1) mu = 0;
* the voxels with mu > 1/2 are exactly the lattice points strictly inside the sphere, counted
  here by brute force over integer offsets, and their number is close to the volume 4/3 pi R^3 / h^3;
* two bumps with opposite weights at one centre cancel (varphi = 0, mu = 0), and a weight of 2
  moves the level set to psi(t) = tau / 2.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import pals

TAU, EPS, NU = workloads.PALS_TAU, workloads.PALS_EPS, workloads.PALS_NU


def _psi_def(t, basis):
    """The basis functions as the readings state them, written out for the root search."""
    if basis == "gaussian":
        return math.exp(-t * t)
    return (1.0 - t) ** 4 * (4.0 * t + 1.0) if t < 1.0 else 0.0


def _root(level, basis):
    """t with psi(t) = level on (0, 1) (Wendland) or (0, 10) (Gaussian), by bisection; both are
    strictly decreasing there."""
    lo, hi = 0.0, (1.0 if basis == "wendland" else 10.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _psi_def(mid, basis) > level:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _grid():
    return workloads.config("tiny", nx=32, ny=30, nz=28)


def _centre_voxel(w):
    i0, j0, k0 = 15, 14, 13
    return (i0, j0, k0), np.array([(i0 + 0.5) * w.h, (j0 + 0.5) * w.h, (k0 + 0.5) * w.h])


def _idx(w, i, j, k):
    return i + w.nx * (j + w.ny * k)


def _params(alpha, beta, centre):
    """p = [alpha, beta, chi_x, chi_y, chi_z] for one bump (Sec. 5 ordering)."""
    return np.array([alpha, beta, centre[0], centre[1], centre[2]], dtype=np.float64)


@pytest.mark.parametrize("basis", ["wendland", "gaussian"])
def test_level_set_radius_and_centre(basis):
    w = _grid()
    (i0, j0, k0), c = _centre_voxel(w)
    t_tau = _root(TAU, basis)
    if basis == "gaussian":
        assert t_tau == pytest.approx(math.sqrt(math.log(2.0)), rel=1e-14)
    n_r = 5                                              # the level set passes through 5 voxels out
    R = n_r * w.h
    beta = t_tau / math.sqrt(R * R + NU * NU)
    mu = pals.shape(w, _params(1.0, beta, c), TAU, EPS, NU, basis)
    assert mu[_idx(w, i0, j0, k0)] == pytest.approx(1.0, abs=1e-12)
    for di, dj, dk in ((n_r, 0, 0), (-n_r, 0, 0), (0, n_r, 0), (0, -n_r, 0), (0, 0, n_r), (0, 0, -n_r),
                       (3, 4, 0), (0, -3, 4), (4, 0, -3)):          # |offset| = 5 voxels in every case
        assert mu[_idx(w, i0 + di, j0 + dj, k0 + dk)] == pytest.approx(0.5, abs=1e-12)
    # one voxel inside and outside the sphere along each axis
    for a in range(3):
        off = [0, 0, 0]
        off[a] = n_r - 1
        assert mu[_idx(w, i0 + off[0], j0 + off[1], k0 + off[2])] > 0.5
        off[a] = n_r + 1
        assert mu[_idx(w, i0 + off[0], j0 + off[1], k0 + off[2])] < 0.5


@pytest.mark.parametrize("basis", ["wendland", "gaussian"])
def test_ball_is_the_lattice_ball(basis):
    w = _grid()
    (i0, j0, k0), c = _centre_voxel(w)
    t_tau = _root(TAU, basis)
    R = 9.37 * w.h                                       # no lattice point on the sphere
    beta = t_tau / math.sqrt(R * R + NU * NU)
    mu = pals.shape(w, _params(1.0, beta, c), TAU, EPS, NU, basis)
    inside = np.zeros(w.N, dtype=bool)
    count = 0
    rr = int(math.ceil(R / w.h))
    for dk in range(-rr, rr + 1):
        for dj in range(-rr, rr + 1):
            for di in range(-rr, rr + 1):
                if (di * di + dj * dj + dk * dk) * w.h * w.h < R * R:
                    inside[_idx(w, i0 + di, j0 + dj, k0 + dk)] = True
                    count += 1
    np.testing.assert_array_equal(mu > 0.5, inside)
    vol = 4.0 / 3.0 * math.pi * (R / w.h) ** 3
    assert abs(count - vol) <= 0.02 * vol


def test_wendland_support_and_weights():
    w = _grid()
    (i0, j0, k0), c = _centre_voxel(w)
    R1 = 6.0 * w.h                                       # support radius: beta ||r - chi||_dag = 1
    beta = 1.0 / math.sqrt(R1 * R1 + NU * NU)
    mu = pals.shape(w, _params(1.0, beta, c), TAU, EPS, NU, "wendland")
    k = np.arange(w.N)
    i, j, kk = k % w.nx, (k // w.nx) % w.ny, k // (w.nx * w.ny)
    d2 = ((i - i0) ** 2 + (j - j0) ** 2 + (kk - k0) ** 2) * w.h * w.h
    # varphi = 0 there, so mu = H(-tau) = H(-eps) = 0, up to the rounding of sin(pi)
    assert np.all(np.abs(mu[d2 >= R1 * R1]) <= 1e-16)
    # opposite weights at one centre cancel everywhere
    p2 = np.array([1.0, -1.0, beta, beta, c[0], c[0], c[1], c[1], c[2], c[2]])
    assert np.all(np.abs(pals.shape(w, p2, TAU, EPS, NU, "wendland")) <= 1e-16)
    # weight 2: the level set moves to psi(t) = tau / 2
    t_half = _root(TAU / 2.0, "wendland")
    R = 4 * w.h
    beta2 = t_half / math.sqrt(R * R + NU * NU)
    mu2 = pals.shape(w, _params(2.0, beta2, c), TAU, EPS, NU, "wendland")
    assert mu2[_idx(w, i0 + 4, j0, k0)] == pytest.approx(0.5, abs=1e-12)
    assert mu2[_idx(w, i0, j0 - 4, k0)] == pytest.approx(0.5, abs=1e-12)
