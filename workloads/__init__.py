"""Seeded synthetic inputs for the hyperspectral DOT Born hot path.

This module is shared by the CPU oracle, the tests and the benchmark.  It
draws and lays out inputs only: grid sizes, wavelengths, scattering and
extinction spectra, optode voxel indices, Born probe vectors and PaLS
parameters.  It holds none of the method's arithmetic (no operator, no
solve, no Born product, no level-set evaluation).

Why synthetic: the paper's breast-phantom mesh, its tabulated chromophore
spectra and its measured data are not available, so seeded stand-ins with
the paper's parameter ranges (Table 1: N in 32^3..100^3, N_lambda in
10..200, N_s in 10..100) are generated here.

Conventions
-----------
* voxel index  n = i + nx*(j + ny*k), voxel centres at ((i+1/2)h, (j+1/2)h, (k+1/2)h);
* optodes sit in the top layer k = nz-1 on a Gx x Gy array: source (a, b)
  at (floor((a+1/4) nx/Gx), floor((b+1/4) ny/Gy)), detector at the 3/4 points;
  optode index s = a + Gx*b;
* extinction spectra (seed 1410):
  eps_l(lam) = ebar_l * exp(sum_{m=1..3} a_lm sin(m pi (lam-650)/350 + theta_lm)),
  a ~ U(-0.4, 0.4), theta ~ U(0, 2 pi), ebar = (2.0e-4, 2.5e-4) per mm per uM
  (HbO2, HbR), background concentrations (40, 20) uM;
* reduced scattering mus'(lam) = (lam/500)^-1.2 per mm;
* modulation 100 MHz, refractive index 1.4, Robin coefficient A_R = 2.5,
  voxel size h = 2 mm.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPEED_OF_LIGHT_MM_PER_S = 299792458.0e3
REFRACTIVE_INDEX = 1.4
MODULATION_HZ = 100.0e6
EBAR = (2.0e-4, 2.5e-4)            # HbO2, HbR  [1/(mm uM)]
BACKGROUND_CONC_UM = (40.0, 20.0)  # HbO2, HbR  [uM]
SPECTRA_SEED = 1410
ALL_ROBIN = 0x3F

# optode array shapes per optode count (Gx, Gy)
OPTODE_ARRAYS = {1: (1, 1), 2: (2, 1), 4: (2, 2), 8: (4, 2), 16: (4, 4),
                 24: (6, 4), 32: (8, 4), 64: (8, 8)}


@dataclass
class Workload:
    """One synthetic hyperspectral DOT workload (all host numpy arrays)."""
    name: str
    nx: int
    ny: int
    nz: int
    h: float                      # voxel edge [mm]
    A_R: float                    # Robin coefficient
    robin_faces: int              # bit f set: Robin on face f (-x,+x,-y,+y,-z,+z), else Dirichlet
    lambdas_nm: np.ndarray        # [L]
    mus_prime: np.ndarray         # [L] reduced scattering [1/mm]
    extinction: np.ndarray        # [n_species, L]  [1/(mm uM)]
    conc_uM: np.ndarray           # [n_species] background concentrations
    omega_over_nu: float          # [1/mm]
    src_voxels: np.ndarray        # [S] int64
    det_voxels: np.ndarray        # [D] int64
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def L(self) -> int:
        return int(self.lambdas_nm.shape[0])

    @property
    def S(self) -> int:
        return int(self.src_voxels.shape[0])

    @property
    def D(self) -> int:
        return int(self.det_voxels.shape[0])

    @property
    def rhs_voxels(self) -> np.ndarray:
        """Sources then detectors: the right-hand sides of one field solve."""
        return np.concatenate([self.src_voxels, self.det_voxels]).astype(np.int64)


def omega_over_nu() -> float:
    """Modulation angular frequency over the speed of light in tissue [1/mm]."""
    nu = SPEED_OF_LIGHT_MM_PER_S / REFRACTIVE_INDEX
    return 2.0 * math.pi * MODULATION_HZ / nu


def extinction_spectra(lambdas_nm: np.ndarray, seed: int = SPECTRA_SEED) -> np.ndarray:
    """Smooth seeded synthetic extinction spectra, shape [2, L]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.4, 0.4, size=(2, 3))
    theta = rng.uniform(0.0, 2.0 * math.pi, size=(2, 3))
    lam = np.asarray(lambdas_nm, dtype=np.float64)
    out = np.empty((2, lam.shape[0]))
    for l in range(2):
        expo = np.zeros_like(lam)
        for m in range(3):
            expo += a[l, m] * np.sin((m + 1) * math.pi * (lam - 650.0) / 350.0 + theta[l, m])
        out[l] = EBAR[l] * np.exp(expo)
    return out


def optode_voxels(nx: int, ny: int, nz: int, count: int, frac: float) -> np.ndarray:
    """Voxel indices of a Gx x Gy optode array in the top layer (frac 1/4: sources, 3/4: detectors)."""
    gx, gy = OPTODE_ARRAYS[count]
    k = nz - 1
    out = []
    for b in range(gy):
        for a in range(gx):
            i = int(math.floor((a + frac) * nx / gx))
            j = int(math.floor((b + frac) * ny / gy))
            out.append(i + nx * (j + ny * k))
    return np.asarray(out, dtype=np.int64)


def make_workload(name: str, nx: int, ny: int, nz: int, n_src: int, n_det: int,
                  n_lambda: int, lam_min: float, lam_max: float, h: float = 2.0,
                  A_R: float = 2.5, robin_faces: int = ALL_ROBIN) -> Workload:
    lambdas = np.linspace(lam_min, lam_max, n_lambda) if n_lambda > 1 else np.array([lam_min])
    return Workload(
        name=name, nx=nx, ny=ny, nz=nz, h=float(h), A_R=float(A_R), robin_faces=int(robin_faces),
        lambdas_nm=lambdas,
        mus_prime=(lambdas / 500.0) ** -1.2,
        extinction=extinction_spectra(lambdas),
        conc_uM=np.asarray(BACKGROUND_CONC_UM, dtype=np.float64),
        omega_over_nu=omega_over_nu(),
        src_voxels=optode_voxels(nx, ny, nz, n_src, 0.25),
        det_voxels=optode_voxels(nx, ny, nz, n_det, 0.75),
    )


# Named workloads.  The sizes follow the hot-path scope of the paper's Table 1
# ranges; each is described by what it is.
CONFIGS = {
    # 16x16x8 grid, 4+4 optodes, 8 wavelengths 650-860 nm
    "tiny": dict(nx=16, ny=16, nz=8, n_src=4, n_det=4, n_lambda=8, lam_min=650.0, lam_max=860.0),
    # 64x64x32 grid, 16+16 optodes, 32 wavelengths 650-900 nm
    "medium": dict(nx=64, ny=64, nz=32, n_src=16, n_det=16, n_lambda=32, lam_min=650.0, lam_max=900.0),
    # 64x64x32 grid, 32+32 optodes, 64 wavelengths 650-900 nm
    "batch": dict(nx=64, ny=64, nz=32, n_src=32, n_det=32, n_lambda=64, lam_min=650.0, lam_max=900.0),
    # 96x96x48 grid, 24+24 optodes, 48 wavelengths 650-900 nm
    "diff": dict(nx=96, ny=96, nz=48, n_src=24, n_det=24, n_lambda=48, lam_min=650.0, lam_max=900.0),
    # 128x128x64 grid, 64+64 optodes, 128 wavelengths 650-1000 nm
    "large": dict(nx=128, ny=128, nz=64, n_src=64, n_det=64, n_lambda=128, lam_min=650.0, lam_max=1000.0),
    # the three smaller grids that accompany the large one
    "large_g32": dict(nx=32, ny=32, nz=16, n_src=16, n_det=16, n_lambda=128, lam_min=650.0, lam_max=1000.0),
    "large_g48": dict(nx=48, ny=48, nz=24, n_src=24, n_det=24, n_lambda=128, lam_min=650.0, lam_max=1000.0),
    "large_g80": dict(nx=80, ny=80, nz=40, n_src=32, n_det=32, n_lambda=128, lam_min=650.0, lam_max=1000.0),
}


def config(name: str, **overrides) -> Workload:
    """Named workload; keyword overrides replace any size field (for shrunk test copies)."""
    spec = dict(CONFIGS[name])
    spec.update(overrides)
    return make_workload(name, **spec)


def subset_lambdas(w: Workload, idx) -> Workload:
    """Copy of a workload keeping only the wavelengths at positions idx."""
    idx = np.asarray(idx, dtype=np.int64)
    return Workload(name=w.name, nx=w.nx, ny=w.ny, nz=w.nz, h=w.h, A_R=w.A_R,
                    robin_faces=w.robin_faces, lambdas_nm=w.lambdas_nm[idx].copy(),
                    mus_prime=w.mus_prime[idx].copy(), extinction=w.extinction[:, idx].copy(),
                    conc_uM=w.conc_uM.copy(), omega_over_nu=w.omega_over_nu,
                    src_voxels=w.src_voxels.copy(), det_voxels=w.det_voxels.copy(),
                    extra=dict(w.extra))


# ---------------------------------------------------------------- Born probes
def born_v(w: Workload, n_v: int = 1, seed: int = 986, dtype=np.float64) -> np.ndarray:
    """Real absorption perturbation(s) v ~ N(0,1) i.i.d. per voxel, shape [n_v, N]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_v, w.N)).astype(dtype)


def born_w(w: Workload, seed: int = 987) -> np.ndarray:
    """Complex data-space vector, Re and Im ~ N(0, 1/2), shape [L, S, D]."""
    rng = np.random.default_rng(seed)
    re = rng.normal(0.0, math.sqrt(0.5), size=(w.L, w.S, w.D))
    im = rng.normal(0.0, math.sqrt(0.5), size=(w.L, w.S, w.D))
    return re + 1j * im


# ------------------------------------------------------------------ PaLS inputs
PALS_BUMPS = 8
PALS_TAU = 0.5          # level of the level set
PALS_EPS = 0.5          # half-width of the smoothed Heaviside
PALS_NU = 1.0e-3        # smoothing of the distance [mm]
TRUTH_DCONC_UM = (8.0, 8.0)


def pals_truth(w: Workload, n_bumps: int = PALS_BUMPS, seed: int = 2014, basis: str = "wendland"):
    """Seeded 'true' PaLS parameters and contrasts.

    Returns (p, dconc) with p = [alpha(n), beta(n), cx(n), cy(n), cz(n)]:
    centres U[1/3, 2/3] of the extent per axis, weights +-1 (Rademacher), and
    beta = 1/radius with support radii U[8, 20] mm for the compactly supported basis
    ("wendland") or beta = 1/width with widths U[3, 8] mm for the Gaussian basis
    ("gaussian"; the 0.5-level shapes of the two are of similar size); dconc = (+8, +8) uM.
    """
    rng = np.random.default_rng(seed)
    ext = np.array([w.nx * w.h, w.ny * w.h, w.nz * w.h])
    centres = rng.uniform(1.0 / 3.0, 2.0 / 3.0, size=(n_bumps, 3)) * ext
    lo, hi = (3.0, 8.0) if basis == "gaussian" else (8.0, 20.0)
    widths = rng.uniform(lo, hi, size=n_bumps)
    alpha = rng.choice([-1.0, 1.0], size=n_bumps)
    p = np.concatenate([alpha, 1.0 / widths, centres[:, 0], centres[:, 1], centres[:, 2]])
    return p, np.asarray(TRUTH_DCONC_UM, dtype=np.float64)


def pals_perturbed(w: Workload, p_true: np.ndarray, dconc_true: np.ndarray, seed: int = 2015):
    """Evaluation point away from the truth: centres +-2 mm, radii x(1+-0.1), alpha x0.9, dconc x0.8."""
    n = p_true.shape[0] // 5
    rng = np.random.default_rng(seed)
    alpha = p_true[:n] * 0.9
    widths = (1.0 / p_true[n:2 * n]) * rng.uniform(0.9, 1.1, size=n)
    cx = p_true[2 * n:3 * n] + rng.uniform(-2.0, 2.0, size=n)
    cy = p_true[3 * n:4 * n] + rng.uniform(-2.0, 2.0, size=n)
    cz = p_true[4 * n:5 * n] + rng.uniform(-2.0, 2.0, size=n)
    p = np.concatenate([alpha, 1.0 / widths, cx, cy, cz])
    return p, np.asarray(dconc_true, dtype=np.float64) * 0.8


def pals_random_start(w: Workload, n_bumps: int, seed: int = 2016) -> np.ndarray:
    """Randomly initialised PaLS parameters: centres U[1/3, 2/3] of the extent, support radii
    U[8, 20] mm, weights +1."""
    rng = np.random.default_rng(seed)
    ext = np.array([w.nx * w.h, w.ny * w.h, w.nz * w.h])
    centres = rng.uniform(1.0 / 3.0, 2.0 / 3.0, size=(n_bumps, 3)) * ext
    radii = rng.uniform(8.0, 20.0, size=n_bumps)
    return np.concatenate([np.ones(n_bumps), 1.0 / radii, centres[:, 0], centres[:, 1], centres[:, 2]])


def observed_noise(shape, scale: float, seed: int = 33) -> np.ndarray:
    """Complex Gaussian noise with per-component standard deviation scale/sqrt(2)."""
    rng = np.random.default_rng(seed)
    s = scale / math.sqrt(2.0)
    return rng.normal(0.0, s, size=shape) + 1j * rng.normal(0.0, s, size=shape)


# ---------------------------------------------------------------- randomized compression
COMPRESS_SEED = 4242


def gaussian_test_matrix(n: int, cols: int, seed: int = COMPRESS_SEED) -> np.ndarray:
    """The i.i.d. N(0,1) test matrix of the randomized range finder, [n, cols]; a run that needs
    fewer columns uses the leading ones, so both implementations see the same draws."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, cols))


def optode_xy(w: Workload, voxels) -> np.ndarray:
    """(x, y) voxel-centre coordinates in mm of optode voxels on the top plate, [count, 2]."""
    v = np.asarray(voxels, dtype=np.int64)
    i = v % w.nx
    j = (v // w.nx) % w.ny
    return np.stack([(i + 0.5) * w.h, (j + 0.5) * w.h], axis=1)
