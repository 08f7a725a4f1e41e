"""Seeded synthetic workloads: fluid grids, cameras, frequency lists, batch job lists.

These stand in for the GRMHD snapshots (BHAC / HARM2D) that the paper renders; those
files are not available.  The fluid recipe is an axisymmetric torus-like flow on a
modified-Kerr-Schild (MKS) grid in CGS units:

* cells are uniform in x1 = ln r over [ln r_in, ln r_out] and in x2 over [0, 1];
  theta(x2) = pi x2 + (1 - h)/2 sin(2 pi x2) (the MKS polar map of the paper's
  appendix on KS-MKS coordinates), values are stored at cell centres;
* n_e = 1e6 (r/r_h)^-1.5 exp(-cos^2 theta / (2 * 0.3^2)) (1 + 0.1 U(-1,1))  [cm^-3];
* Theta_e = 10 r_h / r;
* B from plasma beta 10 with P_gas = 2 n_e m_e c^2 Theta_e (T_p = T_e), P_mag = B^2/8pi;
* Omega = 1 / (r^1.5 + a_gen) (Keplerian angular velocity, 1/M);
* r_h = 1 + sqrt(1 - a_gen^2).

Time series (slow light): snapshot s uses noise seed S0 + s and carries, at sample
time, an azimuthal modulation of n_e by 1 + A sum_{m=1..4} cos(m(phi - Omega_K(r) t_s)
+ psi_m) with psi_m ~ U(0, 2 pi) drawn with seed S0 + 64.  The modulation is analytic
in phi, so it is described by (A, psi_m) rather than stored.

Nothing here computes any step of the ray-tracing method.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .rng import uniform, uniform_stream

S0 = 1801104520

# CGS constants used only to build B from the plasma beta (CODATA 2018 values).
_ME = 9.1093837015e-28
_C = 2.99792458e10

NU_230 = 230e9
NU_VLBI = [22e9, 43e9, 86e9, 230e9]


@dataclass
class Grid:
    cells: np.ndarray            # [n_snap][n2][n1][4] float32 or float64
    r_in: float
    r_out: float
    hslope: float
    a_gen: float
    t0: float = 0.0
    dt_snap: float = 10.0
    mod_amp: float = 0.0
    mod_phase: List[float] = field(default_factory=lambda: [0.0, 0.0, 0.0, 0.0])
    # GRMHD code units (units = 1): fields {rho, u, b, Omega}; the mass unit and electron model
    units: int = 0
    mass_unit_g: float = 0.0
    r_low: float = 1.0
    r_high: float = 1.0
    gamma_ad: float = 13.0 / 9.0

    @property
    def n_snap(self):
        return self.cells.shape[0]

    @property
    def n2(self):
        return self.cells.shape[1]

    @property
    def n1(self):
        return self.cells.shape[2]

    @property
    def is_f64(self):
        return self.cells.dtype == np.float64


@dataclass
class Camera:
    spin: float
    incl_deg: float
    nx: int
    ny: int
    r_cam: float = 1e4
    fov_half: float = 20.0
    t_frame: float = 0.0


def cell_centres(n1, n2, r_in, r_out, hslope):
    x1 = np.log(r_in) + (np.arange(n1) + 0.5) * (np.log(r_out) - np.log(r_in)) / n1
    x2 = (np.arange(n2) + 0.5) / n2
    r = np.exp(x1)
    th = np.pi * x2 + 0.5 * (1.0 - hslope) * np.sin(2.0 * np.pi * x2)
    return r, th


def torus_snapshot(n1, n2, a_gen, seed, r_in=1.1, r_out=50.0, hslope=0.3, noise=0.1):
    """One snapshot [n2][n1][4] in float64 (see the module docstring for the recipe)."""
    r1, th1 = cell_centres(n1, n2, r_in, r_out, hslope)
    th, r = np.meshgrid(th1, r1, indexing="ij")          # theta-major: [n2][n1]
    rh = 1.0 + np.sqrt(1.0 - a_gen * a_gen)
    u = uniform_stream(seed, n1 * n2).reshape(n2, n1)
    ne = 1e6 * (r / rh) ** -1.5 * np.exp(-np.cos(th) ** 2 / (2 * 0.3 ** 2)) * (1.0 + noise * (2.0 * u - 1.0))
    thetae = 10.0 * rh / r
    beta_p = 10.0
    pgas = 2.0 * ne * _ME * _C * _C * thetae
    b = np.sqrt(8.0 * np.pi * pgas / beta_p)
    omega = 1.0 / (r ** 1.5 + a_gen)
    return np.stack([ne, thetae, b, omega], axis=-1)


def make_grid(n1=256, n2=256, a_gen=0.9375, dtype=np.float32, seed=S0, r_in=1.1, r_out=50.0,
              hslope=0.3, n_snap=1, t0=0.0, dt_snap=10.0, mod_amp=0.0, noise=0.1) -> Grid:
    snaps = [torus_snapshot(n1, n2, a_gen, seed + s, r_in, r_out, hslope, noise) for s in range(n_snap)]
    cells = np.ascontiguousarray(np.stack(snaps, axis=0).astype(dtype))
    phase = [0.0] * 4
    if mod_amp != 0.0:
        phase = list(2.0 * np.pi * uniform_stream(S0 + 64, 4))
    return Grid(cells=cells, r_in=r_in, r_out=r_out, hslope=hslope, a_gen=a_gen, t0=t0,
                dt_snap=dt_snap, mod_amp=mod_amp, mod_phase=phase)


def constant_grid(value, n1=8, n2=8, r_in=1.1, r_out=50.0, hslope=0.3, dtype=np.float64, a_gen=0.0, **units):
    """A grid whose four fields are the constants ``value`` ((n_e, Theta_e, B, Omega), or code-unit
    primitives (rho, u, b, Omega) with units=1 and the model keywords)."""
    cells = np.empty((1, n2, n1, 4), dtype=dtype)
    cells[...] = np.asarray(value, dtype=dtype)
    return Grid(cells=cells, r_in=r_in, r_out=r_out, hslope=hslope, a_gen=a_gen, **units)


def torus_snapshot_code(n1, n2, a_gen, seed, r_in=1.1, r_out=50.0, hslope=0.3, noise=0.1, gamma_ad=13.0 / 9.0):
    """One snapshot [n2][n1][4] of GRMHD primitives in code units, float64:
    rho = (r/r_h)^-1.5 exp(-cos^2 theta / (2 * 0.3^2)) (1 + noise U(-1,1)); u = 0.1 rho r_h / r;
    plasma beta 0.1 + 30 exp(-cos^2 theta / (2 * 0.3^2)) (magnetized funnel, weakly magnetized
    disk), b = sqrt(2 (gamma_ad - 1) u / beta); Omega = 1 / (r^1.5 + a_gen)."""
    r1, th1 = cell_centres(n1, n2, r_in, r_out, hslope)
    th, r = np.meshgrid(th1, r1, indexing="ij")
    rh = 1.0 + np.sqrt(1.0 - a_gen * a_gen)
    un = uniform_stream(seed, n1 * n2).reshape(n2, n1)
    disk = np.exp(-np.cos(th) ** 2 / (2 * 0.3 ** 2))
    rho = (r / rh) ** -1.5 * disk * (1.0 + noise * (2.0 * un - 1.0))
    u = 0.1 * rho * rh / r
    beta_p = 0.1 + 30.0 * disk
    b = np.sqrt(2.0 * (gamma_ad - 1.0) * u / beta_p)
    omega = 1.0 / (r ** 1.5 + a_gen)
    return np.stack([rho, u, b, omega], axis=-1)


def make_code_grid(n1=256, n2=256, a_gen=0.9375, dtype=np.float32, seed=S0 + 300, r_in=1.1, r_out=50.0,
                   hslope=0.3, n_snap=1, t0=0.0, dt_snap=10.0, noise=0.1, mass_unit_g=5e17, r_low=1.0,
                   r_high=10.0, gamma_ad=13.0 / 9.0) -> Grid:
    """A code-unit grid (units = 1) of the recipe in torus_snapshot_code; the mass unit 5e17 g
    gives electron densities near those of the CGS recipe for M = 4.5e6 solar masses."""
    snaps = [torus_snapshot_code(n1, n2, a_gen, seed + s, r_in, r_out, hslope, noise, gamma_ad) for s in range(n_snap)]
    cells = np.ascontiguousarray(np.stack(snaps, axis=0).astype(dtype))
    return Grid(cells=cells, r_in=r_in, r_out=r_out, hslope=hslope, a_gen=a_gen, t0=t0, dt_snap=dt_snap,
                units=1, mass_unit_g=mass_unit_g, r_low=r_low, r_high=r_high, gamma_ad=gamma_ad)


# --------------------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------------------

def small_image():
    """64x64 pixels, a = 0.9375, i = 60 deg, 128x128 float64 grid, 230 GHz."""
    cam = Camera(spin=0.9375, incl_deg=60.0, nx=64, ny=64)
    grid = make_grid(128, 128, a_gen=0.9375, dtype=np.float64)
    return cam, grid, [NU_230]


PROD_SPINS = [0.0, 0.5, 0.9375]
PROD_INCLS = [30.0, 60.0, 85.0]


def production_set(res=512, n_grid=256):
    """3 spins x 3 inclinations at res^2, float32 grids regenerated per spin, 230 GHz.

    Returns a list of (camera, grid) with one grid object shared by the cameras of a spin.
    """
    out = []
    for a in PROD_SPINS:
        g = make_grid(n_grid, n_grid, a_gen=a, dtype=np.float32)
        for inc in PROD_INCLS:
            out.append((Camera(spin=a, incl_deg=inc, nx=res, ny=res), g))
    return out


def spectrum_freqs(n=24, lo=1e9, hi=1e16):
    k = np.arange(n)
    return list(lo * (hi / lo) ** (k / (n - 1)))


def slow_light_set(res=256, n_grid=256, n_snap=64, dt_snap=10.0):
    """256^2, a=0.9375, i=60 deg, 24 frequencies, 64 modulated float32 snapshots.

    The frame time is the time of snapshot 32; the fast-light form samples that snapshot.
    """
    grid = make_grid(n_grid, n_grid, a_gen=0.9375, dtype=np.float32, n_snap=n_snap, t0=0.0,
                     dt_snap=dt_snap, mod_amp=0.2)
    t_frame = grid.t0 + 32 * dt_snap
    cam = Camera(spin=0.9375, incl_deg=60.0, nx=res, ny=res, t_frame=t_frame)
    return cam, grid, spectrum_freqs()


def batch_jobs(n_images=256, seed=S0 + 200, res_choices=(64, 128, 256, 512)):
    """Uneven batch: resolution uniform over res_choices, spin U(-0.99,0.99), incl U(5,85)."""
    u = uniform(seed, np.arange(3 * n_images, dtype=np.uint64)).reshape(n_images, 3)
    cams = []
    for k in range(n_images):
        res = res_choices[min(int(u[k, 0] * len(res_choices)), len(res_choices) - 1)]
        cams.append(Camera(spin=-0.99 + 1.98 * u[k, 1], incl_deg=5.0 + 80.0 * u[k, 2], nx=res, ny=res))
    return cams


def mlp_samples(n, seed=S0 + 100, nu_ratio=(1e-2, 1e8), thetae=(0.1, 100.0), cos_max=0.999):
    """Closure inputs (ln(nu/nu_c), ln Theta_e, cos theta_B), log-uniform / uniform over the
    learned closure's box."""
    u = uniform(seed, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)
    l1 = np.log(nu_ratio[0]) + u[:, 0] * (np.log(nu_ratio[1]) - np.log(nu_ratio[0]))
    l2 = np.log(thetae[0]) + u[:, 1] * (np.log(thetae[1]) - np.log(thetae[0]))
    c = -cos_max + 2.0 * cos_max * u[:, 2]
    return np.stack([l1, l2, c], axis=1)
