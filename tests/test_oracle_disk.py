"""Pins of the oracle's thin-disk test (Sec. 4.2.1): Keplerian disk from the ISCO to 15 M,
emission proportional to r^-2, no absorption, first equatorial crossing only.

* ISCO: the closed form equals the radius where the specific energy of circular orbits is
  smallest (found by numerical minimisation of the textbook E(r)).
* Redshift: for every ray that lands on the disk, g = E_obs/E_em equals
  1 / (u^t (1 - Omega L)) with u^t of the circular orbit at the crossing radius (closed form)
  and L = -alpha sin(i) the ray's conserved angular momentum -- an exact relation, since
  k_t = -1 and k_phi = L along the ray.
* Crossing point: in flat space the crossing radius of a straight ray converges with eps to the
  exact intersection of the line with the plane.
* Line profile: bins hold the pixel fluxes; nothing outside the redshift range the closed form
  allows.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import synthetic as S

SPINS = [-0.99, -0.5, 0.0, 0.5, 0.99]


def circular_E(r, a):
    """Specific energy of a prograde (a > 0) or retrograde (a < 0) circular equatorial orbit."""
    return (r ** 1.5 - 2 * r ** 0.5 + a) / (r ** 0.75 * math.sqrt(r ** 1.5 - 3 * r ** 0.5 + 2 * a))


def circular_ut(r, a):
    return (r ** 1.5 + a) / (r ** 0.75 * math.sqrt(r ** 1.5 - 3 * r ** 0.5 + 2 * a))


@pytest.mark.parametrize("a", SPINS + [0.9375])
def test_isco_is_the_energy_minimum(orc, a):
    r_isco = orc.isco(a)
    lo = 1.0 + 1.0e-3 if a > 0.9 else 1.5
    res = minimize_scalar(lambda r: circular_E(r, a), bounds=(max(lo, r_isco * 0.6), 12.0), method="bounded",
                          options={"xatol": 1e-10})
    assert res.x == pytest.approx(r_isco, rel=2e-5)
    assert orc.isco(0.0) == pytest.approx(6.0, rel=1e-15)


@pytest.mark.parametrize("a", SPINS)
def test_redshift_of_disk_rays_is_exact(orc, a):
    cam = S.Camera(spin=a, incl_deg=60.0, nx=48, ny=48, fov_half=16.0)
    opts = orc.make_opts(eps=0.02)
    sin_i = math.sin(math.radians(60.0))
    n_disk = 0
    for p in range(0, cam.nx * cam.ny, 7):
        al, be = orc.pixel_alpha_beta(cam, p % cam.nx, p // cam.nx)
        g, rc, I, info = orc.trace_disk_ray(cam, opts, 15.0, al, be)
        if info.status != orc.DISK:
            assert I == 0.0
            continue
        n_disk += 1
        assert orc.isco(a) <= rc <= 15.0
        L = -al * sin_i
        omega = 1.0 / (rc ** 1.5 + a)
        g_exact = 1.0 / (circular_ut(rc, a) * (1.0 - omega * L))
        assert g == pytest.approx(g_exact, rel=1e-6)   # RK4 drift of k_t, k_phi at eps = 0.02
        assert I == pytest.approx(g ** 3 / rc ** 2, rel=1e-14)
    assert n_disk > 40


def test_flat_space_crossing_radius_converges(orc):
    cam = S.Camera(spin=0.0, incl_deg=50.0, nx=2, ny=2)
    errs = []
    for eps in (0.02, 0.01, 0.005):
        opts = orc.make_opts(eps=eps, metric_mass=0.0)
        worst = 0.0
        for al, be in [(8.0, 3.0), (-6.0, 9.0), (10.0, -2.0)]:
            g, rc, I, info = orc.trace_disk_ray(cam, opts, 15.0, al, be)
            assert info.status in (orc.DISK, orc.PLANE)
            # the straight ray: camera point and initial Cartesian direction
            y0, _ = orc.camera_ray(cam, al, be, M=0.0)
            r0, t0 = y0[1], y0[2]
            P0 = np.array([r0 * math.sin(t0), 0.0, r0 * math.cos(t0)])
            kr, kt, kp = y0[5], y0[6], y0[7]
            d = np.array([kr * math.sin(t0) + r0 * kt * math.cos(t0), r0 * math.sin(t0) * kp,
                          kr * math.cos(t0) - r0 * kt * math.sin(t0)])
            s = -P0[2] / d[2]
            exact = np.linalg.norm(P0 + s * d)
            worst = max(worst, abs(rc / exact - 1))
        errs.append(worst)
    slopes = np.diff(np.log(errs)) / math.log(0.5)
    assert errs[-1] < 1e-4 and np.all(slopes > 1.6), (errs, slopes)


def test_line_profile_bins_and_support(orc):
    a = 0.5
    cam = S.Camera(spin=a, incl_deg=30.0, nx=64, ny=64, fov_half=16.0)
    g, I, st = orc.trace_disk_image(cam, orc.make_opts())
    hit = st[:, 0] == orc.DISK
    assert hit.sum() > 500
    assert np.all(I.ravel()[~hit] == 0.0)
    prof = orc.disk_profile(cam, g, I, 100, 0.0, 2.0)
    dA = (2 * cam.fov_half / cam.nx) * (2 * cam.fov_half / cam.ny)
    assert prof.sum() == pytest.approx(I.sum() * dA, rel=1e-13)
    # the redshift range allowed by the disk: extremes of 1/(u^t (1 - Omega L)) over r in
    # [r_isco, 15] and |L| up to the largest |alpha| sin i of the image
    rs = np.linspace(orc.isco(a), 15.0, 2000)
    Lmax = cam.fov_half * math.sin(math.radians(30.0))
    gs = [1.0 / (circular_ut(r, a) * (1.0 - (1.0 / (r ** 1.5 + a)) * L)) for r in rs for L in (-Lmax, Lmax)]
    nz = np.nonzero(prof)[0]
    centres_lo, centres_hi = nz[0] * 0.02, (nz[-1] + 1) * 0.02
    assert centres_lo >= min(gs) - 0.02 and centres_hi <= max(gs) + 0.02
