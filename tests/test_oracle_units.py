"""Pins of the oracle's GRMHD code-unit conversion and electron model (Sec. 4.2.2 scaling,
Sec. 5 temperature-ratio model): the limits and midpoint of R(beta), the plasma beta recovered
from the converted CGS values (which ties B0 = c sqrt(4 pi rho0) to P_mag = b^2/2), the scaling
of n_e and B with the mass unit and the black-hole mass, the closed form of Theta_e at constant
R, and a uniform code-unit grid rendering like the uniform CGS grid of its converted values."""
import math

import numpy as np
import pytest

import synthetic as S

MP_OVER_ME = 1836.15267343          # CODATA 2018 proton-electron mass ratio
C = 2.99792458e10
ME = 9.1093837015e-28


def grid(orc, r_low=1.0, r_high=10.0, gamma_ad=13.0 / 9.0, mass_unit_g=5e17, value=(1.0, 0.01, 0.05, 0.03)):
    g = S.constant_grid(value, units=1, mass_unit_g=mass_unit_g, r_low=r_low, r_high=r_high, gamma_ad=gamma_ad)
    return g, orc.GridHandle(g)


def test_temperature_ratio_limits_and_midpoint(orc):
    g, h = grid(orc, r_low=2.0, r_high=40.0)
    gam1 = g.gamma_ad - 1.0
    rho, u = 0.7, 0.02
    fac = MP_OVER_ME * gam1 * u / rho

    def theta_of_R(R):
        return fac / (1.0 + R)
    # b = 0: beta infinite, R = R_high
    assert orc.code_to_cgs(h, [rho, u, 0.0, 0.0])[1] == pytest.approx(theta_of_R(40.0), rel=1e-9)
    # strongly magnetized: beta = 1e-6, R = R_low to 1e-12
    b = math.sqrt(2.0 * gam1 * u / 1e-6)
    assert orc.code_to_cgs(h, [rho, u, b, 0.0])[1] == pytest.approx(theta_of_R(2.0), rel=1e-9)
    # weakly magnetized: beta = 1e6
    b = math.sqrt(2.0 * gam1 * u / 1e6)
    assert orc.code_to_cgs(h, [rho, u, b, 0.0])[1] == pytest.approx(theta_of_R(40.0), rel=1e-9)
    # ratios to the b = 0 value cancel the mass ratio: (1 + R_high) / (1 + R(beta))
    t_inf = orc.code_to_cgs(h, [rho, u, 0.0, 0.0])[1]
    # beta = 1 (P_gas = P_mag): R is the mean of R_low and R_high
    b = math.sqrt(2.0 * gam1 * u)
    assert orc.code_to_cgs(h, [rho, u, b, 0.0])[1] / t_inf == pytest.approx(41.0 / 22.0, rel=1e-13)
    # beta = 2: R = (R_low + 4 R_high) / 5
    b = math.sqrt(2.0 * gam1 * u / 2.0)
    assert orc.code_to_cgs(h, [rho, u, b, 0.0])[1] / t_inf == pytest.approx(41.0 / (1.0 + 162.0 / 5.0), rel=1e-13)


def test_constant_ratio_closed_form_and_no_gas(orc):
    for gamma_ad in (4.0 / 3.0, 13.0 / 9.0, 5.0 / 3.0):
        g, h = grid(orc, r_low=3.0, r_high=3.0, gamma_ad=gamma_ad)
        for prim in ([1.0, 0.01, 0.05, 0.0], [0.2, 0.3, 2.0, 0.0], [5.0, 1e-4, 1e-3, 0.0]):
            the = orc.code_to_cgs(h, prim)[1]
            assert the == pytest.approx(MP_OVER_ME * (gamma_ad - 1.0) * prim[1] / prim[0] / 4.0, rel=1e-9)
    g, h = grid(orc)
    assert orc.code_to_cgs(h, [0.0, 0.01, 0.05, 0.0])[1] == 0.0
    assert orc.code_to_cgs(h, [1.0, 0.0, 0.05, 0.0])[1] == 0.0
    assert orc.code_to_cgs(h, [1.0, 0.0, 0.05, 0.5])[3] == 0.5   # Omega passes through


def test_plasma_beta_survives_the_conversion(orc):
    """P_gas = (gamma - 1) u rho0 c^2 and P_mag = B^2 / (8 pi) in CGS give the code-unit beta
    (gamma - 1) u / (b^2 / 2) back, for any mass unit and black-hole mass."""
    for mass_unit_g, msun in ((5e17, 4.5e6), (1e20, 6.2e9), (3e15, 10.0)):
        g, h = grid(orc, mass_unit_g=mass_unit_g)
        gam1 = g.gamma_ad - 1.0
        for rho, u, b in ((1.0, 0.01, 0.05), (0.3, 0.2, 1.5), (2.0, 1e-3, 1e-4)):
            ne, _, B, _ = orc.code_to_cgs(h, [rho, u, b, 0.0], mass_msun=msun)
            rho0 = ne * (ME * MP_OVER_ME + ME) / rho
            beta_cgs = gam1 * u * rho0 * C * C / (B * B / (8.0 * math.pi))
            assert beta_cgs == pytest.approx(gam1 * u / (0.5 * b * b), rel=1e-9)


def test_density_and_field_scaling(orc):
    """n_e is linear in rho and the mass unit and goes as M^-3; B goes as sqrt(mass unit) M^-3/2."""
    prim = [0.8, 0.01, 0.05, 0.0]
    _, h1 = grid(orc, mass_unit_g=1e18)
    _, h2 = grid(orc, mass_unit_g=4e18)
    a = orc.code_to_cgs(h1, prim, mass_msun=4.5e6)
    b = orc.code_to_cgs(h2, prim, mass_msun=4.5e6)
    c = orc.code_to_cgs(h1, prim, mass_msun=9.0e6)
    d = orc.code_to_cgs(h1, [1.6, 0.02, 0.05 * math.sqrt(2.0), 0.0], mass_msun=4.5e6)   # same beta
    assert b[0] / a[0] == pytest.approx(4.0, rel=1e-14) and b[2] / a[2] == pytest.approx(2.0, rel=1e-14)
    assert c[0] / a[0] == pytest.approx(1.0 / 8.0, rel=1e-14)
    assert c[2] / a[2] == pytest.approx(1.0 / math.sqrt(8.0), rel=1e-14)
    assert d[0] / a[0] == pytest.approx(2.0, rel=1e-14)
    assert d[1] == pytest.approx(a[1], rel=1e-14)             # Theta_e depends on u / rho and beta only
    assert b[1] == pytest.approx(a[1], rel=1e-14)             # and not on the units
    # Sgr A*-like numbers: GM/c^2 = 6.645e11 cm for 4.5e6 solar masses; rho0 = M / L^3
    L = 6.6446e11
    assert a[0] == pytest.approx(0.8 * 1e18 / L ** 3 / (ME * (MP_OVER_ME + 1.0)), rel=1e-3)


def test_uniform_code_grid_renders_like_its_cgs_values(orc):
    cam = S.Camera(spin=0.5, incl_deg=60.0, nx=6, ny=6, fov_half=12.0)
    opts = orc.make_opts(mass_msun=4.5e6)
    gc, hc = grid(orc, value=(1.0, 0.01, 0.05, 0.03))
    cgs = orc.code_to_cgs(hc, [1.0, 0.01, 0.05, 0.03], mass_msun=4.5e6)
    gp = S.constant_grid(tuple(cgs))
    nu = [86e9, 230e9]
    ic = orc.trace_image(cam, orc.GridHandle(gc), opts, nu)[0]
    ip = orc.trace_image(cam, orc.GridHandle(gp), opts, nu)[0]
    assert np.abs(ic).max() > 0
    np.testing.assert_allclose(ic, ip, rtol=1e-13, atol=0)
    # and a different black-hole mass changes the code-unit image but not the CGS one's inputs
    ic2 = orc.trace_image(cam, orc.GridHandle(gc), orc.make_opts(mass_msun=9e6), nu)[0]
    assert np.abs(ic2 - ic).max() > 1e-2 * np.abs(ic).max()
