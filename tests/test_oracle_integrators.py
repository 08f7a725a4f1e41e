"""Pins of the oracle's second-order integrators (Sec. 2.2): the midpoint rule (RK2) and
velocity Verlet without and with the corrector pass.

* Global error of order 2: the drift of the constants of motion (E, L_z, Carter Q) at the end
  of the printed convergence orbit and the deviation of flat-space rays from their straight
  line both fall as eps^2 (RK4 falls as eps^4 in the same tests).
* The corrector pass of Verlet lowers the error at a given eps (the paper's remark).
* All integrators converge to the same ray.
"""
import math

import numpy as np
import pytest

from test_oracle_spacetime import _paper_orbits, constants_of_motion


def end_drift(orc, integ, eps):
    import synthetic as S
    a, inc, al, be = _paper_orbits()[0]
    cam = S.Camera(spin=a, incl_deg=inc, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, al, be)
    c0 = np.array(constants_of_motion(orc, a, y0)[:3])
    traj, _, info = orc.integrate(a, 1.0, y0, eps=eps, r_stop=1.01 * (1 + math.sqrt(1 - a * a)), r_escape=1e4,
                                  cap=400000, integrator=integ)
    assert info.status in (1, 2)
    c = np.array(constants_of_motion(orc, a, traj[-1])[:3])
    return np.abs(c - c0).sum(), traj, info


@pytest.mark.parametrize("integ", ["RK2", "VERLET", "VERLET_CORR"])
def test_second_order_convergence_of_constants(orc, integ):
    code = getattr(orc, integ)
    epss = [0.02, 0.01, 0.005]
    errs = [end_drift(orc, code, e)[0] for e in epss]
    slopes = np.diff(np.log(errs)) / np.diff(np.log(epss))
    assert np.all(slopes > 1.6) and np.all(slopes < 2.6), (errs, slopes)


def test_corrector_lowers_the_error(orc):
    for eps in (0.02, 0.01):
        e_v = end_drift(orc, orc.VERLET, eps)[0]
        e_c = end_drift(orc, orc.VERLET_CORR, eps)[0]
        assert e_c < e_v, (eps, e_v, e_c)


@pytest.mark.parametrize("integ", ["RK2", "VERLET", "VERLET_CORR"])
def test_flat_space_lines_second_order(orc, integ):
    """M = 0 (flat space in spherical KS coordinates, where the connection does not vanish):
    the deviation from the straight line through the camera falls as eps^2."""
    import synthetic as S
    code = getattr(orc, integ)
    al, be, inc = 3.0, 4.0, 60.0
    cam = S.Camera(spin=0.0, incl_deg=inc, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, al, be, M=0.0)
    r0, t0 = y0[1], y0[2]
    P0 = np.array([r0 * math.sin(t0), 0.0, r0 * math.cos(t0)])
    kr, kt, kp = y0[5], y0[6], y0[7]
    d = np.array([kr * math.sin(t0) + r0 * kt * math.cos(t0), r0 * math.sin(t0) * kp,
                  kr * math.cos(t0) - r0 * kt * math.sin(t0)])
    d /= np.linalg.norm(d)
    errs = []
    for eps in (0.02, 0.01, 0.005):
        traj, _, info = orc.integrate(0.0, 0.0, y0, eps=eps, r_stop=0.0, r_escape=1e4, cap=200000, integrator=code)
        assert info.status == 2
        r, th, ph = traj[:, 1], traj[:, 2], traj[:, 3]
        P = np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], 1)
        rel = P - P0
        perp = rel - np.outer(rel @ d, d)
        errs.append(np.linalg.norm(perp, axis=1).max())
    slopes = np.diff(np.log(errs)) / math.log(0.5)
    assert np.all(slopes > 1.6) and np.all(slopes < 2.6), (errs, slopes)


def test_integrators_converge_to_the_same_ray(orc):
    """Closest approach of the convergence orbit: RK2 and Verlet at small eps agree with RK4 to
    within their O(eps^2) error."""
    r_min = {}
    for name in ("RK4", "RK2", "VERLET", "VERLET_CORR"):
        _, traj, _ = end_drift(orc, getattr(orc, name), 0.004 if name != "RK4" else 0.02)
        r_min[name] = traj[:, 1].min()
    for name in ("RK2", "VERLET", "VERLET_CORR"):
        assert r_min[name] == pytest.approx(r_min["RK4"], rel=2e-3), r_min


def test_verlet_step_reuses_the_derivative(orc):
    """One Verlet step returns the derivative at the new point evaluated with the predicted
    wave vector (without corrector) or with the corrected one (with corrector); feeding it back
    costs one connection evaluation per step."""
    import synthetic as S
    cam = S.Camera(spin=0.9, incl_deg=50.0, nx=2, ny=2)
    y, _ = orc.camera_ray(cam, 2.0, -3.0)
    y = np.array(y)
    f0 = orc.geodesic_rhs(0.9, 1.0, y)
    dl = -5.0
    yn, acc = orc.verlet_step(0.9, 1.0, y, f0[4:], dl, corrector=False)
    # predicted wave vector, and the derivative there
    kp = y[4:] + f0[4:] * dl
    xp = y[:4] + y[4:] * dl + 0.5 * f0[4:] * dl * dl
    fp = orc.geodesic_rhs(0.9, 1.0, np.concatenate([xp, kp]))
    assert np.allclose(yn[:4], xp, rtol=1e-15, atol=0)
    assert np.allclose(acc, fp[4:], rtol=1e-13, atol=0)
    assert np.allclose(yn[4:], y[4:] + 0.5 * (f0[4:] + fp[4:]) * dl, rtol=1e-13, atol=0)


def test_verlet_last_step_before_horizon_adds_nothing_undefined(orc):
    """Velocity Verlet's last step before the horizon can leave a wave vector whose fluid-frame
    frequency is negative (a = 0, i = 30 deg, a ray aimed at the hole at 512^2).  That sample
    has no defined emission: it is counted and adds nothing, so the intensity stays the finite
    sum of the earlier samples."""
    import math
    import synthetic as S
    c, g = S.production_set()[0]
    assert c.spin == 0.0 and c.incl_deg == 30.0
    opts = orc.make_opts(integrator=orc.VERLET)
    al, be = orc.pixel_alpha_beta(c, 254, 235)
    I, info, rec = orc.trace_ray(c, orc.GridHandle(g), opts, al, be, [230e9], record=4000)
    steps = [rec[i] for i in range(info.steps)]
    assert info.status == orc.HORIZON
    assert math.isfinite(I[0]) and I[0] > 0.0
    # the recorded samples all have positive fluid-frame frequencies; one step was sampled-but-skipped
    nus = [r.nu_r for r in steps if r.sampled]
    assert all(v > 0.0 for v in nus) and info.samples == len(nus) + 1
