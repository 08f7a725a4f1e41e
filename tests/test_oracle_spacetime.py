"""Pins of the oracle's spacetime, connection and geodesic integrator.

Each check compares the oracle with something other than itself: textbook inverse metrics
and determinants, the paper's BL->KS vector matrix (appendix), finite differences,
Schwarzschild connection values, the constants of motion of Sec. 4.1, the photon sphere
and critical impact parameter sqrt(27) M, the Schwarzschild turning-point cubic, the Kerr
critical curve (Bardeen) and straight lines in flat space.
"""
import math

import numpy as np
import pytest

RNG = np.random.default_rng(7)
POINTS = [(a, r, th) for a in (0.0, 0.5, 0.9375, -0.7)
          for r, th in zip(RNG.uniform(1.6, 80.0, 4), RNG.uniform(0.15, math.pi - 0.15, 4))]


def ks_inverse_textbook(a, M, r, th):
    s2, c2 = math.sin(th) ** 2, math.cos(th) ** 2
    sig = r * r + a * a * c2
    z = 2 * M * r / sig
    dl = r * r - 2 * M * r + a * a
    gi = np.zeros((4, 4))
    gi[0, 0] = -(1 + z)
    gi[0, 1] = gi[1, 0] = z
    gi[1, 1] = dl / sig
    gi[1, 3] = gi[3, 1] = a / sig
    gi[2, 2] = 1 / sig
    gi[3, 3] = 1 / (sig * s2)
    return gi


def bl_inverse_textbook(a, M, r, th):
    s2, c2 = math.sin(th) ** 2, math.cos(th) ** 2
    sig = r * r + a * a * c2
    dl = r * r - 2 * M * r + a * a
    A = (r * r + a * a) ** 2 - a * a * dl * s2
    gi = np.zeros((4, 4))
    gi[0, 0] = -A / (sig * dl)
    gi[0, 3] = gi[3, 0] = -2 * M * a * r / (sig * dl)
    gi[1, 1] = dl / sig
    gi[2, 2] = 1 / sig
    gi[3, 3] = (dl - a * a * s2) / (sig * dl * s2)
    return gi


@pytest.mark.parametrize("a,r,th", POINTS)
def test_ks_metric_against_textbook_inverse_and_determinant(orc, a, r, th):
    g = orc.ks_metric(a, 1.0, r, th)
    assert np.allclose(g @ ks_inverse_textbook(a, 1.0, r, th), np.eye(4), atol=1e-12)
    sig = r * r + a * a * math.cos(th) ** 2
    assert np.linalg.det(g) == pytest.approx(-(sig ** 2) * math.sin(th) ** 2, rel=1e-11)


@pytest.mark.parametrize("a,r,th", POINTS)
def test_bl_metric_against_textbook_and_paper_ks_map(orc, a, r, th):
    """g_BL = T^T g_KS T with the paper's contravariant BL->KS matrix T (appendix BL-KS)."""
    gbl = orc.bl_metric(a, 1.0, r, th)
    assert np.allclose(gbl @ bl_inverse_textbook(a, 1.0, r, th), np.eye(4), atol=1e-11)
    dl = r * r - 2 * r + a * a
    T = np.eye(4)
    T[0, 1] = 2 * r / dl
    T[3, 1] = a / dl
    gks = orc.ks_metric(a, 1.0, r, th)
    assert np.allclose(T.T @ gks @ T, gbl, rtol=1e-11, atol=1e-11 * np.abs(gbl).max())


def test_schwarzschild_limit_is_textbook(orc):
    r, th = 7.3, 1.1
    g = orc.bl_metric(0.0, 1.0, r, th)
    assert np.allclose(np.diag(g), [-(1 - 2 / r), 1 / (1 - 2 / r), r * r, r * r * math.sin(th) ** 2])
    gk = orc.ks_metric(0.0, 1.0, r, th)
    assert gk[0, 1] == pytest.approx(2 / r) and gk[1, 1] == pytest.approx(1 + 2 / r)
    flat = orc.ks_metric(0.0, 0.0, r, th)
    assert np.allclose(flat, np.diag([-1, 1, r * r, r * r * math.sin(th) ** 2]))


@pytest.mark.parametrize("a,r,th", POINTS[::3])
def test_metric_derivatives_match_finite_differences(orc, a, r, th):
    g, dg = orc.ks_metric_derivs(a, 1.0, r, th)
    h = 1e-6
    fd_r = (orc.ks_metric(a, 1.0, r + h, th) - orc.ks_metric(a, 1.0, r - h, th)) / (2 * h)
    fd_t = (orc.ks_metric(a, 1.0, r, th + h) - orc.ks_metric(a, 1.0, r, th - h)) / (2 * h)
    scale = np.abs(dg).max()
    assert np.allclose(dg[1], fd_r, atol=1e-7 * scale)
    assert np.allclose(dg[2], fd_t, atol=1e-7 * scale)
    assert not dg[0].any() and not dg[3].any()


def test_christoffel_schwarzschild_ks_values(orc):
    r, th = 5.5, 0.9
    gam = orc.christoffel(0.0, 1.0, [0, r, th, 0])
    assert np.allclose(gam, np.transpose(gam, (0, 2, 1)), atol=1e-14)
    assert gam[1, 2, 2] == pytest.approx(-(r - 2))          # Gamma^r_thth
    assert gam[0, 2, 2] == pytest.approx(-2.0)              # Gamma^t_thth (ingoing KS)
    assert gam[2, 1, 2] == pytest.approx(1 / r)             # Gamma^th_r th
    assert gam[3, 2, 3] == pytest.approx(1 / math.tan(th))  # Gamma^ph_th ph
    assert gam[2, 3, 3] == pytest.approx(-math.sin(th) * math.cos(th))
    assert gam[0, 0, 0] == pytest.approx(2 / r ** 3)        # Gamma^t_tt = 2M^2/r^3


def constants_of_motion(orc, a, y):
    """E = -k_t, L = k_phi, Carter Q (Sec. 4.1, mu = 0) and the null norm, in KS."""
    g = orc.ks_metric(a, 1.0, y[1], y[2])
    kc = g @ y[4:]
    th = y[2]
    E, L = -kc[0], kc[3]
    Q = kc[2] ** 2 + math.cos(th) ** 2 * (a * a * (0 - kc[0] ** 2) + kc[3] ** 2 / math.sin(th) ** 2)
    norm = y[4:] @ g @ y[4:]
    return E, L, Q, norm


def test_camera_ray_constants_and_null(orc):
    import synthetic as S
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=64, ny=64)
    for al, be in [(3.1, -4.2), (-7.5, 0.3), (0.4, 9.9)]:
        y, kc = orc.camera_ray(cam, al, be)
        assert kc[2] == pytest.approx(be, rel=1e-14)        # k_theta = beta at theta = i
        E, L, Q, norm = constants_of_motion(orc, cam.spin, y)
        inc = math.radians(60.0)
        assert E == pytest.approx(1.0, rel=1e-12)
        assert L == pytest.approx(-al * math.sin(inc), rel=1e-12)
        assert Q == pytest.approx(be ** 2 + math.cos(inc) ** 2 * (al ** 2 - cam.spin ** 2), rel=1e-10)
        assert abs(norm) / y[4] ** 2 < 1e-13
        assert y[5] > 0  # outgoing photon at the camera


def _paper_orbits():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_test_orbits.json")) as f:
        d = json.load(f)
    c = d["convergence_orbit"]
    out = [(c["a"], c["incl_deg"], c["alpha"], c["beta"])]
    out += [(o["a"], o["incl_deg"], o["alpha"], o["beta"]) for o in d["difficult_orbits"]]
    return out


@pytest.mark.parametrize("orbit", _paper_orbits() + [(0.9375, 60.0, 2.5, -3.0)])
def test_constants_of_motion_conserved(orc, orbit):
    """E, L, Q and the null norm stay constant along RK4 rays (Sec. 4.1); includes the
    printed convergence orbit and the two 'difficult' orbits of the geodesic table."""
    import synthetic as S
    a, inc, al, be = orbit
    cam = S.Camera(spin=a, incl_deg=inc, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, al, be)
    c0 = constants_of_motion(orc, a, y0)
    rh = 1 + math.sqrt(1 - a * a)
    traj, _, info = orc.integrate(a, 1.0, y0, eps=0.01, max_steps=150000, r_stop=1.01 * rh,
                                    r_escape=1e4, cap=200000)
    assert info.status in (1, 2)
    worst = np.zeros(4)
    for y in traj[:: max(1, len(traj) // 400)]:
        c = constants_of_motion(orc, a, y)
        worst = np.maximum(worst, [abs(c[0] - c0[0]), abs(c[1] - c0[1]) / max(1, abs(c0[1])),
                                   abs(c[2] - c0[2]) / max(1, abs(c0[2])), abs(c[3]) / y[4] ** 2])
    assert worst.max() < 1e-6, worst


def test_rk4_convergence_order_four(orc):
    """Drift of Q, L, E at the end of the printed convergence orbit falls as eps^4 (Sec. 4.1)."""
    import synthetic as S
    a = 0.998
    a, inc, al, be = _paper_orbits()[0]
    cam = S.Camera(spin=a, incl_deg=inc, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, al, be)
    c0 = np.array(constants_of_motion(orc, a, y0)[:3])
    errs = []
    epss = [0.1, 0.05, 0.025]
    for eps in epss:
        traj, _, info = orc.integrate(a, 1.0, y0, eps=eps, r_stop=1.01 * (1 + math.sqrt(1 - a * a)),
                                      r_escape=1e4, cap=400000)
        c = np.array(constants_of_motion(orc, a, traj[-1])[:3])
        errs.append(np.abs(c - c0).sum())
    slopes = np.diff(np.log(errs)) / np.diff(np.log(epss))
    assert np.all(slopes > 3.5) and np.all(slopes < 4.7), (errs, slopes)


def shoot(orc, a, inc, al, be, eps):
    import synthetic as S
    cam = S.Camera(spin=a, incl_deg=inc, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, al, be)
    rh = 1 + math.sqrt(1 - a * a)
    traj, dls, info = orc.integrate(a, 1.0, y0, eps=eps, r_stop=1.01 * rh, r_escape=1e4, cap=100000)
    return traj, dls, info


def test_photon_sphere_critical_impact_parameter(orc):
    """a = 0, equatorial observer: the capture threshold in alpha is sqrt(27) M and the
    near-critical ray skims r = 3M."""
    lo, hi = 4.0, 6.5
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        _, _, info = shoot(orc, 0.0, 90.0, mid, 0.0, 0.02)
        if info.status == 1:
            lo = mid
        else:
            hi = mid
    assert abs(lo - math.sqrt(27)) < 2e-6, lo
    traj, _, _ = shoot(orc, 0.0, 90.0, hi * (1 + 1e-9), 0.0, 0.02)
    assert abs(traj[:, 1].min() - 3.0) < 2e-3


def test_schwarzschild_turning_point(orc):
    """r_min of an escaping ray is the largest root of r^3 - b^2 r + 2 b^2 = 0 (M = 1)."""
    for b in (6.0, 8.0, 12.0):
        traj, dls, info = shoot(orc, 0.0, 90.0, b, 0.0, 0.05)
        assert info.status == 2
        r, kr = traj[:, 1], traj[:, 5]
        i = int(np.argmin(r))
        # cubic Hermite through the two samples bracketing the sign change of dr/dlambda
        best = r[i]
        for i0 in (i - 1, i):
            h = dls[i0 + 1]
            p0, p1, m0, m1 = r[i0], r[i0 + 1], kr[i0] * h, kr[i0 + 1] * h
            s = np.linspace(0, 1, 20001)
            h00, h10, h01, h11 = 2 * s**3 - 3 * s**2 + 1, s**3 - 2 * s**2 + s, -2 * s**3 + 3 * s**2, s**3 - s**2
            best = min(best, (h00 * p0 + h10 * m0 + h01 * p1 + h11 * m1).min())
        exact = 2 * b / math.sqrt(3) * math.cos(math.acos(-3 * math.sqrt(3) / b) / 3)
        assert abs(best - exact) / exact < 2e-5, (b, best, exact)


def test_kerr_critical_curve(orc):
    """Rays just inside the Bardeen critical curve are captured, just outside escape."""
    a, inc = 0.9375, 60.0
    si, ci = math.sin(math.radians(inc)), math.cos(math.radians(inc))
    checked = 0
    for rph in np.linspace(1.3, 3.9, 14):
        xi = -(rph**3 - 3 * rph**2 + a * a * rph + a * a) / (a * (rph - 1))
        eta = -(rph**3) * (rph**3 - 6 * rph**2 + 9 * rph - 4 * a * a) / (a * a * (rph - 1) ** 2)
        b2 = eta + a * a * ci**2 - xi**2 * (ci / si) ** 2
        if b2 <= 0:
            continue
        al = -xi / si
        for be in (math.sqrt(b2), -math.sqrt(b2)):
            _, _, inn = shoot(orc, a, inc, al * 0.99, be * 0.99, 0.02)
            _, _, out = shoot(orc, a, inc, al * 1.01, be * 1.01, 0.02)
            assert inn.status == 1 and out.status == 2, (rph, al, be)
            checked += 1
    assert checked >= 8


def test_flat_space_straight_lines(orc):
    """M = 0: the ray is a straight line with closest approach sqrt(alpha^2 + beta^2); the
    deviation of the RK4 path from that line falls as eps^4."""
    import synthetic as S
    for al, be, inc in [(3.0, 4.0, 60.0), (-7.0, 2.0, 30.0), (0.5, -9.0, 85.0)]:
        cam = S.Camera(spin=0.0, incl_deg=inc, nx=2, ny=2)
        y0, _ = orc.camera_ray(cam, al, be, M=0.0)
        errs = []
        for eps in (0.05, 0.025, 0.0125):
            traj, _, info = orc.integrate(0.0, 0.0, y0, eps=eps, r_stop=0.0, r_escape=1e4, cap=100000)
            assert info.status == 2
            r, th, ph = traj[:, 1], traj[:, 2], traj[:, 3]
            P = np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], 1)
            # the exact line: through the camera point along the initial Cartesian direction
            r0, t0 = y0[1], y0[2]
            P0 = np.array([r0 * math.sin(t0), 0.0, r0 * math.cos(t0)])
            kr, kt, kp = y0[5], y0[6], y0[7]
            d = np.array([kr * math.sin(t0) + r0 * kt * math.cos(t0), r0 * math.sin(t0) * kp,
                          kr * math.cos(t0) - r0 * kt * math.sin(t0)])
            d /= np.linalg.norm(d)
            closest = np.linalg.norm(P0 - (P0 @ d) * d)
            assert closest == pytest.approx(math.hypot(al, be), rel=1e-9)
            rel = P - P0
            perp = rel - np.outer(rel @ d, d)
            errs.append(np.linalg.norm(perp, axis=1).max())
        slopes = np.diff(np.log(errs)) / math.log(0.5)
        assert errs[-1] < 1e-5 and np.all(slopes > 3.5), (errs, slopes)
