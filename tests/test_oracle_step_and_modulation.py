"""Pins of the oracle's step-size rule and of the slow-light density modulation.

Step size (Sec. 2.2, adaptive step-size equations) in the logarithmic KS chart x1 = ln r,
x2 = theta/pi, x3 = phi:

* a state moving along one chart coordinate only advances it, in one step, by exactly eps of
  that coordinate's scale: Delta ln r = eps, Delta theta = eps min(theta, pi - theta),
  Delta phi = eps;
* the three limiters combine as a sum of inverse steps, and the rule is homogeneous of
  degree -1 in k and symmetric under theta -> pi - theta;
* on integrated rays far from the hole the step is Delta r = 0.05 r (the radius-scaled step
  of the production configuration), and near the axis |Delta theta| is bounded by
  eps min(theta, pi - theta) and reaches that bound.

Density modulation of the slow-light time series (Sec. 5 stand-in): at snapshot time t_s,
n_e carries 1 + A sum_{m=1..4} cos(m (phi - Omega_K(r) t_s) + psi_m) with the prograde
Keplerian angular velocity Omega_K = 1/(r^3/2 + a) (Bardeen, Press & Teukolsky 1972):

* the pattern co-rotates at Omega_K: the value at (phi + Omega_K (t_s' - t_s), t_s') equals the
  value at (phi, t_s);
* its mean over azimuth is 1 and |mod - 1| <= 4A;
* its azimuthal Fourier content is exactly modes m = 1..4, each of amplitude A and phase
  psi_m - m Omega_K t_s.
"""
import math

import numpy as np
import pytest

import synthetic as S

EPS = 0.05


def _step(orc, x, k, eps=EPS):
    return orc.step_size(eps, np.asarray(x, float), np.asarray(k, float))


@pytest.mark.parametrize("r", [1.5, 7.0, 300.0, 1e4])
@pytest.mark.parametrize("kr", [-2.0, 0.3, 1.0])
def test_radial_motion_advances_ln_r_by_eps(orc, r, kr):
    dl = _step(orc, [0.0, r, 1.1, 0.0], [1.0, kr, 0.0, 0.0])
    assert abs(kr) * dl / r == pytest.approx(EPS, rel=1e-14)


@pytest.mark.parametrize("th", [0.02, 0.3, 1.0, math.pi / 2, 2.2, math.pi - 0.01])
@pytest.mark.parametrize("kth", [-0.7, 1e-3, 0.05])
def test_polar_motion_advances_theta_by_eps_of_axis_distance(orc, th, kth):
    dl = _step(orc, [0.0, 10.0, th, 0.0], [1.0, 0.0, kth, 0.0])
    assert abs(kth) * dl == pytest.approx(EPS * min(th, math.pi - th), rel=1e-13)


@pytest.mark.parametrize("kph", [-3.0, 0.01, 0.4])
def test_azimuthal_motion_advances_phi_by_eps(orc, kph):
    dl = _step(orc, [0.0, 10.0, 0.8, 0.0], [1.0, 0.0, 0.0, kph])
    assert abs(kph) * dl == pytest.approx(EPS, rel=1e-14)


def test_limiters_add_as_inverse_steps_and_scale(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        r = math.exp(rng.uniform(0.1, 9.0))
        th = rng.uniform(0.01, math.pi - 0.01)
        k = rng.normal(size=4)
        x = [0.0, r, th, 0.0]
        inv = 1.0 / _step(orc, x, k)
        parts = [1.0 / _step(orc, x, [1.0, k[1], 0.0, 0.0]), 1.0 / _step(orc, x, [1.0, 0.0, k[2], 0.0]),
                 1.0 / _step(orc, x, [1.0, 0.0, 0.0, k[3]])]
        assert inv == pytest.approx(sum(parts), rel=1e-13)
        # homogeneous of degree -1 in k, linear in eps, symmetric about the equator
        assert _step(orc, x, 3.0 * k) == pytest.approx(_step(orc, x, k) / 3.0, rel=1e-14)
        assert _step(orc, x, k, eps=0.02) == pytest.approx(_step(orc, x, k) * 0.4, rel=1e-14)
        assert _step(orc, [0.0, r, math.pi - th, 0.0], k) == pytest.approx(_step(orc, x, k), rel=1e-13)


def test_far_steps_are_five_percent_of_r(orc):
    """Config-1 camera at r = 1e4 M: the first steps inward have |Delta r| / r = 0.05 to the order of
    the neglected polar and azimuthal limiters (~ (b/r)^2 for impact parameter b)."""
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=2, ny=2)
    for al, be in [(-15.0, 4.0), (3.0, -18.0), (0.5, 0.5)]:
        y0, _ = orc.camera_ray(cam, al, be)
        traj, dls, info = orc.integrate(0.9375, 1.0, y0, eps=EPS, r_stop=1.01 * (1 + math.sqrt(1 - 0.9375 ** 2)),
                                        r_escape=2e4, cap=60)
        r = np.concatenate([[y0[1]], traj[:40, 1]])
        ratio = np.abs(np.diff(r)) / r[:-1]
        # RK4 over one step of an inward radial ray with dr/dlambda ~ -1: |Delta r| = eps r (1 + O(b^2/r^2))
        assert np.all(np.abs(ratio[:10] - EPS) < 2e-3), ratio[:10]


def test_steps_near_the_axis_shrink_with_axis_distance(orc):
    """A ray passing within a few degrees of the spin axis: every step moves theta by at most
    eps min(theta, pi - theta) (to O(eps) from the RK4 update), and near the axis the bound is
    reached (the polar limiter sets the step)."""
    a = 0.5
    cam = S.Camera(spin=a, incl_deg=4.0, nx=2, ny=2)
    y0, _ = orc.camera_ray(cam, 0.3, 2.0)
    rh = 1 + math.sqrt(1 - a * a)
    traj, dls, info = orc.integrate(a, 1.0, y0, eps=EPS, r_stop=1.01 * rh, r_escape=2e4, cap=20000)
    th = np.concatenate([[y0[2]], traj[: info.steps, 2]])
    ph = np.concatenate([[y0[3]], traj[: info.steps, 3]])
    edge = np.minimum(th[:-1], math.pi - th[:-1])
    dth = np.abs(np.diff(th))
    ok = np.abs(np.diff(ph)) < 1.0          # skip steps through a pole reflection
    ratio = dth[ok] / (EPS * edge[ok])
    assert ratio.max() < 1.0 + 3 * EPS, ratio.max()
    near = (edge[ok] < 0.2)
    assert near.sum() > 10 and ratio[near].max() > 0.5, (near.sum(), ratio[near].max())


# ------------------------------------------------------------------------------------------
# slow-light modulation


def _modulated_grid(a_gen=0.6, amp=0.2, n_snap=8):
    cells = np.ones((n_snap, 4, 4, 4))
    phase = list(2.0 * np.pi * S.uniform_stream(S.S0 + 64, 4))
    return S.Grid(cells=cells, r_in=1.1, r_out=50.0, hslope=0.3, a_gen=a_gen, t0=0.0, dt_snap=10.0,
                  mod_amp=amp, mod_phase=phase)


def _density(orc, gh, r, ph, snap, dt=10.0):
    """n_e of a unit grid at (r, theta = 1, phi) in fast light at snapshot `snap` (its time t_s)."""
    return orc.grid_sample(gh, r, 1.0, ph=ph, slow_light=0, t_frame=snap * dt)[0]


def test_modulation_corotates_at_keplerian_rate(orc):
    g = _modulated_grid()
    gh = orc.GridHandle(g)
    for r in (2.0, 6.0, 31.0):
        om = 1.0 / (r ** 1.5 + g.a_gen)
        for ph in (0.0, 1.3, 4.0):
            v1 = _density(orc, gh, r, ph, 1)
            v5 = _density(orc, gh, r, ph + om * 40.0, 5)
            assert v5 == pytest.approx(v1, rel=1e-12, abs=1e-12)
            # and it does change in time at a fixed azimuth
            assert abs(_density(orc, gh, r, ph, 5) - v1) > 1e-6


def test_modulation_mean_bound_and_fourier_content(orc):
    g = _modulated_grid()
    gh = orc.GridHandle(g)
    n = 16
    phis = 2.0 * np.pi * np.arange(n) / n
    for r in (2.0, 9.0):
        om = 1.0 / (r ** 1.5 + g.a_gen)
        for snap in (0, 3):
            ts = snap * g.dt_snap
            v = np.array([_density(orc, gh, r, p, snap) for p in phis])
            assert v.mean() == pytest.approx(1.0, abs=1e-14)
            assert np.all(np.abs(v - 1.0) <= 4 * g.mod_amp + 1e-14)
            c = np.fft.fft((v - 1.0) / g.mod_amp) * 2.0 / n
            for m in range(1, 5):
                want = np.exp(1j * (g.mod_phase[m - 1] - m * om * ts))
                assert abs(c[m] - want) < 1e-12, (m, c[m], want)
            assert np.all(np.abs(c[5:n // 2]) < 1e-12) and abs(c[n // 2]) < 1e-12
    fine = np.array([_density(orc, gh, 3.0, p, 2) for p in np.linspace(0, 2 * np.pi, 2001)])
    assert np.abs(fine - 1.0).max() <= 4 * g.mod_amp


def test_modulation_off_is_identity(orc):
    g = _modulated_grid(amp=0.0)
    gh = orc.GridHandle(g)
    assert _density(orc, gh, 4.0, 2.0, 3) == 1.0


def test_oracle_refuses_too_many_frequencies(orc):
    cam = S.Camera(spin=0.5, incl_deg=60.0, nx=2, ny=2)
    gh = orc.GridHandle(S.constant_grid([1e5, 2.0, 3.0, 0.0]))
    o = orc.make_opts()
    with pytest.raises(ValueError):
        orc.trace_ray(cam, gh, o, 1.0, 1.0, [230e9] * (orc.MAX_NU + 1))
    with pytest.raises(ValueError):
        orc.trace_pixels(cam, gh, o, [230e9] * (orc.MAX_NU + 1), [0, 1])
    I, info, _ = orc.trace_ray(cam, gh, o, 1.0, 1.0, [230e9] * orc.MAX_NU)
    assert np.all(I == I[0])
