"""The oracle's optical-depth-aware step (Sec. 3.1, backward scheme: a step for the geodesic
and one for the transfer, the smaller taken).

Reading (the paper gives no rule for the transfer step): the step after a sample is at most
tau_step / max_f(alpha_f nu_r L) of affine parameter, so that the last sample's absorption at
its most absorbing frequency would add tau_step of optical depth; without a previous absorbing
sample the step follows the geometry alone.

Pins: the step sequence obeys that rule exactly and an unreachable limit changes nothing; the
most absorbing frequency sets the step; and on a medium whose exact observed intensity is an
integral along a straight line (flat space, static plasma), refining the geodesic step scale
and tau_step together converges to that integral at first order.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synthetic as S

R_IN, R_OUT, N1, N2 = 4.0, 16.0, 2048, 4
X_IN, X_OUT = math.log(R_IN), math.log(R_OUT)
B_IMPACT = 3.0
NU = 230e9


def onset(x):
    """(4 (x - x_in)(x_out - x) / (x_out - x_in)^2)^4: density profile vanishing smoothly at both
    faces of the shell, so that the first samples inside it are optically thin."""
    q = 4.0 * (x - X_IN) * (X_OUT - x) / (X_OUT - X_IN) ** 2
    return q ** 4


def shell(n0):
    """Flat-space static shell 4 < r < 16: n_e = n0 onset(ln r), Theta_e = 20 r_in / r, B = 10 G."""
    x1 = X_IN + (np.arange(N1) + 0.5) * (X_OUT - X_IN) / N1
    cells = np.zeros((1, N2, N1, 4))
    cells[0, :, :, 0] = n0 * onset(x1)
    cells[0, :, :, 1] = 20.0 * np.exp(X_IN - x1)
    cells[0, :, :, 2] = 10.0
    return S.Grid(cells=cells, r_in=R_IN, r_out=R_OUT, hslope=1.0, a_gen=0.0)


CAM = S.Camera(spin=0.0, incl_deg=90.0, nx=2, ny=1, fov_half=6.0)   # pixel 1: alpha = +3, beta = 0


def exact_intensity(orc, n0, nu=NU):
    """The observed intensity along the straight line of impact parameter 3 (equatorial, static
    plasma: nu_r = 1, cos theta_B = -b/r) from the ODE dtau/ds = alpha, dI/ds = j exp(-tau), with
    the oracle's closure as the local coefficients."""
    Lu = orc.length_unit(4.5e6)
    half = math.sqrt(R_OUT ** 2 - B_IMPACT ** 2)
    hole = math.sqrt(R_IN ** 2 - B_IMPACT ** 2)

    def rhs(s, y):
        r = math.hypot(B_IMPACT, s - half)
        if not (R_IN <= r <= R_OUT):
            return [0.0, 0.0]
        x = math.log(r)
        j, a = orc.closure(nu, n0 * onset(x), 20.0 * math.exp(X_IN - x), 10.0, -B_IMPACT / r)
        return [a * Lu, j * Lu * math.exp(-y[0])]

    y = [0.0, 0.0]
    for a0, a1 in ((0.0, half - hole), (half + hole, 2.0 * half)):
        sol = solve_ivp(rhs, (a0, a1), y, method="DOP853", rtol=1e-11, atol=1e-30)
        y = list(sol.y[:, -1])
    return y[1], y[0]


def trace(orc, gh, eps, tau_step, nu=(NU,), record=0):
    o = orc.make_opts(eps=eps, metric_mass=0.0, max_steps=1000000, tau_step=tau_step)
    return orc.trace_ray(CAM, gh, o, B_IMPACT, 0.0, list(nu), record=record)


def test_step_sequence_follows_the_rule(orc):
    g = shell(1e9)
    gh = orc.GridHandle(g)
    Lu = orc.length_unit(4.5e6)
    eps, ts = 0.05, 0.1
    I, info, rec = trace(orc, gh, eps, ts, record=100000)
    n = info.steps
    limited = 0
    for i in range(1, n):
        prev = rec[i - 1]
        h_geo = orc.step_size(eps, list(prev.x), list(prev.k))
        h = abs(rec[i].dl)
        if prev.sampled and prev.alpha > 0.0:
            cap = ts / (prev.alpha * prev.nu_r * Lu)
            assert h == pytest.approx(min(h_geo, cap), rel=1e-13)
            limited += cap < h_geo
            # the optical depth the previous sample's absorption gives this step is at most tau_step
            assert prev.alpha * prev.nu_r * Lu * h <= ts * (1 + 1e-12)
        else:
            assert h == pytest.approx(h_geo, rel=1e-13)
    assert limited > 100
    # an unreachable limit is no limit: bitwise the geometric run
    I0, info0 = trace(orc, gh, eps, 0.0)[:2]
    Ibig, infob = trace(orc, gh, eps, 1e300)[:2]
    assert Ibig[0] == I0[0] and infob.steps == info0.steps
    assert info.steps > info0.steps


def test_most_absorbing_frequency_sets_the_step(orc):
    """At 10 GHz the shell absorbs more than at 230 GHz at every sample, so a run at both takes
    exactly the steps of a run at 10 GHz alone, and its 10 GHz intensity is that run's."""
    gh = orc.GridHandle(shell(1e5))
    I2, info2, rec2 = trace(orc, gh, 0.05, 0.1, nu=(1e10, NU), record=20000)
    I1, info1, rec1 = trace(orc, gh, 0.05, 0.1, nu=(1e10,), record=20000)
    Ih, infoh = trace(orc, gh, 0.05, 0.1, nu=(NU,))[:2]
    assert info2.steps == info1.steps and info1.steps > 2 * infoh.steps and info1.steps <= 20000
    assert all(rec2[i].dl == rec1[i].dl for i in range(info1.steps))
    assert I2[0] == I1[0]


def test_joint_refinement_converges_at_first_order(orc):
    """tau_step = 10 eps, both halved four times: the error against the exact line integral
    (total optical depth 84) falls by a factor near 2 each time, to below 3e-4."""
    n0 = 1e9
    gh = orc.GridHandle(shell(n0))
    exact, tau_tot = exact_intensity(orc, n0)
    assert 50.0 < tau_tot < 150.0
    errs = []
    for k in range(5):
        eps = 0.04 / 2 ** k
        I = trace(orc, gh, eps, 10.0 * eps)[0]
        errs.append(abs(I[0] / exact - 1.0))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    print(f"[tau step] errors {errs} ratios {ratios}")
    assert all(1.6 <= q <= 2.4 for q in ratios)
    assert errs[-1] < 3e-4
