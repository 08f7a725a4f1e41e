"""Pins of the oracle's transfer integration and of its MLP reference.

Independent references: the analytic solution of a uniform emitting/absorbing shell in
flat space, the telescoping identity of the per-step formal solution, the forward
(plasma-to-camera) recursion of Sec. 3.1 over the same path, the optically thin sum, and
torch's float64 autograd for the MLP.
"""
import math

import numpy as np
import pytest

import synthetic as S


def slab_setup(orc, j0, a0_per_M, eps, mass=4.5e6, max_steps=100000):
    g = S.constant_grid((1.0, 1.0, 1.0, 0.0), r_in=5.0, r_out=15.0)
    gh = orc.GridHandle(g)
    Lu = orc.length_unit(mass)
    opts = orc.make_opts(eps=eps, closure=orc.CONST, const_j=j0, const_alpha=a0_per_M / Lu,
                         metric_mass=0.0, mass_msun=mass, max_steps=max_steps)
    return gh, opts, Lu


def chord(b, r1=5.0, r2=15.0):
    if b >= r2:
        return 0.0
    if b >= r1:
        return 2 * math.sqrt(r2 * r2 - b * b)
    return 2 * (math.sqrt(r2 * r2 - b * b) - math.sqrt(r1 * r1 - b * b))


@pytest.mark.parametrize("al,be", [(3.0, 2.0), (-8.0, 6.0), (0.7, -11.5)])
def test_uniform_shell_converges_to_analytic(orc, al, be):
    """Flat space, static fluid, constant j and alpha inside 5 <= r <= 15:
    I = (j/alpha)(1 - exp(-alpha l)) with l the chord; the error falls like eps (the steps
    straddling the shell boundaries)."""
    cam = S.Camera(spin=0.0, incl_deg=55.0, nx=2, ny=2)
    j0, a0 = 2e-20, 0.1
    errs = []
    for eps in (0.02, 0.01, 0.005, 0.0025):
        gh, opts, Lu = slab_setup(orc, j0, a0, eps)
        Iv, info, _ = orc.trace_ray(cam, gh, opts, al, be, [230e9])
        assert info.status == 2
        l = chord(math.hypot(al, be)) * Lu
        exact = j0 / (a0 / Lu) * (1 - math.exp(-(a0 / Lu) * l))
        errs.append(abs(Iv[0] / exact - 1))
    assert errs[-1] < 5e-3, errs
    assert errs[0] / errs[-1] > 3.0, errs     # O(eps): 8x shorter steps, >3x smaller error


def test_optically_thin_shell_is_emission_times_chord(orc):
    cam = S.Camera(spin=0.0, incl_deg=40.0, nx=2, ny=2)
    gh, opts, Lu = slab_setup(orc, 3e-21, 0.0, 0.001)
    Iv, info, _ = orc.trace_ray(cam, gh, opts, 2.0, 1.0, [1e11])
    assert info.status == orc.ESCAPED
    assert Iv[0] == pytest.approx(3e-21 * chord(math.hypot(2.0, 1.0)) * Lu, rel=2e-3)


def test_telescoping_identity_any_partition(orc):
    """sum_n exp(-tau_n) S (1 - exp(-dtau_n)) = S (1 - exp(-tau_total)) for constant S."""
    cam = S.Camera(spin=0.0, incl_deg=55.0, nx=2, ny=2)
    for eps in (0.05, 0.013):
        gh, opts, Lu = slab_setup(orc, 1e-20, 0.3, eps)
        Iv, info, rec = orc.trace_ray(cam, gh, opts, 1.5, -2.5, [230e9], record=20000)
        tot = sum(r.alpha * r.ds for r in rec[: info.steps] if r.sampled)
        S_ = 1e-20 / (0.3 / Lu)
        assert Iv[0] == pytest.approx(S_ * (-math.expm1(-tot)), rel=1e-13)


def test_forward_recursion_equals_backward_sum(orc):
    """Sec. 3.1: integrating the formal solution from the far end toward the camera over the
    stored path gives the same observed intensity as the backward scheme."""
    cam, g, nu = S.small_image()
    gh = orc.GridHandle(g)
    opts = orc.make_opts()
    hits = 0
    for (i, j) in [(40, 20), (31, 33), (10, 50), (52, 12)]:
        al, be = orc.pixel_alpha_beta(cam, i, j)
        Iv, info, rec = orc.trace_ray(cam, gh, opts, al, be, nu, record=20000)
        fw = orc.forward_transfer(rec, info.steps)
        assert fw == pytest.approx(Iv[0], rel=1e-12, abs=1e-300)
        hits += Iv[0] > 0
    assert hits >= 2


def test_spectrum_equals_single_frequencies(orc):
    cam, g, _ = S.small_image()
    gh = orc.GridHandle(g)
    opts = orc.make_opts()
    nus = [2e10, 230e9, 5e12]
    al, be = orc.pixel_alpha_beta(cam, 33, 30)
    Iv, _, _ = orc.trace_ray(cam, gh, opts, al, be, nus)
    for f, nu in enumerate(nus):
        I1, _, _ = orc.trace_ray(cam, gh, opts, al, be, [nu])
        assert I1[0] == Iv[f]


def test_step_limit_and_horizon_rays(orc):
    cam, g, nu = S.small_image()
    gh = orc.GridHandle(g)
    Iv, info, _ = orc.trace_ray(cam, gh, orc.make_opts(max_steps=1), 1.0, 1.0, nu)
    assert info.status == orc.MAXSTEP and info.steps == 1 and Iv[0] == 0.0
    Iv, info, _ = orc.trace_ray(cam, gh, orc.make_opts(), 0.3, 0.2, nu)   # inside the shadow
    assert info.status == orc.HORIZON and Iv[0] > 0.0


def test_flux_of_uniform_image(orc):
    cam = S.Camera(spin=0.0, incl_deg=60.0, nx=8, ny=4, fov_half=20.0)
    opts = orc.make_opts(mass_msun=4.5e6, dist_pc=8500.0)
    img = np.full((1, 4, 8), 2.0e-3)
    Lcm = 6.67430e-8 * 4.5e6 * 1.98847e33 / 2.99792458e10 ** 2
    fov_sr = (40.0 * Lcm / (8500.0 * 3.085677581e18)) ** 2
    assert orc.flux_jy(cam, opts, img)[0] == pytest.approx(2.0e-3 * fov_sr * 1e23, rel=1e-12)


# --------------------------------------------------------------------------- MLP reference

def torch_mlp(params):
    import torch
    dims = [3, 64, 64, 64, 64, 2]
    layers, o = [], 0
    for l in range(5):
        ni, no = dims[l], dims[l + 1]
        lin = torch.nn.Linear(ni, no).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(params[o:o + no * ni].reshape(no, ni)))
            lin.bias.copy_(torch.from_numpy(params[o + no * ni:o + no * ni + no]))
        o += no * ni + no
        layers.append(lin)
        if l < 4:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


def test_mlp_forward_backward_against_torch(orc):
    import torch
    n_p = orc.mlp_param_count()
    assert n_p == 12866
    rng = np.random.default_rng(11)
    params = rng.normal(0, 0.3, n_p)
    x = rng.uniform(-1, 1, (37, 3))
    dy = rng.normal(0, 1, (37, 2))
    net = torch_mlp(params)
    xt = torch.from_numpy(x)
    yt = net(xt)
    assert np.allclose(orc.mlp_forward(params, x), yt.detach().numpy(), rtol=1e-12, atol=1e-13)
    (yt * torch.from_numpy(dy)).sum().backward()
    ref = np.concatenate([torch.cat([m.weight.grad.ravel(), m.bias.grad.ravel()]).numpy()
                          for m in net if isinstance(m, torch.nn.Linear)])
    assert np.allclose(orc.mlp_backward(params, x, dy), ref, rtol=1e-11, atol=1e-12)


def test_mlp_backward_central_differences(orc):
    rng = np.random.default_rng(5)
    n_p = orc.mlp_param_count()
    params = rng.normal(0, 0.3, n_p)
    x = rng.uniform(-1, 1, (5, 3))
    dy = rng.normal(0, 1, (5, 2))
    g = orc.mlp_backward(params, x, dy)
    for idx in rng.choice(n_p, 25, replace=False):
        h = 1e-6
        p1, p2 = params.copy(), params.copy()
        p1[idx] += h
        p2[idx] -= h
        fd = ((orc.mlp_forward(p1, x) - orc.mlp_forward(p2, x)) * dy).sum() / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-9)


def test_tau_cutoff_on_a_uniform_shell(orc):
    """Optical-depth cut-off (Sec. 3.1, backward scheme) on the uniform shell: the ray stops at
    the first step where tau >= tau_c, reports OPAQUE, takes fewer steps, and by the telescoping
    identity I = S (1 - exp(-tau_stop)) with tau_c <= tau_stop < tau_c + (last step's dtau); the
    intensity lost against the full ray is at most S exp(-tau_c)."""
    cam = S.Camera(spin=0.0, incl_deg=55.0, nx=2, ny=2)
    j0, a0 = 2e-20, 0.5          # optical depth ~5 across the shell
    gh, opts, Lu = slab_setup(orc, j0, a0, 0.01)
    full, info_f, _ = orc.trace_ray(cam, gh, opts, 3.0, 2.0, [230e9])
    tau_c = math.log(20.0)
    opts.tau_cutoff = tau_c
    cut, info_c, rec = orc.trace_ray(cam, gh, opts, 3.0, 2.0, [230e9], record=100000)
    assert info_f.status == orc.ESCAPED and info_c.status == orc.OPAQUE
    assert info_c.steps < info_f.steps
    S_ = j0 / (a0 / Lu)
    taus = np.cumsum([r.alpha * r.ds for r in rec[: info_c.steps] if r.sampled])
    assert taus[-1] >= tau_c > taus[-2]
    assert cut[0] == pytest.approx(S_ * -math.expm1(-taus[-1]), rel=1e-13)
    assert 0.0 <= full[0] - cut[0] <= S_ * math.exp(-tau_c)


def test_tau_cutoff_truncates_the_same_sum(orc):
    """On the synthetic torus at 1 GHz (partly opaque): the cut ray's intensity is the full
    ray's backward sum truncated at the first step with tau >= tau_c, and the emission lost
    beyond it is at most exp(-tau_c) times its unattenuated sum."""
    cam, g, nu = S.small_image()
    gh = orc.GridHandle(g)
    tau_c = math.log(1000.0)
    opts = orc.make_opts()
    n_opaque = 0
    for px, py in [(32, 32), (30, 36), (40, 28), (25, 33), (36, 40)]:
        al, be = orc.pixel_alpha_beta(cam, px, py)
        full, info_f, rec = orc.trace_ray(cam, gh, opts, al, be, [1e9], record=20000)
        opts_c = orc.make_opts(tau_cutoff=tau_c)
        cut, info_c, _ = orc.trace_ray(cam, gh, opts_c, al, be, [1e9])
        I, tau, k_stop, lost_bound = 0.0, 0.0, None, 0.0
        for k, r in enumerate(rec[: info_f.steps]):
            if not r.sampled:
                continue
            dtau = r.alpha * r.ds
            A = (r.j / r.alpha) * -math.expm1(-dtau) / r.nu_r ** 3 if dtau > 0 else r.j * r.ds / r.nu_r ** 3
            if k_stop is None:
                I += math.exp(-tau) * A
                tau += dtau
                if tau >= tau_c:
                    k_stop = k
            else:
                lost_bound += A
        if k_stop is None:
            assert info_c.status == info_f.status and cut[0] == full[0]
            continue
        n_opaque += 1
        assert info_c.status == orc.OPAQUE and info_c.steps == k_stop + 1
        assert cut[0] == pytest.approx(I, rel=1e-13)
        assert 0.0 <= full[0] - cut[0] <= math.exp(-tau_c) * lost_bound * (1 + 1e-12)
    assert n_opaque >= 2


def test_tau_cutoff_needs_every_frequency_opaque(orc):
    """With two frequencies a ray stops only once it is opaque at both: the rays the pair stops
    are those both single-frequency runs stop, after the later of their two step counts."""
    cam, g, nu = S.small_image()
    gh = orc.GridHandle(g)
    o1 = orc.make_opts(tau_cutoff=math.log(1000.0))
    pix = np.arange(0, cam.nx * cam.ny, 7, dtype=np.int64)
    _, st_a = orc.trace_pixels(cam, gh, o1, [1e8], pix)
    _, st_b = orc.trace_pixels(cam, gh, o1, [1e9], pix)
    _, st_ab = orc.trace_pixels(cam, gh, o1, [1e8, 1e9], pix)
    both = (st_a[:, 0] == orc.OPAQUE) & (st_b[:, 0] == orc.OPAQUE)
    assert both.sum() > 10 and ((st_a[:, 0] == orc.OPAQUE) & ~both).sum() > 10
    assert np.array_equal(st_ab[:, 0] == orc.OPAQUE, both)
    assert np.array_equal(st_ab[both, 1], np.maximum(st_a[both, 1], st_b[both, 1]))
