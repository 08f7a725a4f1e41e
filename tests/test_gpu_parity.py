"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Gates: per-pixel |I_gpu - I_ref| / max(|I_ref|, 1e-10 max I_ref) <= 1e-6 with FP64 transfer;
identical ray termination codes and step counts; fluxes to 1e-6.  FP32 transfer is held to
the bound stated at its test and its error distribution is printed.
"""
import math

import numpy as np
import pytest

import synthetic as S
from tests.gpu_common import oracle_opts, rel_err, report, sample_pixels

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-6


@pytest.fixture(scope="module")
def R():
    from paper_1801_10452_amd import raptor
    return raptor


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def gpu_and_oracle(R, ctx, orc, cam, grid, nu, **kw):
    opts = R.default_opts(**kw)
    gh = ctx.upload_grid(grid)
    status = np.zeros((cam.ny, cam.nx), np.int32)
    steps = np.zeros((cam.ny, cam.nx), np.int32)
    img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts, ray_status=status, ray_steps=steps)
    ctx.release_grid(gh)
    ref_img, ref_flux, ref_st = orc.trace_image(cam, orc.GridHandle(grid), oracle_opts(orc, opts), nu)
    return img, flux, st, status, steps, ref_img, ref_flux, ref_st


def test_small_image_fp64(R, ctx, orc):
    """64 x 64, a = 0.9375, i = 60 deg, float64 128^2 grid, 230 GHz, FP64 transfer."""
    cam, g, nu = S.small_image()
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(R, ctx, orc, cam, g, nu)
    same_steps = (steps.ravel() == ref_st[:, 1])
    same_status = (status.ravel() == ref_st[:, 0])
    print(f"steps equal {same_steps.mean():.5f} status equal {same_status.mean():.5f} "
          f"ray_steps={st.ray_steps} oracle={ref_st[:, 1].sum()} samples={st.samples}", flush=True)
    assert same_status.all()
    assert same_steps.all()
    assert st.rays == cam.nx * cam.ny and st.ray_steps == ref_st[:, 1].sum()
    err = rel_err(img, ref)
    report("small fp64", err)
    assert err.max() <= TOL_FP64
    assert flux[0] == pytest.approx(ref_flux[0], rel=TOL_FP64)


@pytest.mark.parametrize("nx,ny", [(1, 1), (13, 7), (8, 9), (65, 3)])
def test_ragged_and_tiny_images(R, ctx, orc, nx, ny):
    """Image sizes that leave partial 8x8 tiles (and a single pixel)."""
    g = S.make_grid(32, 24, a_gen=0.5, dtype=np.float64)
    cam = S.Camera(spin=0.5, incl_deg=45.0, nx=nx, ny=ny, fov_half=12.0)
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(R, ctx, orc, cam, g, [86e9, 230e9])
    assert (steps.ravel() == ref_st[:, 1]).all() and (status.ravel() == ref_st[:, 0]).all()
    err = rel_err(img, ref)
    assert err.max() <= TOL_FP64, err.max()
    assert np.allclose(flux, ref_flux, rtol=TOL_FP64, atol=0)   # a sum of pixels each within 1e-6


@pytest.mark.parametrize("spin,incl", [(-0.9, 60.0), (0.998, 85.0), (0.5, 2.0), (0.9375, 178.0), (0.0, 90.0)])
def test_extreme_spins_and_inclinations(R, ctx, orc, spin, incl):
    """Retrograde, near-extremal (horizon at r = 1.063) and zero spin; cameras 2 degrees from
    either pole, whose rays pass close to the axis where the polar term of the step rule
    shortens the steps, and edge-on.  20 x 20 over +-15 M of a float64 48 x 40 grid made with
    the same spin: identical termination codes and step counts, pixels and flux within 1e-6."""
    g = S.make_grid(48, 40, a_gen=spin, dtype=np.float64)
    cam = S.Camera(spin=spin, incl_deg=incl, nx=20, ny=20, fov_half=15.0)
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(R, ctx, orc, cam, g, [230e9])
    print(f"[extreme a={spin} i={incl}] horizon {st.n_horizon} escaped {st.n_escaped} pole {st.n_pole} "
          f"steps {st.ray_steps}", flush=True)
    assert (status.ravel() == ref_st[:, 0]).all() and (steps.ravel() == ref_st[:, 1]).all()
    assert st.n_horizon == (ref_st[:, 0] == R.RAY_HORIZON).sum() and st.n_escaped == (ref_st[:, 0] == R.RAY_ESCAPED).sum()
    err = rel_err(img, ref)
    report(f"extreme a={spin} i={incl}", err)
    assert err.max() <= TOL_FP64
    assert np.allclose(flux, ref_flux, rtol=TOL_FP64, atol=0)


def test_step_limit_writes_zero_and_counts(R, ctx, orc):
    cam, g, nu = S.small_image()
    cam = S.Camera(spin=cam.spin, incl_deg=cam.incl_deg, nx=16, ny=16)
    img, flux, st, status, steps, ref, _, _ = gpu_and_oracle(R, ctx, orc, cam, g, nu, max_steps=1)
    assert (status == R.RAY_MAXSTEP).all() and (steps == 1).all()
    assert st.n_maxstep == 256 and st.ray_steps == 256 and not img.any() and not ref.any()


def test_flat_space_uniform_shell(R, ctx, orc):
    """Flat space, static plasma, constant j and alpha (the analytic-shell configuration)."""
    g = S.constant_grid((1.0, 1.0, 1.0, 0.0), r_in=5.0, r_out=15.0)
    cam = S.Camera(spin=0.0, incl_deg=55.0, nx=24, ny=24)
    Lu = orc.length_unit(4.5e6)
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(
        R, ctx, orc, cam, g, [230e9], closure=R.CLOSURE_CONST, const_j=2e-20, const_alpha=0.1 / Lu,
        metric_mass=0.0, eps=0.01, max_steps=100000)
    assert (steps.ravel() == ref_st[:, 1]).all()
    assert rel_err(img, ref).max() <= TOL_FP64


def test_paper_k2_closure(R, ctx, orc):
    cam, g, nu = S.small_image()
    cam = S.Camera(spin=cam.spin, incl_deg=cam.incl_deg, nx=32, ny=32)
    img, flux, st, status, steps, ref, ref_flux, _ = gpu_and_oracle(R, ctx, orc, cam, g, nu,
                                                                    closure=R.CLOSURE_K2_PAPER)
    assert rel_err(img, ref).max() <= TOL_FP64


def test_spectrum_matches_single_frequency_calls(R, ctx):
    cam, g, _ = S.small_image()
    cam = S.Camera(spin=cam.spin, incl_deg=cam.incl_deg, nx=24, ny=24)
    gh = ctx.upload_grid(g)
    nus = [2e10, 86e9, 230e9, 1e13]
    imgs, flux, _ = ctx.trace_spectrum(cam, gh, nus)
    for f, nu in enumerate(nus):
        one, fl1, _ = ctx.trace_image(cam, gh, nu)
        assert np.array_equal(one, imgs[f]) and fl1[0] == flux[f]
    ctx.release_grid(gh)


def test_batch_matches_single_calls(R, ctx):
    g1 = S.make_grid(64, 64, a_gen=0.9375, dtype=np.float32)
    g2 = S.make_grid(64, 64, a_gen=0.3, dtype=np.float32)
    h1, h2 = ctx.upload_grid(g1), ctx.upload_grid(g2)
    cams = [S.Camera(0.9375, 60.0, 16, 16), S.Camera(0.3, 20.0, 24, 8), S.Camera(-0.5, 85.0, 9, 17),
            S.Camera(0.9375, 40.0, 32, 32)]
    grids = [h1, h2, h2, h1]
    nus = [[230e9, 86e9], [43e9, 22e9], [230e9, 1e12], [1e11, 2e11]]
    from paper_1801_10452_amd.raptor import split_batch_images
    for prec in (R.F64, R.F32):
        opts = R.default_opts(transfer_prec=prec)
        imgs, flux, st = ctx.trace_batch(cams, grids, nus, opts)
        parts = split_batch_images(imgs, cams, 2)
        for k, c in enumerate(cams):
            one, fl, _ = ctx.trace_spectrum(c, grids[k], nus[k], opts)
            assert np.array_equal(one, parts[k]), (prec, k)
            assert np.array_equal(fl, flux[k])
    ctx.release_grid(h1)
    ctx.release_grid(h2)


def test_slow_light_and_fast_light(R, ctx, orc):
    """Time series of 64 modulated snapshots, three frequencies; slow and fast light."""
    g = S.make_grid(48, 48, a_gen=0.9375, dtype=np.float32, n_snap=64, dt_snap=10.0, mod_amp=0.2)
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=24, ny=24, t_frame=320.0)
    for slow in (1, 0):
        img, flux, st, status, steps, ref, ref_flux, _ = gpu_and_oracle(R, ctx, orc, cam, g, [1e10, 230e9, 1e14],
                                                                        slow_light=slow)
        err = rel_err(img, ref)
        report(f"slow_light={slow}", err)
        assert err.max() <= TOL_FP64


def test_fp32_transfer_error(R, ctx, orc):
    """FP64 geodesic with FP32 emission, absorption and per-step contributions (exponent
    arguments and the running sums in FP64) against the FP64 oracle: the same 1e-6 per-pixel
    bound as the FP64 form; the distribution is printed."""
    cam, g, nu = S.small_image()
    img, flux, st, status, steps, ref, ref_flux, _ = gpu_and_oracle(R, ctx, orc, cam, g, nu,
                                                                    transfer_prec=R.F32)
    err = rel_err(img, ref)
    report("small fp32 transfer", err)
    assert err.max() <= TOL_FP64
    assert flux[0] == pytest.approx(ref_flux[0], rel=TOL_FP64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_production_batch_sampled_parity(R, ctx, orc, prec):
    """The benchmark's launch: 9 images of 512 x 512 (spins {0, 0.5, 0.9375} x inclinations
    {30, 60, 85}) on float32 256^2 grids in one batch, 230 GHz; per image 24 seeded random pixels
    and the 24 brightest pixels of the GPU image against the oracle; with FP32 transfer also the
    benchmark's own launch (device memory, graph capture and replay) bit for bit against that."""
    sets = S.production_set()
    cams = [c for c, _ in sets]
    handles = {}
    grids = []
    for c, g in sets:
        if id(g) not in handles:
            handles[id(g)] = ctx.upload_grid(g)
        grids.append(handles[id(g)])
    opts = R.default_opts(transfer_prec=R.F64 if prec == "f64" else R.F32)
    imgs, flux, st = ctx.trace_batch(cams, grids, [S.NU_230], opts)
    print(f"[production {prec}] rays={st.rays} steps={st.ray_steps} samples={st.samples} "
          f"kernel_ms={st.kernel_ms:.1f} horizon={st.n_horizon} escaped={st.n_escaped} max={st.n_maxstep}",
          flush=True)
    assert st.rays == 9 * 512 * 512 and st.n_numeric == 0
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, cams, 1)
    worst = 0.0
    for k, (c, g) in enumerate(sets):
        bright = np.argsort(parts[k][0].ravel())[-24:]
        pix = np.unique(np.concatenate([sample_pixels(c, 24, seed=S.S0 + 300 + k), bright]))
        ref, info = orc.trace_pixels(c, orc.GridHandle(g), oracle_opts(orc, opts), [S.NU_230], pix)
        got = parts[k][0].ravel()[pix]
        scale = max(np.abs(ref).max(), np.abs(parts[k]).max())
        e = np.abs(got - ref[:, 0]) / np.maximum(np.abs(ref[:, 0]), 1e-10 * scale)
        worst = max(worst, e.max())
    print(f"[production {prec}] worst sampled rel err {worst:.3e}", flush=True)
    assert worst <= TOL_FP64
    if prec == "f32":
        # the benchmark's launch configuration (device-resident outputs, the launch captured as a
        # graph and replayed) gives bitwise the images and fluxes checked above
        import torch
        dimg = torch.empty(imgs.size, dtype=torch.float64, device="cuda")
        dflux = torch.empty(flux.size, dtype=torch.float64, device="cuda")
        gopts = R.default_opts(transfer_prec=R.F32, mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH)
        for rep in range(2):
            dimg.fill_(-1.0)
            dflux.fill_(-1.0)
            torch.cuda.synchronize()
            gst = ctx.trace_batch(cams, grids, [S.NU_230], gopts, images=dimg, flux=dflux)[2]
            assert np.array_equal(dimg.cpu().numpy(), np.ravel(imgs)), rep
            assert np.array_equal(dflux.cpu().numpy(), np.ravel(flux)), rep
            assert gst.ray_steps == st.ray_steps and gst.samples == st.samples
    for h in handles.values():
        ctx.release_grid(h)


def test_device_memory_outputs_match_host(R, ctx):
    import torch
    cam, g, nu = S.small_image()
    gh = ctx.upload_grid(g)
    host, hflux, _ = ctx.trace_spectrum(cam, gh, nu)
    dimg = torch.zeros((1, cam.ny, cam.nx), dtype=torch.float64, device="cuda")
    dflux = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ctx.trace_spectrum(cam, gh, nu, R.default_opts(mem=R.MEM_DEVICE), images=dimg, flux=dflux)
    assert np.array_equal(dimg.cpu().numpy(), host) and dflux.item() == hflux[0]
    ctx.release_grid(gh)


def test_invalid_arguments_write_nothing(R, ctx):
    cam, g, nu = S.small_image()
    gh = ctx.upload_grid(g)
    img = np.full((1, cam.ny, cam.nx), 7.0)
    for bad_cam, kw in [(S.Camera(spin=1.2, incl_deg=60, nx=64, ny=64), {}),
                        (S.Camera(spin=0.5, incl_deg=0.0, nx=64, ny=64), {}),
                        (S.Camera(spin=0.5, incl_deg=60, nx=64, ny=64, r_cam=30.0), {}),
                        (S.Camera(spin=0.5, incl_deg=60, nx=0, ny=64), {}),
                        (S.Camera(spin=0.5, incl_deg=60, nx=64, ny=64), {"eps": -1.0}),
                        (S.Camera(spin=0.5, incl_deg=60, nx=64, ny=64), {"transfer_prec": 7})]:
        with pytest.raises(R.RaptorError) as ei:
            ctx.trace_spectrum(bad_cam, gh, nu, R.default_opts(**kw), images=img)
        assert ei.value.status == R.E_INVALID
        assert (img == 7.0).all()
    with pytest.raises(R.RaptorError):
        ctx.trace_spectrum(cam, gh, [-1.0], images=img)
    with pytest.raises(R.RaptorError):
        ctx.trace_spectrum(cam, gh, [1.0] * 40)
    ctx.release_grid(gh)


def test_graph_replay_matches_direct_launch(R, ctx):
    """RAPTOR_LAUNCH_GRAPH: the captured launch replayed several times, with direct launches and
    other device work in between and with new camera values in the same job-table shape, gives
    bitwise the results of the direct launch each time."""
    import torch
    sets = S.production_set(res=64)
    cams = [c for c, _ in sets]
    handles, grids = {}, []
    for c, g in sets:
        if id(g) not in handles:
            handles[id(g)] = ctx.upload_grid(g)
        grids.append(handles[id(g)])
    nu = [S.NU_230, 2 * S.NU_230]
    direct = R.default_opts(transfer_prec=R.F32)
    graph = R.default_opts(transfer_prec=R.F32, launch=R.LAUNCH_GRAPH)
    ref_img, ref_flux, ref_st = ctx.trace_batch(cams, grids, nu, direct)
    cams_b = [S.Camera(spin=c.spin, incl_deg=c.incl_deg + 5.0, nx=c.nx, ny=c.ny) for c in cams]
    ref_img_b, ref_flux_b, _ = ctx.trace_batch(cams_b, grids, nu, direct)
    for rep in range(4):
        use_b = rep == 2
        img, flux, st = ctx.trace_batch(cams_b if use_b else cams, grids, nu, graph)
        assert np.array_equal(img, ref_img_b if use_b else ref_img), rep
        assert np.array_equal(flux, ref_flux_b if use_b else ref_flux), rep
        if not use_b:
            assert st.ray_steps == ref_st.ray_steps and st.samples == ref_st.samples
        # eager work between replays: a direct launch and an unrelated torch reduction
        ctx.trace_batch(cams[:2], grids[:2], nu, direct)
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float64)
        assert float(x.sum()) == float((1 << 20) * ((1 << 20) - 1) // 2)
        torch.cuda.synchronize()
    for h in handles.values():
        ctx.release_grid(h)


@pytest.mark.parametrize("integ", ["RK2", "VERLET", "VERLET_CORRECTED"])
def test_second_order_integrators_match_oracle(R, ctx, orc, integ):
    """The 64^2 image with the midpoint rule and velocity Verlet (with and without corrector)
    against the oracle's same integrator: same status per pixel, step counts, 1e-6 per pixel."""
    cam, g, nu = S.small_image()
    opts = R.default_opts(integrator=getattr(R, integ))
    gh = ctx.upload_grid(g)
    status = np.zeros((cam.ny, cam.nx), np.int32)
    steps = np.zeros((cam.ny, cam.nx), np.int32)
    img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts, ray_status=status, ray_steps=steps)
    ctx.release_grid(gh)
    ref, ref_flux, ref_st = orc.trace_image(cam, orc.GridHandle(g), oracle_opts(orc, opts), nu)
    same_steps = (steps.ravel() == ref_st[:, 1]).mean()
    err = rel_err(img, ref)
    report(f"small {integ}", err)
    print(f"[small {integ}] ray_steps={st.ray_steps} (oracle {ref_st[:, 1].sum()}) steps equal {same_steps:.5f}",
          flush=True)
    assert (status.ravel() == ref_st[:, 0]).all()
    assert same_steps == 1.0
    assert err.max() <= TOL_FP64
    assert flux[0] == pytest.approx(ref_flux[0], rel=TOL_FP64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tau_cutoff_matches_oracle(R, ctx, orc, prec):
    """Optical-depth cut-off at ln 1000 on the 64^2 image at 0.1 and 1 GHz (opaque core): the
    same rays stop (status OPAQUE) after the same step as in the oracle, and the intensities
    agree to 1e-6; samples queued after the cut are dropped."""
    cam, g, _ = S.small_image()
    nu = [1e8, 1e9]
    opts = R.default_opts(transfer_prec=R.F64 if prec == "f64" else R.F32, tau_cutoff=math.log(1000.0))
    gh = ctx.upload_grid(g)
    status = np.zeros((cam.ny, cam.nx), np.int32)
    steps = np.zeros((cam.ny, cam.nx), np.int32)
    img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts, ray_status=status, ray_steps=steps)
    ctx.release_grid(gh)
    ref, ref_flux, ref_st = orc.trace_image(cam, orc.GridHandle(g), oracle_opts(orc, opts), nu)
    n_opq = int((ref_st[:, 0] == orc.OPAQUE).sum())
    print(f"[tau cutoff {prec}] opaque rays {st.n_opaque} (oracle {n_opq})", flush=True)
    assert n_opq > 50 and st.n_opaque == n_opq
    assert np.array_equal(status.ravel(), ref_st[:, 0])
    assert np.array_equal(steps.ravel(), ref_st[:, 1])
    err = rel_err(img, ref)
    report(f"tau cutoff {prec}", err)
    assert err.max() <= TOL_FP64


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n_nu", [6, 12])
def test_eight_and_sixteen_frequency_kernels(R, ctx, orc, prec, n_nu):
    """6 and 12 frequencies select the kernels compiled for up to 8 and 16 frequencies per ray
    (the spectrum tests use 1-4 and 24).  24 x 20 pixels (ragged 8 x 8 tiles) on a float32 48^2
    grid, log-spaced 1 GHz to 10 THz: same status and steps per ray as the oracle, every
    frequency's image within 1e-6 per pixel of its own brightest pixel's floor, fluxes to 1e-6."""
    g = S.make_grid(48, 48, a_gen=0.9375, dtype=np.float32)
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=24, ny=20, fov_half=15.0)
    nu = list(np.geomspace(1e9, 1e13, n_nu))
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(
        R, ctx, orc, cam, g, nu, transfer_prec=R.F64 if prec == "f64" else R.F32)
    assert (status.ravel() == ref_st[:, 0]).all() and (steps.ravel() == ref_st[:, 1]).all()
    err = rel_err(img, ref)
    for f in range(n_nu):
        report(f"{n_nu} frequencies {prec}, {nu[f]:.3g} Hz", err[f])
    assert err.max() <= TOL_FP64
    assert np.allclose(flux, ref_flux, rtol=TOL_FP64, atol=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scale,nu", [(1e-3, [1e8, 1e9, 1e10]), (3e-3, [1e8, 1e9, 230e9]),
                                      (3e3, [1e9, 230e9, 1e13])])
def test_cold_and_hot_plasma(R, ctx, orc, prec, scale, nu):
    """Electron temperatures beyond the K2 table: the torus with Theta_e scaled by 1e-3 and 3e-3
    (Theta_e from 4e-4 to 0.05, where 1/K2 alone exceeds the float range and, below ~0.0014, the
    double range) and by 3e3 (up to 5e4, above the table's 2^14).  The closure applies 1/K2 and the
    cut-off exp(-X^1/3) as one exponential in both precisions; per pixel and flux within 1e-6 of
    the oracle, whose K2 is the integral representation (no table)."""
    g = S.make_grid(40, 40, a_gen=0.5, dtype=np.float64)
    g.cells[..., 1] *= scale
    cam = S.Camera(spin=0.5, incl_deg=60.0, nx=24, ny=24, fov_half=15.0)
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(
        R, ctx, orc, cam, g, nu, transfer_prec=R.F64 if prec == "f64" else R.F32)
    assert np.isfinite(img).all() and st.n_numeric == 0
    assert all((ref[f] > 0).any() for f in range(len(nu)))
    err = rel_err(img, ref)
    for f in range(len(nu)):
        report(f"Theta_e x {scale:g} {prec}, {nu[f]:.3g} Hz", err[f])
    assert err.max() <= TOL_FP64
    assert np.allclose(flux, ref_flux, rtol=TOL_FP64, atol=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nu,cut", [([1e9, 3e9], math.log(1000.0)), ([3e9], 0.0)])
def test_optical_depth_aware_step_matches_oracle(R, ctx, orc, prec, nu, cut):
    """The optical-depth-aware step (tau_step = 0.1: after a sample the next step is at most the
    affine step over which that sample's absorption at its most absorbing frequency gives an
    optical depth of 0.1) on the 64^2 image at 1 and 3 GHz with the ln 1000 cut-off, and at 3 GHz
    without it: the same statuses and step counts as the oracle (FP32 transfer: the step is set
    by FP32 optical depths, and step counts may differ by one on up to 0.5% of the rays) and
    intensities within 1e-6 per pixel.  The limited steps add rays' steps where the torus is
    opaque."""
    cam, g, _ = S.small_image()
    kw = dict(transfer_prec=R.F64 if prec == "f64" else R.F32, tau_step=0.1, tau_cutoff=cut)
    img, flux, st, status, steps, ref, ref_flux, ref_st = gpu_and_oracle(R, ctx, orc, cam, g, nu, **kw)
    _, _, st0, _, steps0, _, _, _ = gpu_and_oracle(R, ctx, orc, cam, g, nu, **dict(kw, tau_step=0.0))
    same = steps.ravel() == ref_st[:, 1]
    err = rel_err(img, ref)
    print(f"[tau step {prec} nu={nu}] ray-steps {st.ray_steps} (geometric {st0.ray_steps}), steps equal "
          f"{same.mean():.5f}, flux {flux} oracle {ref_flux}", flush=True)
    report(f"tau step {prec} nu={nu}", err)
    assert st.ray_steps > st0.ray_steps
    assert np.array_equal(status.ravel(), ref_st[:, 0])
    if prec == "f64":
        assert same.all()
    else:
        assert same.mean() >= 0.995 and np.abs(steps.ravel() - ref_st[:, 1]).max() <= 1
    assert err.max() <= TOL_FP64
    assert np.allclose(flux, ref_flux, rtol=TOL_FP64, atol=0)
