"""Full-size workloads through the C ABI, sampled against the CPU oracle.

* spectrum + slow light: 256^2, a = 0.9375, i = 60 deg, 24 frequencies 1e9..1e16 Hz on shared
  geodesics, 64 modulated float32 snapshots (slow light) or the frame's snapshot (fast light);
* uneven batch: 256 images of {64, 128, 256, 512}^2 with random spin and inclination, 4 VLBI
  frequencies, one shared float32 grid, in one persistent launch.

Per sampled pixel and frequency the relative error against the oracle is bounded by 1e-6
(floor 1e-10 of the image maximum at that frequency), for the FP64 and FP32 transfer forms.
"""
import math

import numpy as np
import pytest

import synthetic as S
from gpu_common import oracle_opts, sample_pixels

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def R():
    from paper_1801_10452_amd import raptor
    return raptor


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def sampled_errors(orc, cam, grid, opts, nu, img, pix):
    """Max over the sampled pixels and all frequencies of the parity metric; img [n_nu][ny][nx]."""
    ref, _ = orc.trace_pixels(cam, orc.GridHandle(grid), oracle_opts(orc, opts), nu, pix)
    worst = 0.0
    for f in range(len(nu)):
        got = img[f].ravel()[pix]
        scale = max(np.abs(img[f]).max(), np.abs(ref[:, f]).max(), 1e-300)
        e = np.abs(got - ref[:, f]) / np.maximum(np.abs(ref[:, f]), 1e-10 * scale)
        worst = max(worst, float(e.max()))
    return worst


@pytest.fixture(scope="module")
def slow_set():
    return S.slow_light_set()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("slow", [0, 1])
def test_spectrum_slow_light_full_size(R, ctx, orc, slow_set, prec, slow):
    cam, grid, nu = slow_set
    gh = ctx.upload_grid(grid)
    opts = R.default_opts(transfer_prec=R.F32 if prec == "f32" else R.F64, slow_light=slow)
    img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts)
    print(f"[spectrum slow={slow} {prec}] rays={st.rays} steps={st.ray_steps} samples={st.samples} "
          f"kernel_ms={st.kernel_ms:.1f} flux[0,11,23]={flux[0]:.4e},{flux[11]:.4e},{flux[23]:.4e}", flush=True)
    assert st.rays == cam.nx * cam.ny and st.n_numeric == 0
    assert np.isfinite(img).all() and (img >= 0).all()
    f_peak = int(np.argmax(flux))
    bright = np.argsort(img[f_peak].ravel())[-12:]
    pix = np.unique(np.concatenate([sample_pixels(cam, 12, seed=S.S0 + 400 + slow), bright]))
    worst = sampled_errors(orc, cam, grid, opts, nu, img, pix)
    print(f"[spectrum slow={slow} {prec}] {pix.size} pixels x {len(nu)} frequencies: worst rel err {worst:.3e}",
          flush=True)
    assert worst <= TOL
    ctx.release_grid(gh)


@pytest.mark.parametrize("slow", [0, 1])
def test_spectrum_autotuned_graph_replay(R, ctx, slow_set, slow):
    """The 24-frequency spectrum in its timed form (FP32 transfer, fast and slow light): the plan the
    autotuner picks, with the launch captured as a graph and replayed, gives bitwise the images
    and fluxes of the default plan's direct launch, the one checked against the oracle above."""
    import torch
    cam, grid, nu = slow_set
    gh = ctx.upload_grid(grid)
    opts = R.default_opts(transfer_prec=R.F32, slow_light=slow)
    ref_i, ref_f, ref_st = ctx.trace_spectrum(cam, gh, nu, opts)
    default_plan = R.get_plan(ctx, len(nu), R.F32)
    plan, ms = R.autotune_batch(ctx, [cam], [gh], nu, opts, reps=1)
    print(f"[spectrum slow={slow} autotune] plan {plan.as_dict()} best kernel {ms:.2f} ms (default {ref_st.kernel_ms:.2f} ms)",
          flush=True)
    img = torch.empty(ref_i.size, dtype=torch.float64, device="cuda")
    flux = torch.empty(ref_f.size, dtype=torch.float64, device="cuda")
    graph = R.default_opts(transfer_prec=R.F32, mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH, slow_light=slow)
    for rep in range(2):
        img.fill_(-1.0)
        flux.fill_(-1.0)
        torch.cuda.synchronize()
        st = ctx.trace_spectrum(cam, gh, nu, graph, images=img, flux=flux)[2]
        assert np.array_equal(img.cpu().numpy(), np.ravel(ref_i)), rep
        assert np.array_equal(flux.cpu().numpy(), np.ravel(ref_f)), rep
        assert st.ray_steps == ref_st.ray_steps and st.samples == ref_st.samples
    R.set_plan(ctx, len(nu), R.F32, default_plan)
    ctx.release_grid(gh)


def test_uneven_batch_full_size(R, ctx, orc):
    cams = S.batch_jobs()
    grid = S.make_grid(256, 256, a_gen=0.9375, dtype=np.float32)
    gh = ctx.upload_grid(grid)
    nu = S.NU_VLBI
    opts = R.default_opts(transfer_prec=R.F32)
    imgs, flux, st = ctx.trace_batch(cams, [gh] * len(cams), nu, opts)
    n_pix = sum(c.nx * c.ny for c in cams)
    print(f"[uneven batch] images={len(cams)} rays={st.rays} steps={st.ray_steps} samples={st.samples} "
          f"kernel_ms={st.kernel_ms:.1f}", flush=True)
    assert st.rays == n_pix and st.n_numeric == 0
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, cams, len(nu))
    worst = 0.0
    for k in range(0, len(cams), 16):   # a fixed 16-image subset
        c = cams[k]
        bright = np.argsort(parts[k][3].ravel())[-2:]
        pix = np.unique(np.concatenate([sample_pixels(c, 2, seed=S.S0 + 500 + k), bright]))
        worst = max(worst, sampled_errors(orc, c, grid, opts, nu, parts[k], pix))
    print(f"[uneven batch] 16 images, 4 pixels x 4 frequencies each: worst rel err {worst:.3e}", flush=True)
    assert worst <= TOL
    # images of the batch equal their single calls bit for bit
    for k in (0, 101, 255):
        one, fone, _ = ctx.trace_spectrum(cams[k], gh, nu, opts)
        assert np.array_equal(one, parts[k]) and np.array_equal(fone, np.asarray(flux)[k])
    ctx.release_grid(gh)


def test_uneven_batch_autotuned_graph_replay(R, ctx):
    """The uneven batch in its timed form: the autotuner picks a plan on the 256 images (exact
    closure, FP32 transfer), and the graph-captured launch replayed twice under that plan gives
    bitwise the images and fluxes of the direct launch under the same plan, which equal those of
    the default plan (checked against the oracle above) bit for bit."""
    import torch
    cams = S.batch_jobs()
    grid = S.make_grid(256, 256, a_gen=0.9375, dtype=np.float32)
    gh = ctx.upload_grid(grid)
    grids = [gh] * len(cams)
    nu = S.NU_VLBI
    dflt_i, dflt_f, _ = ctx.trace_batch(cams, grids, nu, R.default_opts(transfer_prec=R.F32))
    default_plan = R.get_plan(ctx, len(nu), R.F32)
    plan, ms = R.autotune_batch(ctx, cams, grids, nu, R.default_opts(transfer_prec=R.F32), reps=1)
    print(f"[uneven batch autotune] plan {plan.as_dict()} best kernel {ms:.1f} ms", flush=True)
    n = sum(c.nx * c.ny for c in cams) * len(nu)
    ref_i, ref_f, ref_st = ctx.trace_batch(cams, grids, nu, R.default_opts(transfer_prec=R.F32))
    assert np.array_equal(ref_i, dflt_i) and np.array_equal(ref_f, dflt_f)
    img = torch.empty(n, dtype=torch.float64, device="cuda")
    flux = torch.empty((len(cams), len(nu)), dtype=torch.float64, device="cuda")
    graph = R.default_opts(transfer_prec=R.F32, mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH)
    for rep in range(2):
        _, _, st = ctx.trace_batch(cams, grids, nu, graph, images=img, flux=flux)
        torch.cuda.synchronize()
        assert np.array_equal(img.cpu().numpy(), ref_i) and np.array_equal(flux.cpu().numpy(), ref_f), rep
        assert st.ray_steps == ref_st.ray_steps
    print(f"[uneven batch graph] {st.kernel_ms:.1f} ms, {st.ray_steps / st.kernel_ms * 1e3:.3e} ray-steps/s",
          flush=True)
    R.set_plan(ctx, len(nu), R.F32, default_plan)
    ctx.release_grid(gh)


def test_light_curve_batch(R, ctx, orc):
    """Light curve (Sec. 5): 16 slow-light frames of one camera, t_frame stepping by 10 M across
    the 64-snapshot stack, traced as one batch at 4 VLBI frequencies.  Each frame's flux equals
    the flux of its single call, and sampled pixels match the oracle; the fast-light curve of the
    same frames is printed beside it (the synthetic modulation rotates with the Keplerian flow)."""
    cam0, grid, _ = S.slow_light_set(res=64)
    gh = ctx.upload_grid(grid)
    frames = [S.Camera(spin=cam0.spin, incl_deg=cam0.incl_deg, nx=64, ny=64, t_frame=grid.t0 + 100.0 + 10.0 * k)
              for k in range(16)]
    nu = S.NU_VLBI
    slow = R.default_opts(transfer_prec=R.F32, slow_light=1)
    fast = R.default_opts(transfer_prec=R.F32, slow_light=0)
    imgs, flux_s, st = ctx.trace_batch(frames, [gh] * len(frames), nu, slow)
    _, flux_f, _ = ctx.trace_batch(frames, [gh] * len(frames), nu, fast)
    flux_s, flux_f = np.asarray(flux_s), np.asarray(flux_f)
    rel = flux_s[:, 3] / flux_f[:, 3] - 1
    print(f"[light curve] 230 GHz slow/fast - 1 per frame: {np.array2string(rel, precision=3)}; "
          f"kernel_ms {st.kernel_ms:.2f}", flush=True)
    for k in (0, 7, 15):
        _, one, _ = ctx.trace_spectrum(frames[k], gh, nu, slow)
        assert np.array_equal(one, flux_s[k])
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, frames, len(nu))
    worst = 0.0
    for k in (3, 11):
        pix = sample_pixels(frames[k], 12, seed=S.S0 + 700 + k)
        worst = max(worst, sampled_errors(orc, frames[k], grid, slow, nu, parts[k], pix))
    print(f"[light curve] sampled worst rel err {worst:.3e}", flush=True)
    assert worst <= TOL
    assert np.all(np.abs(rel) < 0.5) and np.abs(rel).max() > 1e-6   # slow light changes the curve
    ctx.release_grid(gh)


@pytest.mark.parametrize("integ", ["RK4", "RK2", "VERLET", "VERLET_CORRECTED"])
def test_integrators_production_batch(R, ctx, orc, integ):
    """The production batch (9 x 512^2, 230 GHz, FP32 transfer) with each integrator of
    Sec. 2.2: throughput, and sampled pixels against the oracle's same integrator."""
    sets = S.production_set()
    hs = {}
    for _, g in sets:
        if id(g) not in hs:
            hs[id(g)] = ctx.upload_grid(g)
    cams = [c for c, _ in sets]
    opts = R.default_opts(transfer_prec=R.F32, integrator=getattr(R, integ))
    ctx.trace_batch(cams, [hs[id(g)] for _, g in sets], [S.NU_230], opts)   # warm-up
    imgs, flux, st = ctx.trace_batch(cams, [hs[id(g)] for _, g in sets], [S.NU_230], opts)
    print(f"[integrator {integ}] 9 x 512^2: kernel_ms {st.kernel_ms:.2f}, ray_steps {st.ray_steps}, "
          f"{st.ray_steps / st.kernel_ms * 1e3:.3e} ray-steps/s, {9 / st.kernel_ms * 1e3:.0f} images/s", flush=True)
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, cams, 1)
    worst = 0.0
    for k, (c, g) in enumerate(sets):
        pix = sample_pixels(c, 4, seed=S.S0 + 900 + k)
        worst = max(worst, sampled_errors(orc, c, g, opts, [S.NU_230], parts[k], pix))
    print(f"[integrator {integ}] 36 sampled pixels: worst rel err {worst:.3e}", flush=True)
    assert st.n_numeric == 0 and worst <= TOL
    assert np.isfinite(imgs).all() and (imgs >= 0).all() and np.isfinite(flux).all()
    for h in hs.values():
        ctx.release_grid(h)


@pytest.mark.parametrize("nu_set", ["1GHz", "24"])
def test_tau_cutoff_full_size(R, ctx, orc, slow_set, nu_set):
    """Optical-depth cut-off (ln 1000) on the 256^2 spectrum camera, fast light: at 1 GHz (an
    opaque core) and over the 24 frequencies (a ray stops only when opaque at all of them).
    Timing with and without the cut, the flux-level difference (the lost emission is below
    e^-tau_cut of each stopped ray's source function), and sampled pixels against the oracle."""
    cam, grid, nu24 = slow_set
    nu = [1e9] if nu_set == "1GHz" else nu24
    gh = ctx.upload_grid(grid)
    base = R.default_opts(transfer_prec=R.F32)
    cut = R.default_opts(transfer_prec=R.F32, tau_cutoff=math.log(1000.0))
    ctx.trace_spectrum(cam, gh, nu, cut)   # warm-up
    i0, f0, s0 = ctx.trace_spectrum(cam, gh, nu, base)
    i1, f1, s1 = ctx.trace_spectrum(cam, gh, nu, cut)
    f0, f1 = np.asarray(f0), np.asarray(f1)
    rel = np.abs(f1 / f0 - 1.0)
    print(f"[tau cutoff {nu_set}] no cut {s0.kernel_ms:.2f} ms {s0.ray_steps} steps; cut {s1.kernel_ms:.2f} ms "
          f"{s1.ray_steps} steps, {s1.n_opaque} opaque rays; max |dF/F| {rel.max():.3e}", flush=True)
    assert s1.ray_steps <= s0.ray_steps and rel.max() <= 1e-3
    if nu_set == "1GHz":
        assert s1.n_opaque > 1000 and s1.ray_steps < s0.ray_steps
    pix = sample_pixels(cam, 10, seed=S.S0 + 950)
    worst = sampled_errors(orc, cam, grid, cut, nu, i1, pix)
    print(f"[tau cutoff {nu_set}] sampled worst rel err {worst:.3e}", flush=True)
    assert worst <= TOL
    ctx.release_grid(gh)


def test_optical_depth_aware_step_full_size(R, ctx, orc, slow_set):
    """The optical-depth-aware step (tau_step 0.1) on the 256^2 spectrum camera, fast light, FP32,
    at the spectrum's three lowest frequencies (1, 2 and 4.1 GHz, where the torus is opaque) with
    the ln 1000 cut-off: its cost in steps and time, the flux change against the geometric step alone
    (both are first-order discretisations of the same transfer integral, so they differ by less
    than 1%), and sampled pixels against the oracle's same rule."""
    cam, grid, nu24 = slow_set
    nu = list(nu24[:3])
    gh = ctx.upload_grid(grid)
    geo = R.default_opts(transfer_prec=R.F32, tau_cutoff=math.log(1000.0))
    lim = R.default_opts(transfer_prec=R.F32, tau_cutoff=math.log(1000.0), tau_step=0.1)
    ctx.trace_spectrum(cam, gh, nu, lim)   # warm-up
    i0, f0, s0 = ctx.trace_spectrum(cam, gh, nu, geo)
    i1, f1, s1 = ctx.trace_spectrum(cam, gh, nu, lim)
    f0, f1 = np.asarray(f0), np.asarray(f1)
    rel = f1 / f0 - 1.0
    print(f"[tau step full] geometric {s0.kernel_ms:.2f} ms {s0.ray_steps} steps; tau_step 0.1 {s1.kernel_ms:.2f} ms "
          f"{s1.ray_steps} steps, {s1.n_opaque} opaque rays; dF/F per frequency "
          f"{' '.join(f'{x:+.2e}' for x in rel)}",
          flush=True)
    assert s1.ray_steps > s0.ray_steps and s1.n_maxstep == 0 and np.abs(rel).max() < 1e-2
    pix = sample_pixels(cam, 10, seed=S.S0 + 960)
    worst = sampled_errors(orc, cam, grid, lim, nu, i1, pix)
    print(f"[tau step full] sampled worst rel err {worst:.3e}", flush=True)
    assert worst <= TOL
    ctx.release_grid(gh)


def test_light_curve_full_size(R, ctx, orc, slow_set):
    """A light curve of 32 slow-light frames of the 256^2 camera (t_frame stepping 10 M through
    the 64-snapshot stack) at the 4 VLBI frequencies, traced as one batch: throughput, frames
    equal to their single calls, and sampled pixels of two frames against the oracle."""
    cam0, grid, _ = slow_set
    gh = ctx.upload_grid(grid)
    frames = [S.Camera(spin=cam0.spin, incl_deg=cam0.incl_deg, nx=256, ny=256, t_frame=grid.t0 + 160.0 + 10.0 * k)
              for k in range(32)]
    nu = S.NU_VLBI
    opts = R.default_opts(transfer_prec=R.F32, slow_light=1)
    ctx.trace_batch(frames, [gh] * len(frames), nu, opts)   # warm-up
    imgs, flux, st = ctx.trace_batch(frames, [gh] * len(frames), nu, opts)
    flux = np.asarray(flux)
    print(f"[light curve 32 x 256^2] kernel_ms {st.kernel_ms:.2f}, {st.ray_steps / st.kernel_ms * 1e3:.3e} ray-steps/s, "
          f"{32 / st.kernel_ms * 1e3:.0f} frames/s; 230 GHz flux min/max "
          f"{flux[:, 3].min():.4e}/{flux[:, 3].max():.4e} Jy", flush=True)
    assert st.n_numeric == 0 and np.isfinite(flux).all()
    assert flux[:, 3].max() > flux[:, 3].min()          # the modulation makes the curve vary
    for k in (5, 26):
        _, one, _ = ctx.trace_spectrum(frames[k], gh, nu, opts)
        assert np.array_equal(np.asarray(one), flux[k])
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, frames, len(nu))
    worst = 0.0
    for k in (9, 22):
        pix = sample_pixels(frames[k], 8, seed=S.S0 + 970 + k)
        worst = max(worst, sampled_errors(orc, frames[k], grid, opts, nu, parts[k], pix))
    print(f"[light curve 32 x 256^2] sampled worst rel err {worst:.3e}", flush=True)
    assert worst <= TOL
    ctx.release_grid(gh)
