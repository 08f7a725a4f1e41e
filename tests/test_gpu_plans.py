"""Launch plans and the autotuner (scheduling row of the path): every plan of the search space
-- work-group size, tile width, refill threshold, work-groups per CU and the waves-per-SIMD
variant, which also sets the depth of the LDS sample queue -- gives the same images bit for bit
for every integrator and both transfer precisions; the autotuner installs a plan that is no
slower than the default and leaves the images unchanged."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu

PLANS = [dict(), dict(threads=64), dict(threads=128, tile_width=16), dict(tile_width=64, refill_threshold=32),
         dict(min_waves_per_simd=1), dict(min_waves_per_simd=2, blocks_per_cu=1),
         dict(min_waves_per_simd=3, refill_threshold=8, tile_width=32), dict(threads=512, blocks_per_cu=4),
         dict(min_waves_per_simd=3, rays_per_wave=32, tile_width=16), dict(min_waves_per_simd=3, rays_per_wave=16),
         dict(rays_per_wave=16, tile_width=64)]


@pytest.fixture(scope="module")
def R():
    from paper_1801_10452_amd import raptor
    return raptor


@pytest.fixture
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("integ", ["RK4", "RK2", "VERLET"])
def test_every_plan_gives_the_same_images(R, ctx, prec, integ):
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=96, ny=72)   # tiles of every width end ragged
    grid = S.make_grid(128, 128, a_gen=0.9375, dtype=np.float64)
    gh = ctx.upload_grid(grid)
    nu = S.NU_VLBI
    tp = R.F32 if prec == "f32" else R.F64
    opts = R.default_opts(transfer_prec=tp, integrator=getattr(R, integ))
    ref = None
    for pl in PLANS:
        R.set_plan(ctx, len(nu), tp, R.make_plan(**pl))
        img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts)
        if ref is None:
            ref, ref_flux, ref_st = img.copy(), np.array(flux), st
            assert np.abs(ref).max() > 0
            continue
        diff = np.abs(img - ref).max()
        print(f"[plans {integ} {prec}] {pl}: max |diff| {diff:.3e}, kernel_ms {st.kernel_ms:.3f}", flush=True)
        assert np.array_equal(img, ref) and np.array_equal(np.array(flux), ref_flux), pl
        assert (st.ray_steps, st.samples, st.rays) == (ref_st.ray_steps, ref_st.samples, ref_st.rays)
    ctx.release_grid(gh)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("depth", ["plain", "cutoff", "tau_step"])
def test_rays_per_wave_same_images(R, ctx, prec, depth):
    """Twelve frequencies (one queued sample per lane in every variant): 64, 32 and 16 rays per
    wave, with tiles as wide as the rays or narrower, give the same images bit for bit -- also
    with the optical-depth cut-off and the optical-depth-aware step, whose per-sample reductions
    run across the lanes that share a sample -- and the installed plan reports the rays and the
    tile width the launch uses."""
    import math
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=80, ny=56)   # ragged in both directions for every tile
    grid = S.make_grid(128, 128, a_gen=0.9375, dtype=np.float32)
    gh = ctx.upload_grid(grid)
    # the cut-off needs a ray opaque at every frequency: low frequencies where the torus is thick
    nu = S.spectrum_freqs(12, 1e9, 1e13) if depth == "plain" else S.spectrum_freqs(12, 1e8, 2e9)
    tp = R.F32 if prec == "f32" else R.F64
    kw = {"plain": {}, "cutoff": dict(tau_cutoff=math.log(1000.0)),
          "tau_step": dict(tau_cutoff=math.log(1000.0), tau_step=0.1)}[depth]
    opts = R.default_opts(transfer_prec=tp, **kw)
    ref = None
    for rays, tw, w in ((64, 8, 3), (32, 16, 3), (32, 32, 2), (16, 8, 1), (16, 64, 3), (32, 8, 2)):
        R.set_plan(ctx, len(nu), tp, R.make_plan(rays_per_wave=rays, tile_width=tw, min_waves_per_simd=w))
        got = R.get_plan(ctx, len(nu), tp)
        assert got.rays_per_wave == rays and got.tile_width == min(tw, rays)
        img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts)
        if ref is None:
            ref, ref_flux, ref_st = img.copy(), np.array(flux), st
            assert np.abs(ref).max() > 0
            continue
        print(f"[rays per wave {prec} {depth}] {rays} rays, tiles {tw}, {w} waves/SIMD: max |diff| "
              f"{np.abs(img - ref).max():.3e}, kernel_ms {st.kernel_ms:.3f}", flush=True)
        assert np.array_equal(img, ref) and np.array_equal(np.array(flux), ref_flux), (rays, tw, w)
        assert (st.ray_steps, st.samples, st.rays, st.n_opaque) == (ref_st.ray_steps, ref_st.samples, ref_st.rays,
                                                                    ref_st.n_opaque)
    print(f"[rays per wave {prec} {depth}] opaque {ref_st.n_opaque}, step limit {ref_st.n_maxstep} of {ref_st.rays} rays",
          flush=True)
    if depth == "cutoff":
        assert ref_st.n_opaque > 0   # the cut-off ends some rays here
    # where the variant keeps several samples per lane (one frequency) the plan runs 64 rays
    R.set_plan(ctx, 1, tp, R.make_plan(rays_per_wave=16))
    assert R.get_plan(ctx, 1, tp).rays_per_wave == 64
    ctx.release_grid(gh)


def test_invalid_plans_are_refused(R, ctx):
    for bad in (dict(threads=96), dict(tile_width=12), dict(min_waves_per_simd=4), dict(refill_threshold=0),
                dict(blocks_per_cu=-1), dict(rays_per_wave=8), dict(rays_per_wave=48)):
        with pytest.raises(R.RaptorError) as e:
            R.set_plan(ctx, 1, R.F32, R.make_plan(**bad))
        assert e.value.status == R.E_INVALID


def test_autotuner_installs_a_plan_no_slower_and_images_unchanged(R, ctx):
    sets = S.production_set(res=256)
    hs = {}
    for _, g in sets:
        if id(g) not in hs:
            hs[id(g)] = ctx.upload_grid(g)
    cams = [c for c, _ in sets]
    grids = [hs[id(g)] for _, g in sets]
    opts = R.default_opts(transfer_prec=R.F32)
    nu = [S.NU_230]
    before = [ctx.trace_batch(cams, grids, nu, opts) for _ in range(3)]
    ms_default = min(b[2].kernel_ms for b in before)
    best, best_ms = R.autotune_batch(ctx, cams, grids, nu, opts, reps=2)
    got = R.get_plan(ctx, 1, R.F32)
    assert got.as_dict() == best.as_dict()
    after = [ctx.trace_batch(cams, grids, nu, opts) for _ in range(3)]
    ms_tuned = min(a[2].kernel_ms for a in after)
    print(f"[autotune] default {ms_default:.3f} ms, tuned plan {best.as_dict()} {best_ms:.3f} ms "
          f"(re-timed {ms_tuned:.3f} ms)", flush=True)
    assert best_ms <= ms_default * 1.05
    assert np.array_equal(after[0][0], before[0][0])
    for h in hs.values():
        ctx.release_grid(h)
