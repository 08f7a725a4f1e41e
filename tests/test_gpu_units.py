"""GRMHD code-unit grids with the R_low / R_high electron model (Sec. 4.2.2 scaling, Sec. 5
temperature ratio) through the C ABI against the CPU oracle: a 64^2 image at full parity in
both transfer precisions, a uniform grid against the CGS grid of its converted values, and the
production-size batch (3 spins x 3 inclinations at 512^2 on 256^2 float32 code-unit grids)
sampled against the oracle and timed."""
import numpy as np
import pytest

import synthetic as S
from gpu_common import oracle_opts, rel_err, report, sample_pixels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1801_10452_amd import raptor
    return raptor


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-6)])
def test_code_unit_image_matches_oracle(R, ctx, orc, prec, tol):
    cam = S.Camera(spin=0.9375, incl_deg=60.0, nx=64, ny=64)
    grid = S.make_code_grid(128, 128, a_gen=0.9375, dtype=np.float64)
    gh = ctx.upload_grid(grid)
    opts = R.default_opts(transfer_prec=R.F64 if prec == "f64" else R.F32)
    nu = S.NU_VLBI
    img, flux, st = ctx.trace_spectrum(cam, gh, nu, opts)
    ref, rflux, _ = orc.trace_image(cam, orc.GridHandle(grid), oracle_opts(orc, opts), nu)
    assert st.n_numeric == 0 and np.abs(img).max() > 0
    err = rel_err(img, ref)
    report(f"code units {prec}", err)
    print(f"[code units {prec}] flux {np.array2string(np.asarray(flux), precision=4)} Jy", flush=True)
    assert err.max() <= tol
    np.testing.assert_allclose(flux, rflux, rtol=tol)
    ctx.release_grid(gh)


def test_uniform_code_grid_equals_its_cgs_values(R, ctx, orc):
    cam = S.Camera(spin=0.5, incl_deg=60.0, nx=32, ny=32, fov_half=12.0)
    value = (1.0, 0.01, 0.05, 0.03)
    gc = S.constant_grid(value, units=1, mass_unit_g=5e17, r_low=1.0, r_high=10.0)
    cgs = orc.code_to_cgs(orc.GridHandle(gc), list(value), mass_msun=4.5e6)
    gp = S.constant_grid(tuple(cgs))
    opts = R.default_opts(transfer_prec=R.F64)
    hc, hp = ctx.upload_grid(gc), ctx.upload_grid(gp)
    ic, _, _ = ctx.trace_spectrum(cam, hc, [230e9], opts)
    ip, _, _ = ctx.trace_spectrum(cam, hp, [230e9], opts)
    e = rel_err(ic, ip)
    print(f"[uniform code grid] max rel diff to the CGS grid {e.max():.3e}", flush=True)
    assert np.abs(ic).max() > 0 and e.max() <= 1e-12
    ctx.release_grid(hc)
    ctx.release_grid(hp)


def test_code_unit_production_batch(R, ctx, orc):
    """9 x 512^2 on code-unit grids (one per spin), FP32 transfer: timing and sampled parity."""
    cams, grids, hs = [], [], {}
    for a in S.PROD_SPINS:
        g = S.make_code_grid(256, 256, a_gen=a, dtype=np.float32)
        hs[a] = (g, ctx.upload_grid(g))
        for inc in S.PROD_INCLS:
            cams.append(S.Camera(spin=a, incl_deg=inc, nx=512, ny=512))
            grids.append(a)
    opts = R.default_opts(transfer_prec=R.F32)
    imgs, flux, st = ctx.trace_batch(cams, [hs[a][1] for a in grids], [S.NU_230], opts)
    ms = st.kernel_ms
    print(f"[code-unit batch] 9 x 512^2: kernel_ms {ms:.2f}, {st.ray_steps / ms * 1e3:.3e} ray-steps/s, "
          f"samples {st.samples}, flux {np.array2string(np.asarray(flux)[:, 0], precision=4)} Jy", flush=True)
    from paper_1801_10452_amd.raptor import split_batch_images
    parts = split_batch_images(imgs, cams, 1)
    worst = 0.0
    for k, c in enumerate(cams):
        g = hs[grids[k]][0]
        bright = np.argsort(parts[k][0].ravel())[-3:]
        pix = np.unique(np.concatenate([sample_pixels(c, 5, seed=S.S0 + 800 + k), bright]))
        ref, _ = orc.trace_pixels(c, orc.GridHandle(g), oracle_opts(orc, opts), [S.NU_230], pix)
        got = parts[k][0].ravel()[pix]
        scale = max(np.abs(parts[k][0]).max(), 1e-300)
        e = np.abs(got - ref[:, 0]) / np.maximum(np.abs(ref[:, 0]), 1e-10 * scale)
        worst = max(worst, float(e.max()))
    print(f"[code-unit batch] sampled worst rel err {worst:.3e}", flush=True)
    assert st.n_numeric == 0 and worst <= 1e-6
    for a in hs:
        ctx.release_grid(hs[a][1])
