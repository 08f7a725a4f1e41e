"""raptor_trace_batch_noalloc, the batch call that allocates nothing (its launch buffers live in
a fixed device array per GPU), against raptor_trace_batch: two calls in a row, the second with a
smaller batch, and the limits it refuses."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


def _device_batch(R, ctx, cams, grids, nu, opts, noalloc, with_flux=True):
    import torch
    n_nu = len(nu)
    total = sum(c.nx * c.ny for c in cams) * n_nu
    img = torch.full((total,), -1.0, dtype=torch.float64, device="cuda")
    flux = torch.full((len(cams), n_nu), -1.0, dtype=torch.float64, device="cuda") if with_flux else None
    torch.cuda.synchronize()
    if noalloc:
        st = R.trace_batch_noalloc(ctx, cams, grids, nu, opts, img, flux)
    else:
        st = ctx.trace_batch(cams, grids, nu, opts, images=img, flux=flux)[2]
    torch.cuda.synchronize()
    return img.cpu().numpy(), (flux.cpu().numpy() if with_flux else None), st


def test_noalloc_matches_trace_batch_twice_then_smaller():
    from paper_1801_10452_amd import raptor as R
    ctx = R.Context(0, use_torch_stream=True)
    g1 = S.make_grid(64, 64, a_gen=0.9375, dtype=np.float32)
    g2 = S.make_grid(48, 40, a_gen=0.3, dtype=np.float32)
    h1, h2 = ctx.upload_grid(g1), ctx.upload_grid(g2)
    # first call: six images of uneven size on two grids, four frequencies, FP32 transfer
    cams = [S.Camera(0.9375, 60.0, 64, 64), S.Camera(0.3, 20.0, 40, 24), S.Camera(-0.5, 85.0, 8, 9),
            S.Camera(0.9375, 40.0, 96, 32), S.Camera(0.3, 70.0, 17, 13), S.Camera(0.9375, 10.0, 64, 48)]
    grids = [h1, h2, h2, h1, h2, h1]
    nu = S.NU_VLBI
    opts = R.default_opts(transfer_prec=R.F32, mem=R.MEM_DEVICE)
    ref_img, ref_flux, ref_st = _device_batch(R, ctx, cams, grids, nu, opts, noalloc=False)
    img, flux, st = _device_batch(R, ctx, cams, grids, nu, opts, noalloc=True)
    print(f"[noalloc 1] rays={st.rays} steps={st.ray_steps} samples={st.samples}", flush=True)
    assert np.array_equal(img, ref_img) and np.array_equal(flux, ref_flux)
    assert st.rays == ref_st.rays and st.ray_steps == ref_st.ray_steps and st.samples == ref_st.samples
    assert (ref_flux > 0).all()
    # second call, smaller: two images, two frequencies, FP64 transfer, no flux output
    cams2 = [S.Camera(0.5, 45.0, 24, 16), S.Camera(-0.2, 30.0, 9, 7)]
    grids2 = [h2, h1]
    nu2 = [86e9, 230e9]
    opts2 = R.default_opts(transfer_prec=R.F64, mem=R.MEM_DEVICE)
    ref2, ref_flux2, ref_st2 = _device_batch(R, ctx, cams2, grids2, nu2, opts2, noalloc=False)
    img2, _, st2 = _device_batch(R, ctx, cams2, grids2, nu2, opts2, noalloc=True, with_flux=False)
    img3, flux3, st3 = _device_batch(R, ctx, cams2, grids2, nu2, opts2, noalloc=True)
    print(f"[noalloc 2] rays={st2.rays} steps={st2.ray_steps}", flush=True)
    assert np.array_equal(img2, ref2) and np.array_equal(img3, ref2) and np.array_equal(flux3, ref_flux2)
    assert st2.rays == ref_st2.rays == 24 * 16 + 9 * 7 and st2.ray_steps == ref_st2.ray_steps
    ctx.release_grid(h1)
    ctx.release_grid(h2)
    ctx.close()


def test_noalloc_refuses_what_it_cannot_do():
    import torch
    from paper_1801_10452_amd import raptor as R
    ctx = R.Context(0, use_torch_stream=True)
    g = S.make_grid(16, 16, a_gen=0.5, dtype=np.float32)
    h = ctx.upload_grid(g)
    cam = S.Camera(0.5, 60.0, 4, 4)
    img = torch.zeros(4 * 4 * R.RAPTOR_NOALLOC_MAX_CAMS * 2, dtype=torch.float64, device="cuda")
    dev = R.default_opts(mem=R.MEM_DEVICE)
    with pytest.raises(R.RaptorError) as ei:   # more cameras than the scratch holds
        R.trace_batch_noalloc(ctx, [cam] * (R.RAPTOR_NOALLOC_MAX_CAMS + 1), [h] * (R.RAPTOR_NOALLOC_MAX_CAMS + 1),
                              [230e9], dev, img)
    assert ei.value.status == R.E_RANGE
    with pytest.raises(R.RaptorError) as ei:   # host outputs
        R.trace_batch_noalloc(ctx, [cam], [h], [230e9], R.default_opts(), np.zeros(16))
    assert ei.value.status == R.E_INVALID
    with pytest.raises(R.RaptorError) as ei:   # graph launch
        R.trace_batch_noalloc(ctx, [cam], [h], [230e9], R.default_opts(mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH), img)
    assert ei.value.status == R.E_UNSUPPORTED
    # the largest batch it takes runs
    n = R.RAPTOR_NOALLOC_MAX_CAMS
    st = R.trace_batch_noalloc(ctx, [cam] * n, [h] * n, [230e9, 86e9], dev, img)
    assert st.rays == 16 * n
    ctx.release_grid(h)
    ctx.close()
