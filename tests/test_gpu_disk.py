"""The thin-disk line test (Sec. 4.2.1) on the GPU through the C ABI against the CPU oracle:
same status per pixel, redshift and intensity per pixel to 1e-6, and the line profile; the full
workload (five spins from -0.99 to 0.99 at 512^2) sampled against the oracle."""
import numpy as np
import pytest

import synthetic as S
from gpu_common import oracle_opts, rel_err, sample_pixels

pytestmark = pytest.mark.gpu

SPINS = [-0.99, -0.5, 0.0, 0.5, 0.99]


@pytest.fixture(scope="module")
def R():
    from paper_1801_10452_amd import raptor
    return raptor


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("a,integ", [(0.99, "RK4"), (-0.99, "RK4"), (0.0, "RK4"), (0.5, "VERLET_CORRECTED")])
def test_disk_image_matches_oracle(R, ctx, orc, a, integ):
    cam = S.Camera(spin=a, incl_deg=60.0, nx=96, ny=96, fov_half=16.0)
    opts = R.default_opts(integrator=getattr(R, integ))
    status = np.zeros((cam.ny, cam.nx), np.int32)
    steps = np.zeros((cam.ny, cam.nx), np.int32)
    I, g, prof, st = ctx.trace_disk(cam, opts, 15.0, 200, 0.0, 2.0, ray_status=status, ray_steps=steps)
    og, oI, ost = orc.trace_disk_image(cam, oracle_opts(orc, opts), 15.0)
    hit = ost[:, 0] == orc.DISK
    print(f"[disk a={a} {integ}] disk rays {st.samples} (oracle {hit.sum()}) ray_steps {st.ray_steps} "
          f"kernel_ms {st.kernel_ms:.2f}", flush=True)
    assert np.array_equal(status.ravel(), ost[:, 0])
    assert np.array_equal(steps.ravel(), ost[:, 1])
    assert st.samples == hit.sum() and hit.sum() > 1000
    eg = rel_err(g, og)
    eI = rel_err(I, oI)
    print(f"[disk a={a} {integ}] max rel err g {eg.max():.3e} I {eI.max():.3e}", flush=True)
    assert eg.max() <= 1e-6 and eI.max() <= 1e-6
    # the GPU binning of the GPU pixels equals the oracle's binning of the same pixels
    ref_prof = orc.disk_profile(cam, g, I, 200, 0.0, 2.0)
    assert np.allclose(prof, ref_prof, rtol=1e-12, atol=0)
    # and the oracle's own profile up to pixels whose g sits within the parity error of a bin edge
    own = orc.disk_profile(cam, og, oI, 200, 0.0, 2.0)
    assert abs(prof.sum() - own.sum()) <= 1e-6 * own.sum()


def test_disk_workload_full_size(R, ctx, orc):
    """Five spins at 512^2, i = 60 deg: throughput and sampled parity."""
    opts = R.default_opts()
    total_ms, total_steps = 0.0, 0
    worst = 0.0
    for k, a in enumerate(SPINS):
        cam = S.Camera(spin=a, incl_deg=60.0, nx=512, ny=512, fov_half=16.0)
        I, g, prof, st = ctx.trace_disk(cam, opts, 15.0, 200, 0.0, 2.0)
        total_ms += st.kernel_ms
        total_steps += st.ray_steps
        pix = sample_pixels(cam, 24, seed=S.S0 + 600 + k)
        for p in pix:
            al, be = orc.pixel_alpha_beta(cam, int(p % cam.nx), int(p // cam.nx))
            og, orc_r, oI, info = orc.trace_disk_ray(cam, oracle_opts(orc, opts), 15.0, al, be)
            for got, ref in ((g.ravel()[p], og), (I.ravel()[p], oI)):
                worst = max(worst, abs(got - ref) / max(abs(ref), 1e-300) if ref != 0 else abs(got))
    print(f"[disk workload] 5 x 512^2: {total_ms:.1f} ms, {total_steps / total_ms * 1e3:.3e} ray-steps/s, "
          f"worst sampled rel err {worst:.3e}", flush=True)
    assert worst <= 1e-6
