"""Helpers shared by the GPU tests: contexts, oracle references and the parity metric."""
import math

import numpy as np

import synthetic as S


def rel_err(gpu, ref, floor_frac=1e-10):
    """|I_gpu - I_ref| / max(|I_ref|, floor_frac * max|I_ref|), elementwise.  For a stack of
    images ([n_nu][ny][nx], or more leading axes) the floor is taken per image, from that
    image's own brightest pixel, so that a dim frequency is judged against itself and not
    against the brightest frequency of the stack."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim >= 3:
        peak = np.abs(ref).max(axis=(-2, -1), keepdims=True)
    else:
        peak = np.abs(ref).max() if ref.size else 0.0
    floor = floor_frac * np.maximum(peak, 1e-300)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)


def oracle_opts(orc, o):
    """The oracle options equal to a GPU raptor_opts."""
    return orc.make_opts(eps=o.eps, r_stop_factor=o.r_stop_factor, max_steps=o.max_steps, closure=o.closure,
                         slow_light=o.slow_light, mass_msun=o.mass_msun, dist_pc=o.dist_pc, const_j=o.const_j,
                         const_alpha=o.const_alpha, metric_mass=o.metric_mass, integrator=o.integrator,
                         tau_cutoff=o.tau_cutoff, tau_step=o.tau_step)


def sample_pixels(cam, n, seed):
    """n distinct pixel indices of the image, seeded (from the synthetic generator)."""
    u = S.uniform_stream(seed, 4 * n)
    pix = np.unique((u * (cam.nx * cam.ny)).astype(np.int64))
    return pix[:n]


def report(name, err, mask=None):
    e = err if mask is None else err[mask]
    if e.size == 0:
        print(f"[{name}] no pixels", flush=True)
        return
    print(f"[{name}] n={e.size} max={e.max():.3e} p99.9={np.quantile(e, 0.999):.3e} median={np.median(e):.3e}",
          flush=True)
