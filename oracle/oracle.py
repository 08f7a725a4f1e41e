"""ctypes binding of the CPU FP64 oracle (test infrastructure only).

Loaded by tests/, the smoke check and the benchmark's CPU-baseline leg; never by the
product package.  Inputs come from the ``synthetic`` module.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraptor_oracle.so")

EXACT, K2_PAPER, CONST = 0, 1, 2
MAX_NU = 64   # frequencies per ray the oracle accepts
RK4, RK2, VERLET, VERLET_CORR = 0, 1, 2, 3
RUNNING, HORIZON, ESCAPED, MAXSTEP, NUMERIC, OPAQUE, DISK, PLANE = 0, 1, 2, 3, 4, 5, 6, 7

DP = C.POINTER(C.c_double)


class Camera(C.Structure):
    _fields_ = [("spin", C.c_double), ("incl_deg", C.c_double), ("r_cam", C.c_double),
                ("fov_half", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32), ("t_frame", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n_snap", C.c_int32), ("is_f64", C.c_int32),
                ("r_in", C.c_double), ("r_out", C.c_double), ("hslope", C.c_double), ("a_gen", C.c_double),
                ("t0", C.c_double), ("dt_snap", C.c_double), ("mod_amp", C.c_double),
                ("mod_phase", C.c_double * 4), ("cells", C.c_void_p), ("units", C.c_int32),
                ("reserved", C.c_int32), ("mass_unit_g", C.c_double), ("r_low", C.c_double),
                ("r_high", C.c_double), ("gamma_ad", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("r_stop_factor", C.c_double), ("max_steps", C.c_int32),
                ("closure", C.c_int32), ("slow_light", C.c_int32), ("integrator", C.c_int32),
                ("mass_msun", C.c_double), ("dist_pc", C.c_double), ("const_j", C.c_double),
                ("const_alpha", C.c_double), ("metric_mass", C.c_double), ("tau_cutoff", C.c_double),
                ("tau_step", C.c_double)]


class RayInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int32), ("samples", C.c_int32), ("poles", C.c_int32)]


class StepRec(C.Structure):
    _fields_ = [("x", C.c_double * 4), ("k", C.c_double * 4), ("dl", C.c_double),
                ("sampled", C.c_int32), ("pad_", C.c_int32), ("nu_r", C.c_double), ("j", C.c_double),
                ("alpha", C.c_double), ("ds", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.orc_ks_metric.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, DP]
        L.orc_ks_metric_derivs.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, DP, DP]
        L.orc_bl_metric.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, DP]
        L.orc_invert4.argtypes = [DP, DP]
        L.orc_christoffel.argtypes = [C.c_double, C.c_double, DP, DP]
        L.orc_geodesic_rhs.argtypes = [C.c_double, C.c_double, DP, DP]
        L.orc_step_size.argtypes = [C.c_double, DP, DP]
        L.orc_step_size.restype = C.c_double
        L.orc_rk4_step.argtypes = [C.c_double, C.c_double, DP, C.c_double, DP]
        L.orc_integrate.argtypes = [C.c_double, C.c_double, DP, C.c_double, C.c_int, C.c_double,
                                    C.c_double, C.c_int, DP, DP, C.c_int, C.POINTER(RayInfo)]
        L.orc_rk2_step.argtypes = [C.c_double, C.c_double, DP, C.c_double, DP]
        L.orc_isco.argtypes = [C.c_double]
        L.orc_isco.restype = C.c_double
        L.orc_trace_disk_ray.argtypes = [C.POINTER(Camera), C.POINTER(Opts), C.c_double, C.c_double, C.c_double,
                                         DP, DP, DP, C.POINTER(RayInfo)]
        L.orc_trace_disk_image.argtypes = [C.POINTER(Camera), C.POINTER(Opts), C.c_double, DP, DP,
                                           C.POINTER(RayInfo), C.c_int]
        L.orc_disk_profile.argtypes = [C.POINTER(Camera), DP, DP, C.c_int, C.c_double, C.c_double, DP]
        L.orc_verlet_step.argtypes = [C.c_double, C.c_double, DP, DP, C.c_double, C.c_int, DP]
        L.orc_integrate.restype = C.c_int
        L.orc_pixel_alpha_beta.argtypes = [C.POINTER(Camera), C.c_int, C.c_int, DP, DP]
        L.orc_camera_ray.argtypes = [C.POINTER(Camera), C.c_double, C.c_double, C.c_double, C.c_double, DP, DP]
        L.orc_mks_x2.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int)]
        L.orc_mks_x2.restype = C.c_double
        L.orc_grid_sample.argtypes = [C.POINTER(Grid), C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, DP]
        L.orc_grid_sample.restype = C.c_int
        L.orc_code_to_cgs.argtypes = [C.POINTER(Grid), C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_code_to_cgs.restype = None
        L.orc_fluid_frame.argtypes = [C.c_double, C.c_double, DP, DP, C.c_double, DP, DP, DP, DP]
        L.orc_fluid_frame.restype = C.c_int
        L.orc_bessel_k2.argtypes = [C.c_double]
        L.orc_bessel_k2.restype = C.c_double
        L.orc_bessel_k2_scaled.argtypes = [C.c_double]
        L.orc_bessel_k2_scaled.restype = C.c_double
        L.orc_ln_bessel_k2.argtypes = [C.c_double]
        L.orc_ln_bessel_k2.restype = C.c_double
        L.orc_closure.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, DP, DP]
        L.orc_planck.argtypes = [C.c_double, C.c_double]
        L.orc_planck.restype = C.c_double
        L.orc_trace_ray.argtypes = [C.POINTER(Camera), C.POINTER(Grid), C.POINTER(Opts), C.c_double,
                                    C.c_double, DP, C.c_int, DP, C.POINTER(RayInfo), C.POINTER(StepRec), C.c_int]
        L.orc_trace_ray.restype = C.c_int
        L.orc_trace_pixels.argtypes = [C.POINTER(Camera), C.POINTER(Grid), C.POINTER(Opts), DP, C.c_int,
                                       C.POINTER(C.c_int64), C.c_int64, DP, C.POINTER(RayInfo), C.c_int]
        L.orc_trace_pixels.restype = C.c_int
        L.orc_pixel_solid_angle.argtypes = [C.POINTER(Camera), C.POINTER(Opts)]
        L.orc_pixel_solid_angle.restype = C.c_double
        L.orc_forward_transfer.argtypes = [C.POINTER(StepRec), C.c_int]
        L.orc_forward_transfer.restype = C.c_double
        L.orc_length_unit.argtypes = [C.c_double]
        L.orc_length_unit.restype = C.c_double
        L.orc_mlp_param_count.restype = C.c_int
        L.orc_mlp_forward.argtypes = [DP, DP, C.c_int64, DP]
        L.orc_mlp_backward.argtypes = [DP, DP, DP, C.c_int64, DP]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(DP)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n
    return a


# ------------------------------------------------------------------------------------------
# Structure builders from the synthetic inputs
# ------------------------------------------------------------------------------------------

def make_camera(cam) -> Camera:
    return Camera(cam.spin, cam.incl_deg, cam.r_cam, cam.fov_half, cam.nx, cam.ny, cam.t_frame)


class GridHandle:
    """Keeps the numpy cells alive while the C struct points at them."""

    def __init__(self, g):
        self.cells = np.ascontiguousarray(g.cells)
        ph = (C.c_double * 4)(*g.mod_phase)
        self.s = Grid(g.n1, g.n2, g.n_snap, 1 if self.cells.dtype == np.float64 else 0, g.r_in, g.r_out,
                      g.hslope, g.a_gen, g.t0, g.dt_snap, g.mod_amp, ph, self.cells.ctypes.data,
                      getattr(g, "units", 0), 0, getattr(g, "mass_unit_g", 0.0), getattr(g, "r_low", 1.0),
                      getattr(g, "r_high", 1.0), getattr(g, "gamma_ad", 13.0 / 9.0))


def make_opts(eps=0.05, r_stop_factor=1.01, max_steps=10000, closure=EXACT, slow_light=0,
              mass_msun=4.5e6, dist_pc=8500.0, const_j=0.0, const_alpha=0.0, metric_mass=1.0,
              integrator=0, tau_cutoff=0.0, tau_step=0.0) -> Opts:
    return Opts(eps, r_stop_factor, max_steps, closure, slow_light, integrator, mass_msun, dist_pc,
                const_j, const_alpha, metric_mass, tau_cutoff, tau_step)


# ------------------------------------------------------------------------------------------
# Thin wrappers
# ------------------------------------------------------------------------------------------

def ks_metric(a, M, r, th):
    g = np.zeros(16)
    lib().orc_ks_metric(a, M, r, th, _dp(g))
    return g.reshape(4, 4)


def ks_metric_derivs(a, M, r, th):
    g = np.zeros(16)
    dg = np.zeros(64)
    lib().orc_ks_metric_derivs(a, M, r, th, _dp(g), _dp(dg))
    return g.reshape(4, 4), dg.reshape(4, 4, 4)


def bl_metric(a, M, r, th):
    g = np.zeros(16)
    lib().orc_bl_metric(a, M, r, th, _dp(g))
    return g.reshape(4, 4)


def invert4(m):
    m = _f64(m, 16)
    inv = np.zeros(16)
    assert lib().orc_invert4(_dp(m), _dp(inv)) == 0
    return inv.reshape(4, 4)


def christoffel(a, M, x):
    x = _f64(x, 4)
    gam = np.zeros(64)
    lib().orc_christoffel(a, M, _dp(x), _dp(gam))
    return gam.reshape(4, 4, 4)


def geodesic_rhs(a, M, y):
    y = _f64(y, 8)
    f = np.zeros(8)
    lib().orc_geodesic_rhs(a, M, _dp(y), _dp(f))
    return f


def step_size(eps, x, k):
    x = _f64(x, 4)
    k = _f64(k, 4)
    return lib().orc_step_size(eps, _dp(x), _dp(k))


def rk4_step(a, M, y, dl):
    y = _f64(y, 8)
    out = np.zeros(8)
    lib().orc_rk4_step(a, M, _dp(y), dl, _dp(out))
    return out


def rk2_step(a, M, y, dl):
    y = _f64(y, 8)
    out = np.zeros(8)
    lib().orc_rk2_step(a, M, _dp(y), dl, _dp(out))
    return out


def verlet_step(a, M, y, acc, dl, corrector=False):
    """Returns (y_new, last evaluated derivative)."""
    y = _f64(y, 8)
    acc = _f64(acc, 4).copy()
    out = np.zeros(8)
    lib().orc_verlet_step(a, M, _dp(y), _dp(acc), dl, int(corrector), _dp(out))
    return out, acc


def integrate(a, M, y0, eps=0.05, max_steps=10000, r_stop=0.0, r_escape=1e4, cap=20000, integrator=RK4):
    y0 = _f64(y0, 8)
    traj = np.zeros((cap, 8))
    dls = np.zeros(cap)
    info = RayInfo()
    n = lib().orc_integrate(a, M, _dp(y0), eps, max_steps, r_stop, r_escape, integrator, _dp(traj), _dp(dls),
                            cap, C.byref(info))
    n = min(n, cap)
    return traj[:n], dls[:n], info


def pixel_alpha_beta(cam, i, j):
    al, be = C.c_double(), C.c_double()
    c = make_camera(cam)
    lib().orc_pixel_alpha_beta(C.byref(c), i, j, C.byref(al), C.byref(be))
    return al.value, be.value


def camera_ray(cam, alpha, beta, M=1.0, t_init=0.0):
    c = make_camera(cam)
    y = np.zeros(8)
    kc = np.zeros(4)
    lib().orc_camera_ray(C.byref(c), M, alpha, beta, t_init, _dp(y), _dp(kc))
    return y, kc


def mks_x2(h, th):
    it = C.c_int()
    x = lib().orc_mks_x2(h, th, C.byref(it))
    return x, it.value


def code_to_cgs(grid_handle, prim, mass_msun=4.5e6):
    """{rho, u, b, Omega} in code units -> {n_e, Theta_e, B, Omega} (orc_code_to_cgs)."""
    out = np.zeros(4)
    lib().orc_code_to_cgs(C.byref(grid_handle.s), mass_msun, _dp(_f64(prim, 4)), _dp(out))
    return out


def grid_sample(grid_handle, r, th, ph=0.0, t=0.0, slow_light=0, t_frame=0.0):
    out = np.zeros(4)
    ok = lib().orc_grid_sample(C.byref(grid_handle.s), slow_light, t_frame, r, th, ph, t, _dp(out))
    return (out if ok else None)


def fluid_frame(a, M, x, k, omega):
    x = _f64(x, 4)
    k = _f64(k, 4)
    u = np.zeros(4)
    b = np.zeros(4)
    nr, cb = C.c_double(), C.c_double()
    z = lib().orc_fluid_frame(a, M, _dp(x), _dp(k), omega, _dp(u), _dp(b), C.byref(nr), C.byref(cb))
    return u, b, nr.value, cb.value, bool(z)


def bessel_k2(x):
    return lib().orc_bessel_k2(x)


def bessel_k2_scaled(x):
    """e^x K_2(x)."""
    return lib().orc_bessel_k2_scaled(x)


def ln_bessel_k2(x):
    return lib().orc_ln_bessel_k2(x)


def planck(nu, thetae):
    return lib().orc_planck(nu, thetae)


def closure(nu, ne, thetae, bfield, cos_b, mode=EXACT, const_j=0.0, const_alpha=0.0):
    j, a = C.c_double(), C.c_double()
    lib().orc_closure(mode, nu, ne, thetae, bfield, cos_b, const_j, const_alpha, C.byref(j), C.byref(a))
    return j.value, a.value


def length_unit(mass_msun=4.5e6):
    return lib().orc_length_unit(mass_msun)


def trace_ray(cam, grid_handle, opts, alpha, beta, nu, record=0):
    nu = _f64(nu)
    Iv = np.zeros(nu.size)
    info = RayInfo()
    c = make_camera(cam)
    rec = (StepRec * record)() if record else None
    rc = lib().orc_trace_ray(C.byref(c), C.byref(grid_handle.s), C.byref(opts), alpha, beta, _dp(nu), nu.size,
                             _dp(Iv), C.byref(info), rec, record)
    if rc != 0:
        raise ValueError(f"oracle: n_nu = {nu.size} outside [1, {MAX_NU}]")
    return Iv, info, rec


def trace_pixels(cam, grid_handle, opts, nu, pix, n_threads=0):
    """Intensity [len(pix)][n_nu] and per-ray info (status, steps, samples, poles) arrays."""
    nu = _f64(nu)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    Iv = np.zeros((pix.size, nu.size))
    info = (RayInfo * max(pix.size, 1))()
    c = make_camera(cam)
    rc = lib().orc_trace_pixels(C.byref(c), C.byref(grid_handle.s), C.byref(opts), _dp(nu), nu.size,
                                pix.ctypes.data_as(C.POINTER(C.c_int64)), pix.size, _dp(Iv), info, n_threads)
    if rc != 0:
        raise ValueError(f"oracle: n_nu = {nu.size} outside [1, {MAX_NU}]")
    arr = np.ctypeslib.as_array(info)[: pix.size]
    st = np.array([(r[0], r[1], r[2], r[3]) for r in arr], dtype=np.int64).reshape(-1, 4)
    return Iv, st


def trace_image(cam, grid_handle, opts, nu, n_threads=0):
    """Full image [n_nu][ny][nx], flux [n_nu] (Jy) and per-pixel info [ny*nx][4]."""
    pix = np.arange(cam.nx * cam.ny, dtype=np.int64)
    Iv, st = trace_pixels(cam, grid_handle, opts, nu, pix, n_threads)
    img = Iv.T.reshape(len(np.atleast_1d(nu)), cam.ny, cam.nx)
    flux = flux_jy(cam, opts, img)
    return img, flux, st


def pixel_solid_angle(cam, opts):
    c = make_camera(cam)
    return lib().orc_pixel_solid_angle(C.byref(c), C.byref(opts))


def flux_jy(cam, opts, img):
    """Flux density in Jy: sum of I over pixels times the pixel solid angle."""
    dom = pixel_solid_angle(cam, opts)
    import math
    return np.array([math.fsum(im.ravel()) * dom * 1e23 for im in img])


def forward_transfer(rec, n):
    return lib().orc_forward_transfer(rec, n)


def mlp_param_count():
    return lib().orc_mlp_param_count()


def mlp_forward(params, x):
    params = _f64(params)
    x = _f64(x)
    n = x.size // 3
    y = np.zeros((n, 2))
    lib().orc_mlp_forward(_dp(params), _dp(x), n, _dp(y))
    return y


def mlp_backward(params, x, dy):
    params = _f64(params)
    x = _f64(x)
    dy = _f64(dy)
    n = x.size // 3
    dp = np.zeros(params.size)
    lib().orc_mlp_backward(_dp(params), _dp(x), _dp(dy), n, _dp(dp))
    return dp


# ------------------------------------------------------------------------------------------
# Thin disk (Sec. 4.2.1)
# ------------------------------------------------------------------------------------------

def isco(a):
    return lib().orc_isco(a)


def trace_disk_ray(cam, opts, r_disk_out, alpha, beta):
    """(g, r_cross, I, info) of one ray of the thin-disk test."""
    g, r, I = C.c_double(), C.c_double(), C.c_double()
    info = RayInfo()
    c = make_camera(cam)
    lib().orc_trace_disk_ray(C.byref(c), C.byref(opts), r_disk_out, alpha, beta, C.byref(g), C.byref(r), C.byref(I),
                             C.byref(info))
    return g.value, r.value, I.value, info


def trace_disk_image(cam, opts, r_disk_out=15.0, n_threads=0):
    """(g [ny][nx], I [ny][nx], info [n][4] = status, steps, samples, poles)."""
    n = cam.nx * cam.ny
    g = np.zeros(n)
    I = np.zeros(n)
    info = (RayInfo * n)()
    c = make_camera(cam)
    lib().orc_trace_disk_image(C.byref(c), C.byref(opts), r_disk_out, _dp(g), _dp(I), info, n_threads)
    arr = np.ctypeslib.as_array(info)
    st = np.array([(r[0], r[1], r[2], r[3]) for r in arr], dtype=np.int64).reshape(-1, 4)
    return g.reshape(cam.ny, cam.nx), I.reshape(cam.ny, cam.nx), st


def disk_profile(cam, g, I, n_bins, g_lo, g_hi):
    prof = np.zeros(n_bins)
    c = make_camera(cam)
    lib().orc_disk_profile(C.byref(c), _dp(np.ascontiguousarray(g, dtype=np.float64).ravel()),
                           _dp(np.ascontiguousarray(I, dtype=np.float64).ravel()), n_bins, g_lo, g_hi, _dp(prof))
    return prof
