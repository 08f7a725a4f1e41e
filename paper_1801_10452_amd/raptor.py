"""Thin ctypes binding of libraptor_hip.so (the C ABI of include/raptor.h).

Argument marshalling only: every step of the ray-tracing path runs in the HIP library.
Output buffers are numpy arrays (host mode) or torch CUDA tensors (device mode); torch
provides device memory and the current stream.  The binding refuses to run without the
compiled library -- there is no fallback path.
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libraptor_hip.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_RANGE = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
CLOSURE_EXACT, CLOSURE_K2_PAPER, CLOSURE_CONST, CLOSURE_MLP, CLOSURE_MLP_BF16 = 0, 1, 2, 3, 4
MLP_SPLIT, MLP_BF16, MLP_F32 = 0, 1, 2
LAUNCH_DIRECT, LAUNCH_GRAPH = 0, 1
UNITS_CGS, UNITS_CODE = 0, 1
RK4, RK2, VERLET, VERLET_CORRECTED = 0, 1, 2, 3
MLP_PARAMS = 12866
RAY_HORIZON, RAY_ESCAPED, RAY_MAXSTEP, RAY_NUMERIC = 1, 2, 3, 4
MAX_NU = 32
RAPTOR_NOALLOC_MAX_CAMS = 256

DP = C.POINTER(C.c_double)
IP = C.POINTER(C.c_int32)


class RaptorError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"raptor status {status}: {msg}")
        self.status = status


class CCamera(C.Structure):
    _fields_ = [("spin", C.c_double), ("incl_deg", C.c_double), ("r_cam", C.c_double), ("fov_half", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("t_frame", C.c_double)]


class CGridDesc(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n_snap", C.c_int32), ("dtype", C.c_int32),
                ("r_in", C.c_double), ("r_out", C.c_double), ("hslope", C.c_double), ("a_gen", C.c_double),
                ("t0", C.c_double), ("dt_snap", C.c_double), ("mod_amp", C.c_double), ("mod_phase", C.c_double * 4),
                ("cells", C.c_void_p), ("units", C.c_int32), ("reserved", C.c_int32),
                ("mass_unit_g", C.c_double), ("r_low", C.c_double), ("r_high", C.c_double), ("gamma_ad", C.c_double)]


class COpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("r_stop_factor", C.c_double), ("max_steps", C.c_int32),
                ("transfer_prec", C.c_int32), ("closure", C.c_int32), ("slow_light", C.c_int32), ("mem", C.c_int32),
                ("launch", C.c_int32), ("mass_msun", C.c_double), ("dist_pc", C.c_double),
                ("const_j", C.c_double), ("const_alpha", C.c_double), ("metric_mass", C.c_double),
                ("integrator", C.c_int32), ("reserved", C.c_int32), ("tau_cutoff", C.c_double),
                ("tau_step", C.c_double)]


class CStats(C.Structure):
    _fields_ = [("rays", C.c_uint64), ("ray_steps", C.c_uint64), ("samples", C.c_uint64),
                ("n_horizon", C.c_uint64), ("n_escaped", C.c_uint64), ("n_maxstep", C.c_uint64),
                ("n_pole", C.c_uint64), ("n_numeric", C.c_uint64), ("n_mlp_fallback", C.c_uint64),
                ("n_zamo_fallback", C.c_uint64), ("kernel_ms", C.c_double), ("n_opaque", C.c_uint64),
                ("n_mlp_dropped", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CPlan(C.Structure):
    _fields_ = [("threads", C.c_int32), ("blocks_per_cu", C.c_int32), ("refill_threshold", C.c_int32),
                ("tile_width", C.c_int32), ("min_waves_per_simd", C.c_int32), ("rays_per_wave", C.c_int32),
                ("reserved", C.c_int32 * 2)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CMlpCfg(C.Structure):
    _fields_ = [("n_train", C.c_int64), ("n_val", C.c_int64), ("epochs", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_float), ("lr_final", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("adam_eps", C.c_float), ("weight_decay", C.c_float), ("train_seed", C.c_uint64),
                ("val_seed", C.c_uint64), ("form", C.c_int32), ("reserved", C.c_int32)]


class CMlpReport(C.Structure):
    _fields_ = [("steps", C.c_int64), ("train_loss", C.c_double), ("val_rms", C.c_double * 2),
                ("val_max", C.c_double * 2), ("val_rms_bright", C.c_double), ("train_ms", C.c_double)]

    def as_dict(self):
        return {"steps": self.steps, "train_loss": self.train_loss, "val_rms": list(self.val_rms),
                "val_max": list(self.val_max), "val_rms_bright": self.val_rms_bright, "train_ms": self.train_ms}


# every symbol include/raptor.h declares
EXPORTS = ["raptor_create", "raptor_destroy", "raptor_last_error", "raptor_grid_upload", "raptor_grid_release",
           "raptor_default_opts", "raptor_trace_image", "raptor_trace_spectrum", "raptor_trace_spectrum_ex",
           "raptor_trace_batch", "raptor_trace_batch_noalloc", "raptor_work_per_unit", "raptor_work_per_step", "raptor_get_plan", "raptor_set_plan",
           "raptor_isco", "raptor_trace_disk",
           "raptor_autotune_batch", "raptor_kernel_info", "raptor_mlp_default_cfg", "raptor_mlp_init",
           "raptor_mlp_train", "raptor_mlp_get_params", "raptor_mlp_set_params", "raptor_mlp_get_weights",
           "raptor_mlp_set_weights", "raptor_mlp_forward", "raptor_mlp_backward", "raptor_mlp_closure"]

_lib = None


def lib():
    """Load the compiled HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1801_10452_amd/build.py "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        # torch carries its own HIP runtime (SONAME libamdhip64.so.7).  Loading it first makes
        # the dynamic loader resolve this library's HIP dependency to that same runtime, so a
        # process holds one HIP runtime and torch's streams and pointers are valid here.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        L.raptor_create.argtypes = [C.c_int, V, C.POINTER(V)]
        L.raptor_destroy.argtypes = [V]
        L.raptor_destroy.restype = None
        L.raptor_last_error.argtypes = [V]
        L.raptor_last_error.restype = C.c_char_p
        L.raptor_grid_upload.argtypes = [V, C.POINTER(CGridDesc), C.POINTER(V)]
        L.raptor_grid_release.argtypes = [V, V]
        L.raptor_grid_release.restype = None
        L.raptor_default_opts.argtypes = [C.POINTER(COpts)]
        L.raptor_trace_image.argtypes = [V, C.POINTER(CCamera), V, C.POINTER(COpts), C.c_double, V, V,
                                         C.POINTER(CStats)]
        L.raptor_trace_spectrum.argtypes = [V, C.POINTER(CCamera), V, C.POINTER(COpts), DP, C.c_int32, V, V,
                                            C.POINTER(CStats)]
        L.raptor_trace_spectrum_ex.argtypes = [V, C.POINTER(CCamera), V, C.POINTER(COpts), DP, C.c_int32, V, V, V,
                                               V, C.POINTER(CStats)]
        L.raptor_trace_batch.argtypes = [V, C.POINTER(CCamera), C.c_int32, C.POINTER(V), C.POINTER(COpts), DP,
                                         C.c_int32, V, V, C.POINTER(CStats)]
        L.raptor_trace_batch_noalloc.argtypes = [V, C.POINTER(CCamera), C.c_int32, C.POINTER(V), C.POINTER(COpts),
                                                 DP, C.c_int32, V, V, C.POINTER(CStats)]
        L.raptor_work_per_unit.argtypes = [DP] * 6
        L.raptor_work_per_step.argtypes = [C.c_int32, DP, DP]
        L.raptor_isco.argtypes = [C.c_double, DP]
        L.raptor_trace_disk.argtypes = [V, C.POINTER(CCamera), C.POINTER(COpts), C.c_double, C.c_int32, C.c_double,
                                        C.c_double, V, V, V, V, V, C.POINTER(CStats)]
        L.raptor_get_plan.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, C.POINTER(CPlan)]
        L.raptor_set_plan.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, C.POINTER(CPlan)]
        L.raptor_autotune_batch.argtypes = [V, C.POINTER(CCamera), C.c_int32, C.POINTER(V), C.POINTER(COpts), DP,
                                            C.c_int32, C.c_int32, C.POINTER(CPlan), DP]
        L.raptor_kernel_info.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, C.POINTER(CPlan), IP, IP, IP]
        FP = C.POINTER(C.c_float)
        L.raptor_mlp_default_cfg.argtypes = [C.POINTER(CMlpCfg)]
        L.raptor_mlp_init.argtypes = [V, C.c_uint64]
        L.raptor_mlp_train.argtypes = [V, C.POINTER(CMlpCfg), C.POINTER(CMlpReport)]
        L.raptor_mlp_get_params.argtypes = [V, FP, C.c_int32]
        L.raptor_mlp_set_params.argtypes = [V, FP, C.c_int32]
        L.raptor_mlp_get_weights.argtypes = [V, V, C.POINTER(C.c_size_t)]
        L.raptor_mlp_set_weights.argtypes = [V, V, C.c_size_t]
        L.raptor_mlp_forward.argtypes = [V, C.c_int32, FP, C.c_int64, FP]
        L.raptor_mlp_backward.argtypes = [V, C.c_int32, FP, FP, C.c_int64, FP]
        L.raptor_mlp_closure.argtypes = [V, C.c_int32, FP, C.c_int64, FP, FP]
        for name in EXPORTS:
            if name not in ("raptor_destroy", "raptor_last_error", "raptor_grid_release"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def default_opts(**kw) -> COpts:
    o = COpts()
    lib().raptor_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_camera(cam) -> CCamera:
    return CCamera(cam.spin, cam.incl_deg, cam.r_cam, cam.fov_half, cam.nx, cam.ny, cam.t_frame)


TRACE_KERNEL_SOURCES = ("trace.hip", "ks_geodesic.hpp", "plasma.hpp", "rt_math.hpp", "device_types.hpp",
                        "mlp_device.hpp")


def kernel_build_id():
    """A digest of the sources the trace kernel is compiled from: measurements tied to one
    kernel build (hardware counters) carry it, so that they are not reused after a change."""
    import hashlib
    h = hashlib.sha256()
    for name in TRACE_KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def isco(spin):
    v = C.c_double()
    st = lib().raptor_isco(spin, C.byref(v))
    if st != 0:
        raise RaptorError(st, "spin out of range")
    return v.value


def work_per_step(integrator=RK4):
    """(FP64 flops, special ops) of one accepted step of the integrator."""
    v = [C.c_double() for _ in range(2)]
    st = lib().raptor_work_per_step(integrator, C.byref(v[0]), C.byref(v[1]))
    if st != 0:
        raise RaptorError(st, "bad integrator")
    return v[0].value, v[1].value


def work_per_unit():
    v = [C.c_double() for _ in range(6)]
    lib().raptor_work_per_unit(*[C.byref(x) for x in v])
    keys = ["step_flops", "step_special", "sample_flops", "sample_special", "freq_flops", "freq_special"]
    return {k: x.value for k, x in zip(keys, v)}


def _out(a, n, kind, mem, device, name):
    """Check a caller-supplied output buffer before its address is handed to the library: in
    host mode a C-contiguous numpy array, in device mode a contiguous torch tensor on the
    context's device; dtype float64 (kind "f8") or int32 ("i4"); at least n elements.  Raises
    RaptorError(E_INVALID) on a mismatch.  Returns the address (None for None)."""
    if a is None:
        return None
    if mem == MEM_HOST:
        if not isinstance(a, np.ndarray):
            raise RaptorError(E_INVALID, f"{name}: host mode needs a numpy array, got {type(a).__name__}")
        if a.dtype != np.dtype(kind) or not a.flags.c_contiguous or not a.flags.writeable:
            raise RaptorError(E_INVALID, f"{name}: needs a writeable C-contiguous {np.dtype(kind)} array, "
                                         f"got {a.dtype} (contiguous={a.flags.c_contiguous})")
        if a.size < n:
            raise RaptorError(E_INVALID, f"{name}: {a.size} elements, {n} needed")
        return a.ctypes.data
    import torch
    if not isinstance(a, torch.Tensor):
        raise RaptorError(E_INVALID, f"{name}: device mode needs a torch tensor, got {type(a).__name__}")
    want = torch.float64 if kind == "f8" else torch.int32
    if a.dtype != want or not a.is_contiguous():
        raise RaptorError(E_INVALID, f"{name}: needs a contiguous {want} tensor, got {a.dtype}")
    if not a.is_cuda or (a.device.index if a.device.index is not None else 0) != device:
        raise RaptorError(E_INVALID, f"{name}: tensor on {a.device}, the context is on cuda:{device}")
    if a.numel() < n:
        raise RaptorError(E_INVALID, f"{name}: {a.numel()} elements, {n} needed")
    return a.data_ptr()


@dataclass
class GridHandle:
    ptr: int
    ctx: "Context"


class Context:
    """A raptor context on one HIP device.  stream: a hipStream_t as int (None: the context's own
    stream, or torch's current stream when use_torch_stream=True)."""

    def __init__(self, device=0, stream=None, use_torch_stream=False):
        if use_torch_stream:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        st = lib().raptor_create(device, C.c_void_p(stream) if stream else None, C.byref(h))
        if st != OK:
            raise RaptorError(st, lib().raptor_last_error(None).decode())
        self.h = h
        self.device = device
        self._grids = []

    def close(self):
        if self.h:
            lib().raptor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise RaptorError(st, lib().raptor_last_error(self.h).decode())

    def upload_grid(self, g) -> GridHandle:
        cells = np.ascontiguousarray(g.cells)
        d = CGridDesc(g.n1, g.n2, g.n_snap, F64 if cells.dtype == np.float64 else F32, g.r_in, g.r_out, g.hslope,
                      g.a_gen, g.t0, g.dt_snap, g.mod_amp, (C.c_double * 4)(*g.mod_phase), cells.ctypes.data,
                      getattr(g, "units", UNITS_CGS), 0, getattr(g, "mass_unit_g", 0.0), getattr(g, "r_low", 1.0),
                      getattr(g, "r_high", 1.0), getattr(g, "gamma_ad", 13.0 / 9.0))
        h = C.c_void_p()
        self._check(lib().raptor_grid_upload(self.h, C.byref(d), C.byref(h)))
        gh = GridHandle(h.value, self)
        self._grids.append(gh)
        return gh

    def release_grid(self, gh: GridHandle):
        lib().raptor_grid_release(self.h, C.c_void_p(gh.ptr))

    def trace_spectrum(self, cam, grid, nu, opts=None, images=None, flux=None, ray_status=None, ray_steps=None):
        """Trace one image at the frequencies nu.  In host mode (opts.mem == MEM_HOST) outputs
        are numpy arrays allocated here when not given; in device mode pass torch tensors.
        Returns (images, flux, stats) with images [n_nu][ny][nx]."""
        opts = opts or default_opts()
        nu = np.ascontiguousarray(np.atleast_1d(nu), dtype=np.float64)
        if opts.mem == MEM_HOST:
            if images is None:
                images = np.zeros((nu.size, cam.ny, cam.nx))
            if flux is None:
                flux = np.zeros(nu.size)
        st = CStats()
        c = make_camera(cam)
        npix, m, d = cam.nx * cam.ny, opts.mem, self.device
        args = (_out(images, nu.size * npix, "f8", m, d, "images"), _out(flux, nu.size, "f8", m, d, "flux"),
                _out(ray_status, npix, "i4", m, d, "ray_status"), _out(ray_steps, npix, "i4", m, d, "ray_steps"))
        self._check(lib().raptor_trace_spectrum_ex(self.h, C.byref(c), C.c_void_p(grid.ptr), C.byref(opts),
                                                   nu.ctypes.data_as(DP), nu.size, *args, C.byref(st)))
        return images, flux, st

    def trace_image(self, cam, grid, nu, opts=None, image=None, flux=None):
        opts = opts or default_opts()
        if opts.mem == MEM_HOST:
            if image is None:
                image = np.zeros((cam.ny, cam.nx))
            if flux is None:
                flux = np.zeros(1)
        st = CStats()
        c = make_camera(cam)
        npix, m, d = cam.nx * cam.ny, opts.mem, self.device
        self._check(lib().raptor_trace_image(self.h, C.byref(c), C.c_void_p(grid.ptr), C.byref(opts), float(nu),
                                             _out(image, npix, "f8", m, d, "image"), _out(flux, 1, "f8", m, d, "flux"),
                                             C.byref(st)))
        return image, flux, st

    def trace_disk(self, cam, opts=None, r_disk_out=15.0, n_bins=256, g_lo=0.0, g_hi=2.0, intensity=None,
                   redshift=None, profile=None, ray_status=None, ray_steps=None):
        """Thin-disk line test.  Returns (intensity [ny][nx], redshift [ny][nx], profile [n_bins],
        stats); in host mode arrays are allocated here when not given."""
        opts = opts or default_opts()
        if opts.mem == MEM_HOST:
            if intensity is None:
                intensity = np.zeros((cam.ny, cam.nx))
            if redshift is None:
                redshift = np.zeros((cam.ny, cam.nx))
            if profile is None and n_bins > 0:
                profile = np.zeros(n_bins)
        st = CStats()
        c = make_camera(cam)
        npix, m, d = cam.nx * cam.ny, opts.mem, self.device
        self._check(lib().raptor_trace_disk(self.h, C.byref(c), C.byref(opts), r_disk_out, n_bins, g_lo, g_hi,
                                            _out(intensity, npix, "f8", m, d, "intensity"),
                                            _out(redshift, npix, "f8", m, d, "redshift"),
                                            _out(profile, max(n_bins, 0), "f8", m, d, "profile"),
                                            _out(ray_status, npix, "i4", m, d, "ray_status"),
                                            _out(ray_steps, npix, "i4", m, d, "ray_steps"), C.byref(st)))
        return intensity, redshift, profile, st

    def trace_batch(self, cams, grids, nu, opts=None, images=None, flux=None):
        """cams: list of cameras; grids: one GridHandle per camera; nu: [n_cams][n_nu] (or one
        list used for every camera).  images: all images concatenated, flux [n_cams][n_nu]."""
        opts = opts or default_opts()
        n = len(cams)
        nu = np.asarray(nu, dtype=np.float64)
        if nu.ndim == 1:
            nu = np.tile(nu, (n, 1))
        nu = np.ascontiguousarray(nu)
        n_nu = nu.shape[1]
        total = sum(c.nx * c.ny for c in cams) * n_nu
        if opts.mem == MEM_HOST:
            if images is None:
                images = np.zeros(total)
            if flux is None:
                flux = np.zeros((n, n_nu))
        carr = (CCamera * n)(*[make_camera(c) for c in cams])
        garr = (C.c_void_p * n)(*[g.ptr for g in grids])
        st = CStats()
        m, d = opts.mem, self.device
        self._check(lib().raptor_trace_batch(self.h, carr, n, garr, C.byref(opts), nu.ctypes.data_as(DP), n_nu,
                                             _out(images, total, "f8", m, d, "images"),
                                             _out(flux, n * n_nu, "f8", m, d, "flux"), C.byref(st)))
        return images, flux, st


def trace_batch_noalloc(ctx, cams, grids, nu, opts, images, flux=None):
    """raptor_trace_batch_noalloc: as Context.trace_batch with device outputs (opts.mem =
    MEM_DEVICE, images a CUDA tensor of all images concatenated, flux a CUDA tensor or None);
    the call allocates nothing.  Returns the stats."""
    n, nu, carr, garr = _batch_args(cams, grids, nu)
    n_nu = nu.shape[1]
    total = sum(c.nx * c.ny for c in cams) * n_nu
    m, d = opts.mem, ctx.device
    st = CStats()
    ctx._check(lib().raptor_trace_batch_noalloc(ctx.h, carr, n, garr, C.byref(opts), nu.ctypes.data_as(DP), n_nu,
                                                _out(images, total, "f8", m, d, "images"),
                                                _out(flux, n * n_nu, "f8", m, d, "flux"), C.byref(st)))
    return st


def make_plan(threads=256, blocks_per_cu=0, refill_threshold=1, tile_width=8, min_waves_per_simd=2,
              rays_per_wave=64) -> CPlan:
    return CPlan(threads, blocks_per_cu, refill_threshold, tile_width, min_waves_per_simd, rays_per_wave,
                 (C.c_int32 * 2)())


def _batch_args(cams, grids, nu):
    n = len(cams)
    nu = np.asarray(nu, dtype=np.float64)
    if nu.ndim == 1:
        nu = np.tile(nu, (n, 1))
    nu = np.ascontiguousarray(nu)
    carr = (CCamera * n)(*[make_camera(c) for c in cams])
    garr = (C.c_void_p * n)(*[g.ptr for g in grids])
    return n, nu, carr, garr


def get_plan(ctx, n_nu, prec, closure=CLOSURE_EXACT):
    pl = CPlan()
    ctx._check(lib().raptor_get_plan(ctx.h, n_nu, prec, closure, C.byref(pl)))
    return pl


def set_plan(ctx, n_nu, prec, plan, closure=CLOSURE_EXACT):
    ctx._check(lib().raptor_set_plan(ctx.h, n_nu, prec, closure, C.byref(plan)))


def autotune_batch(ctx, cams, grids, nu, opts=None, reps=2):
    """Run the library's autotuner on this batch; returns (best plan, best kernel ms)."""
    opts = opts or default_opts()
    n, nu, carr, garr = _batch_args(cams, grids, nu)
    best = CPlan()
    ms = C.c_double()
    ctx._check(lib().raptor_autotune_batch(ctx.h, carr, n, garr, C.byref(opts), nu.ctypes.data_as(DP), nu.shape[1],
                                           reps, C.byref(best), C.byref(ms)))
    return best, ms.value


def kernel_info(ctx, n_nu, prec, plan, closure=CLOSURE_EXACT):
    v = [C.c_int32() for _ in range(3)]
    ctx._check(lib().raptor_kernel_info(ctx.h, n_nu, prec, closure, C.byref(plan), *[C.byref(x) for x in v]))
    return {"vgprs": v[0].value, "scratch_bytes": v[1].value, "blocks_per_cu": v[2].value}


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def mlp_default_cfg(**kw) -> CMlpCfg:
    c = CMlpCfg()
    lib().raptor_mlp_default_cfg(C.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def mlp_init(ctx, seed=1801104520 + 102):
    ctx._check(lib().raptor_mlp_init(ctx.h, seed))


def mlp_train(ctx, cfg=None):
    cfg = cfg or mlp_default_cfg()
    rep = CMlpReport()
    ctx._check(lib().raptor_mlp_train(ctx.h, C.byref(cfg), C.byref(rep)))
    return rep


def mlp_get_params(ctx):
    out = np.zeros(MLP_PARAMS, dtype=np.float32)
    ctx._check(lib().raptor_mlp_get_params(ctx.h, _fp(out), MLP_PARAMS))
    return out


def mlp_set_params(ctx, params):
    params = np.ascontiguousarray(params, dtype=np.float32)
    ctx._check(lib().raptor_mlp_set_params(ctx.h, _fp(params), params.size))


def mlp_get_weights(ctx) -> bytes:
    n = C.c_size_t(0)
    ctx._check(lib().raptor_mlp_get_weights(ctx.h, None, C.byref(n)))
    buf = (C.c_char * n.value)()
    ctx._check(lib().raptor_mlp_get_weights(ctx.h, buf, C.byref(n)))
    return bytes(buf)


def mlp_set_weights(ctx, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    ctx._check(lib().raptor_mlp_set_weights(ctx.h, buf, len(blob)))


def mlp_forward(ctx, x, form=MLP_SPLIT):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
    y = np.zeros((x.shape[0], 2), dtype=np.float32)
    ctx._check(lib().raptor_mlp_forward(ctx.h, form, _fp(x), x.shape[0], _fp(y)))
    return y


def mlp_backward(ctx, x, dy, form=MLP_BF16):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
    dy = np.ascontiguousarray(dy, dtype=np.float32).reshape(-1, 2)
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    ctx._check(lib().raptor_mlp_backward(ctx.h, form, _fp(x), _fp(dy), x.shape[0], _fp(g)))
    return g


def mlp_closure(ctx, raw, form=MLP_SPLIT, net=True, exact=True):
    """(network, exact) (ln j_hat, ln alpha_hat) for raw inputs (ln(nu/nu_c), ln Theta_e, cos)."""
    raw = np.ascontiguousarray(raw, dtype=np.float32).reshape(-1, 3)
    n = raw.shape[0]
    out_n = np.zeros((n, 2), dtype=np.float32) if net else None
    out_e = np.zeros((n, 2), dtype=np.float32) if exact else None
    ctx._check(lib().raptor_mlp_closure(ctx.h, form, _fp(raw), n, _fp(out_n) if net else None,
                                        _fp(out_e) if exact else None))
    return out_n, out_e


def split_batch_images(images, cams, n_nu):
    """View the concatenated batch output as a list of [n_nu][ny][nx] arrays."""
    out, o = [], 0
    for c in cams:
        n = n_nu * c.nx * c.ny
        out.append(images[o:o + n].reshape(n_nu, c.ny, c.nx))
        o += n
    return out
