"""Benchmark of the ray-tracing hot path on one MI355X.

One step = one batched call through the C ABI over the production workload: 9 images of
512 x 512 pixels (spins {0, 0.5, 0.9375} x inclinations {30, 60, 85} deg), camera at
r = 1e4 M with a +-20 M field of view, 230 GHz, on seeded synthetic float32 256 x 256 MKS fluid
grids (one per spin), FP64 geodesics with FP32 transfer (or FP64 with --prec f64), replayed as
a HIP graph (reset, persistent trace kernel, flux reduction).  Inputs are resident in device
memory before timing starts and outputs stay in device memory.

Two forms run on the same GPU: the plain method (exact thermal-synchrotron closure) gives the
headline value; the learned closure (network trained on the device by the library's own
kernels before timing) is reported beside it with its total-flux error against the plain form.
Beside them, each with its own roofline: the spectrum camera (256^2, 24 frequencies, fast and
slow light over 64 snapshots) and the uneven batch (256 images of 64^2..512^2 at four
frequencies, autotuned plan, graph replay, exact and learned closure).  The CPU oracle is timed
on a bounded sample on all host cores and on one.  Prints one JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_sample(sets, oo, threads, budget_s):
    """The oracle over a bounded, strided pixel sample of the workload (chunks of 64 rays per
    image until the time budget is spent): (ray-steps, rays, seconds)."""
    import numpy as np
    from oracle import oracle as O
    import synthetic as S
    handles = {id(g): O.GridHandle(g) for _, g in sets}
    steps = 0
    rays = 0
    t0 = time.perf_counter()
    chunk = 0
    while time.perf_counter() - t0 < budget_s and chunk < 4096:
        for k, (cam, g) in enumerate(sets):
            pix = np.arange(chunk * 97 + k, cam.nx * cam.ny, 4099, dtype=np.int64)[:64]
            _, st = O.trace_pixels(cam, handles[id(g)], oo, [S.NU_230], pix, n_threads=threads)
            steps += int(st[:, 1].sum())
            rays += pix.size
        chunk += 1
    return steps, rays, time.perf_counter() - t0


def progress(msg):
    """One line on stderr per finished part of the run (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(sets, opts_gpu, budget_s=15.0, budget_1core_s=8.0):
    """The oracle on this host's cores, then on one core, over bounded strided pixel samples of
    the same workload: ray-steps per second and the equivalent 512^2 images per second."""
    from oracle import oracle as O
    from tests.gpu_common import oracle_opts
    oo = oracle_opts(O, opts_gpu)
    threads = len(os.sched_getaffinity(0))
    env_threads = os.environ.get("OMP_NUM_THREADS")
    if env_threads and env_threads.isdigit():
        threads = min(threads, int(env_threads))
    steps, rays, dt = oracle_sample(sets, oo, threads, budget_s)
    steps1, rays1, dt1 = oracle_sample(sets, oo, 1, budget_1core_s)
    return {"value": steps / dt, "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{rays} rays ({rays // len(sets)} per image, strided over the 9 images of the "
                      f"workload), {steps} ray-steps in {dt:.1f} s, FP64, 230 GHz",
            "cpu_model": cpu_model(), "rays_per_s": rays / dt, "images_512_per_s": rays / dt / (512 * 512),
            "one_core": {"value": steps1 / dt1, "unit": "ray-steps/s", "cores": 1,
                         "rays_per_s": rays1 / dt1, "images_512_per_s": rays1 / dt1 / (512 * 512),
                         "sample": f"{rays1} rays, {steps1} ray-steps in {dt1:.1f} s"}}


def roofline_of(R, st, kernel_ms, fp64_transfer, n_nu):
    """FP64 vector roofline of a trace launch from its counted work (ray-steps and samples)."""
    w = R.work_per_unit()
    fp64 = st["ray_steps"] * w["step_flops"] + st["samples"] * w["sample_flops"]
    if fp64_transfer:
        fp64 += st["samples"] * n_nu * w["freq_flops"]
    achieved = fp64 / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
            "kernel": "trace_kernel (fused RK4 geodesic + transfer)"}


def time_spectrum(ctx, R, cam, gh, nu, opts, images, flux, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.trace_spectrum(cam, gh, nu, opts, images=images, flux=flux)
    torch.cuda.synchronize()
    profile_mark()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(ctx.trace_spectrum(cam, gh, nu, opts, images=images, flux=flux)[2])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    profile_mark()
    return {"ms": dt * 1e3 / steps, "ray_steps": sum(s.ray_steps for s in stats) / steps,
            "samples": sum(s.samples for s in stats) / steps,
            "kernel_ms": sum(s.kernel_ms for s in stats) / steps}


def spectrum_section(args, R, S, ctx, prec):
    """The spectrum camera: 256^2 pixels, a = 0.9375, i = 60 deg, 24 log-spaced frequencies
    1e9..1e16 Hz on shared geodesics; fast light (the snapshot at the frame time) and slow light
    (64 modulated float32 256^2 snapshots interpolated along each ray); the launch plan chosen by
    the library's autotuner for each form, then graph launch.  With a trained network, the fast-
    light spectrum also with the learned closure, and its flux error against the exact one."""
    import numpy as np
    import torch
    cam, grid, nu = S.slow_light_set()
    gh = ctx.upload_grid(grid)
    images = torch.empty(len(nu) * cam.nx * cam.ny, dtype=torch.float64, device="cuda")
    flux = torch.empty(len(nu), dtype=torch.float64, device="cuda")
    out = {"config": {"workload": "spectrum camera 256x256, a 0.9375, i 60 deg, 24 frequencies 1e9..1e16 Hz, "
                                  "64 float32 256^2 snapshots (m=1..4 modulation, amplitude 0.2), autotuned plan",
                      "n_nu": len(nu)}}
    forms = [("fast_light", 0, R.CLOSURE_EXACT), ("slow_light", 1, R.CLOSURE_EXACT)]
    if args.mlp_ready:
        forms.append(("fast_light_mlp", 0, R.CLOSURE_MLP))
    fluxes = {}
    for name, slow, cl in forms:
        progress(f"spectrum {name}: autotuning, then timing")
        tune = R.default_opts(transfer_prec=prec, slow_light=slow, closure=cl)
        plan, _ = R.autotune_batch(ctx, [cam], [gh], nu, tune, reps=3)   # ~10 ms per trial: best of three
        opts = R.default_opts(transfer_prec=prec, mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH, slow_light=slow,
                              closure=cl)
        r = time_spectrum(ctx, R, cam, gh, nu, opts, images, flux, args.steps, args.warmup)
        fluxes[name] = flux.cpu().numpy().copy()
        out[name] = {"ms_per_step": r["ms"], "kernel_ms": r["kernel_ms"],
                     "value": r["ray_steps"] / (r["ms"] * 1e-3), "unit": "ray-steps/s",
                     "spectra_per_s": 1e3 / r["ms"], "ray_steps_per_step": r["ray_steps"],
                     "samples_per_step": r["samples"], "plan": plan.as_dict(),
                     "roofline": roofline_of(R, r, r["kernel_ms"], prec == R.F64, len(nu))}
    if "fast_light_mlp" in fluxes:
        ex = fluxes["fast_light"]
        rel = np.abs(fluxes["fast_light_mlp"] / np.where(ex != 0, ex, 1.0) - 1.0)
        out["fast_light_mlp"]["max_rel_flux_err_vs_exact"] = float(rel.max())
        out["fast_light_mlp"]["rel_flux_err_per_frequency"] = [float(x) for x in rel]
        out["fast_light"]["flux_jy"] = [float(x) for x in ex]
        out["fast_light_mlp"]["time_vs_exact"] = out["fast_light_mlp"]["kernel_ms"] / out["fast_light"]["kernel_ms"]
    ctx.release_grid(gh)
    return out


def uneven_batch_section(args, R, S, ctx, prec):
    """The uneven batch: 256 images of 64^2..512^2 (seeded), spin U(-0.99, 0.99), inclination
    U(5, 85) deg, the four VLBI frequencies, one shared float32 256^2 grid; the launch plan chosen
    by the library's autotuner on this batch, then graph replay; exact closure and, when the
    network is trained, the learned closure with its flux error against the exact one."""
    import numpy as np
    import torch
    cams = S.batch_jobs()
    grid = S.make_grid(256, 256, a_gen=0.9375, dtype=np.float32)
    gh = ctx.upload_grid(grid)
    grids = [gh] * len(cams)
    nu = S.NU_VLBI
    n_pix = sum(c.nx * c.ny for c in cams)
    images = torch.empty(n_pix * len(nu), dtype=torch.float64, device="cuda")
    flux = torch.empty((len(cams), len(nu)), dtype=torch.float64, device="cuda")
    out = {"config": {"workload": "256 images (res uniform over {64,128,256,512}^2, a U(-0.99,0.99), "
                                  "i U(5,85) deg), 22/43/86/230 GHz, shared float32 256^2 grid, "
                                  "autotuned plan, graph launch",
                      "images_per_step": len(cams), "rays_per_step": n_pix,
                      "images_512_equiv_per_step": n_pix / (512 * 512)}}
    forms = [("exact", R.CLOSURE_EXACT)]
    if args.mlp_ready:
        forms.append(("mlp", R.CLOSURE_MLP))
    fluxes = {}
    for name, cl in forms:
        progress(f"uneven batch {name}: autotuning, then timing")
        tune = R.default_opts(transfer_prec=prec, closure=cl)
        t0 = time.perf_counter()
        plan, tuned_ms = R.autotune_batch(ctx, cams, grids, nu, tune, reps=1)
        tune_s = time.perf_counter() - t0
        opts = R.default_opts(transfer_prec=prec, mem=R.MEM_DEVICE, launch=R.LAUNCH_GRAPH, closure=cl)
        r = time_form(ctx, R, cams, grids, nu, opts, images, flux, args.steps, args.warmup)
        fluxes[name] = r["flux"]
        out[name] = {"ms_per_step": r["ms"], "kernel_ms": r["kernel_ms"],
                     "value": r["ray_steps"] / (r["ms"] * 1e-3), "unit": "ray-steps/s",
                     "images_per_s": len(cams) / (r["ms"] * 1e-3),
                     "images_512_per_s": n_pix / (512 * 512) / (r["ms"] * 1e-3),
                     "ray_steps_per_step": r["ray_steps"], "samples_per_step": r["samples"],
                     "plan": plan.as_dict(), "autotune_s": tune_s,
                     "roofline": roofline_of(R, r, r["kernel_ms"], prec == R.F64, len(nu))}
        if name == "mlp":
            out[name]["exact_fallback_fraction"] = r["fallback"] / max(r["samples"] * len(nu), 1.0)
            out[name]["dropped_exact_zero_fraction"] = r["dropped"] / max(r["samples"] * len(nu), 1.0)
    if "mlp" in fluxes:
        rel = fluxes["mlp"] / fluxes["exact"] - 1.0
        out["mlp"]["max_abs_flux_rel_err"] = float(np.abs(rel).max())
    ctx.release_grid(gh)
    return out


_MARK = []


def profile_mark():
    """One one-element fill kernel on the current stream: in a kernel trace of this script, the
    launches of each timed region lie between two of these (the autotuner's trial launches,
    which carry the same kernel names, lie outside)."""
    import torch
    if not _MARK:
        _MARK.append(torch.empty(1, dtype=torch.float32, device="cuda"))
    _MARK[0].fill_(float(len(_MARK)))
    _MARK.append(None)


def time_form(ctx, R, cams, grids, nu, opts, images, flux, steps, warmup):
    import torch

    def step():
        return ctx.trace_batch(cams, grids, nu, opts, images=images, flux=flux)[2]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    profile_mark()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    profile_mark()
    return {"ms": dt * 1e3 / steps,
            "ray_steps": sum(s.ray_steps for s in stats) / steps,
            "samples": sum(s.samples for s in stats) / steps,
            "fallback": sum(s.n_mlp_fallback for s in stats) / steps,
            "dropped": sum(s.n_mlp_dropped for s in stats) / steps,
            "kernel_ms": sum(s.kernel_ms for s in stats) / steps,
            "kernel_ms_median": statistics.median(s.kernel_ms for s in stats),
            "flux": flux.detach().cpu().numpy().ravel().copy()}


def spectrum_slow_light(args):
    """The slow-light spectrum: 256^2 pixels, 24 frequencies, 64 modulated float32 snapshots;
    prints one JSON line (kernel time, ray-steps/s and the grid bytes the samples gather)."""
    import torch
    import synthetic as S
    from paper_1801_10452_amd import raptor as R
    cam, grid, nu = S.slow_light_set()
    ctx = R.Context(0, use_torch_stream=True)
    gh = ctx.upload_grid(grid)
    opts = R.default_opts(transfer_prec=R.F32, slow_light=1)
    plan, _ = R.autotune_batch(ctx, [cam], [gh], nu, opts, reps=1)   # the plan the benchmark times
    for _ in range(args.warmup):
        ctx.trace_spectrum(cam, gh, nu, opts)
    ms, st = [], None
    for _ in range(args.steps):
        _, _, st = ctx.trace_spectrum(cam, gh, nu, opts)
        ms.append(st.kernel_ms)
    k = sum(ms) / len(ms)
    # two snapshots x four cells x 16 bytes per sample
    gather = st.samples * 2 * 4 * 16
    print(json.dumps({"workload": "spectrum 256x256, 24 frequencies, slow light (64 float32 256^2 snapshots)",
                      "plan": plan.as_dict(), "kernel_ms": k, "ray_steps": st.ray_steps, "samples": st.samples,
                      "ray_steps_per_s": st.ray_steps / k * 1e3, "gather_bytes_per_launch": gather,
                      "gather_GBps": gather / k * 1e-6, "grid_bytes": int(grid.cells.nbytes)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--launch", choices=["graph", "direct"], default="graph")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-closure form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "trace_kernel_traffic.json"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy 3 times (HBM counter calibration)")
    ap.add_argument("--mlp-epochs", type=int, default=0,
                    help="training epochs of the network (0: the library default); fewer only for profiling the "
                         "learned-closure kernel, whose cost does not depend on the weights")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the spectrum camera and the uneven 256-image batch")
    ap.add_argument("--spectrum-slow-light", action="store_true",
                    help="only time the 256^2 x 24-frequency slow-light spectrum (64 snapshots, 64 MiB of grids): "
                         "the workload whose grid gathers can reach HBM, for the memory counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: the library shards nothing across GPUs"}))
        sys.exit(2)
    if args.spectrum_slow_light:
        spectrum_slow_light(args)
        return

    import numpy as np
    import torch
    import synthetic as S
    from paper_1801_10452_amd import raptor as R

    sets = S.production_set(res=args.res)
    cams = [c for c, _ in sets]
    ctx = R.Context(0, use_torch_stream=True)
    handles, grids = {}, []
    for c, g in sets:
        if id(g) not in handles:
            handles[id(g)] = ctx.upload_grid(g)
        grids.append(handles[id(g)])
    prec = R.F32 if args.prec == "f32" else R.F64
    launch = R.LAUNCH_GRAPH if args.launch == "graph" else R.LAUNCH_DIRECT
    n_pix = sum(c.nx * c.ny for c in cams)
    images = torch.empty(n_pix, dtype=torch.float64, device="cuda")
    flux = torch.empty((len(cams), 1), dtype=torch.float64, device="cuda")
    nu = [S.NU_230]
    torch.cuda.synchronize()

    progress("production batch: timing the exact closure")
    plain = time_form(ctx, R, cams, grids, nu, R.default_opts(transfer_prec=prec, mem=R.MEM_DEVICE, launch=launch),
                      images, flux, args.steps, args.warmup)
    ms = plain["ms"]
    w = R.work_per_unit()
    fp64_flops = plain["ray_steps"] * w["step_flops"] + plain["samples"] * w["sample_flops"]
    if args.prec == "f64":
        fp64_flops += plain["samples"] * w["freq_flops"]
    achieved = fp64_flops / (plain["kernel_ms"] * 1e-3) / 1e12
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("prec") == args.prec and tj.get("res") == args.res and tj.get("kernel_build") == R.kernel_build_id():
            traffic = tj.get("bytes_per_launch")
    out = {
        "metric": "ray-steps/sec and 512^2 images/sec, plain vs MLP-emissivity at <=1e-3 flux err",
        "value": plain["ray_steps"] / (ms * 1e-3),
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "f64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"9 images {args.res}x{args.res} (a in {{0,0.5,0.9375}} x i in {{30,60,85}} deg), "
                               f"r_cam 1e4 M, FOV +-20 M, 230 GHz, float32 256^2 MKS grids, RK4 eps 0.05, "
                               f"FP64 geodesic + {args.prec.upper()} transfer, exact closure, {args.launch} launch",
                   "closure": "exact", "images_per_step": len(cams), "rays_per_step": n_pix},
        "images_per_s": len(cams) / (ms * 1e-3),
        "images_512_per_s": len(cams) * (args.res * args.res) / (512 * 512) / (ms * 1e-3),
        "ray_steps_per_step": plain["ray_steps"],
        "samples_per_step": plain["samples"],
        "kernel_ms": plain["kernel_ms"],
        "kernel_ms_median": plain["kernel_ms_median"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "trace_kernel (fused RK4 geodesic + transfer)",
                     "flops_per_ray_step": w["step_flops"], "flops_per_sample": w["sample_flops"]},
    }
    args.mlp_ready = False
    if not args.no_mlp:
        R.mlp_init(ctx)
        cfg = R.mlp_default_cfg()
        if args.mlp_epochs > 0:
            cfg.epochs = args.mlp_epochs
        progress("training the learned closure")
        rep = R.mlp_train(ctx, cfg)
        progress(f"trained in {rep.train_ms / 1e3:.1f} s; timing the production batch with the network")
        mlp = time_form(ctx, R, cams, grids, nu,
                        R.default_opts(transfer_prec=prec, mem=R.MEM_DEVICE, launch=launch, closure=R.CLOSURE_MLP),
                        images, flux, args.steps, args.warmup)
        rel = mlp["flux"] / plain["flux"] - 1.0
        out["mlp"] = {"value": mlp["ray_steps"] / (mlp["ms"] * 1e-3), "unit": "ray-steps/s",
                      "ms_per_step": mlp["ms"], "kernel_ms": mlp["kernel_ms"],
                      "images_512_per_s": len(cams) * (args.res * args.res) / (512 * 512) / (mlp["ms"] * 1e-3),
                      "max_abs_flux_rel_err": float(np.abs(rel).max()),
                      "flux_rel_err_per_image": [float(x) for x in rel],
                      "exact_fallback_fraction": mlp["fallback"] / max(mlp["samples"], 1.0),
                      "dropped_exact_zero_fraction": mlp["dropped"] / max(mlp["samples"], 1.0),
                      "form": "split BF16 MFMA, FP32 accumulate",
                      "training": {"steps": rep.steps, "train_ms": rep.train_ms,
                                   "val_rms_ln_j": rep.val_rms[0], "val_rms_ln_alpha": rep.val_rms[1]}}
        args.mlp_ready = True
    if not args.no_extra:
        progress("spectrum camera")
        out["spectrum"] = spectrum_section(args, R, S, ctx, prec)
        progress("uneven batch")
        out["uneven_batch"] = uneven_batch_section(args, R, S, ctx, prec)
    if not args.no_cpu_baseline:
        progress("CPU baseline (the oracle)")
        out["cpu_baseline"] = cpu_baseline(sets, R.default_opts(transfer_prec=prec))
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
