"""Benchmark of the ray-tracing hot path on one MI355X.

One step = one persistent batched launch that traces the production workload through the C
ABI: 9 images of 512 x 512 pixels (spins {0, 0.5, 0.9375} x inclinations {30, 60, 85} deg),
camera at r = 1e4 M with a +-20 M field of view, 230 GHz, on seeded synthetic float32
256 x 256 MKS fluid grids (one per spin), FP64 geodesics with FP32 transfer (or FP64 with
--prec f64).  Inputs are resident in device memory before timing starts and outputs stay in
device memory.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz


def cpu_baseline(sets, opts_gpu, budget_s=12.0):
    """The oracle on this host's cores over a bounded, strided pixel sample of the same
    workload: ray-steps per second."""
    import numpy as np
    from oracle import oracle as O
    import synthetic as S
    from tests.gpu_common import oracle_opts
    oo = oracle_opts(O, opts_gpu)
    threads = len(os.sched_getaffinity(0))
    env_threads = os.environ.get("OMP_NUM_THREADS")
    if env_threads and env_threads.isdigit():
        threads = min(threads, int(env_threads))
    steps = 0
    rays = 0
    t0 = time.perf_counter()
    chunk = 0
    while time.perf_counter() - t0 < budget_s and chunk < 64:
        for k, (cam, g) in enumerate(sets):
            pix = np.arange(chunk * 97 + k, cam.nx * cam.ny, 4099, dtype=np.int64)[:64]
            _, st = O.trace_pixels(cam, O.GridHandle(g), oo, [S.NU_230], pix, n_threads=threads)
            steps += int(st[:, 1].sum())
            rays += pix.size
        chunk += 1
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "ray-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{rays} rays ({rays // len(sets)} per image, strided over the 9 images of the "
                      f"workload), {steps} ray-steps in {dt:.1f} s, FP64, 230 GHz"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "trace_kernel_traffic.json"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy 3 times (HBM counter calibration)")
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
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is described "
                                   "in DESIGN.md but not launched"}))
        sys.exit(2)

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
    opts = R.default_opts(transfer_prec=R.F32 if args.prec == "f32" else R.F64, mem=R.MEM_DEVICE)
    n_pix = sum(c.nx * c.ny for c in cams)
    images = torch.empty(n_pix, dtype=torch.float64, device="cuda")
    flux = torch.empty((len(cams), 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step():
        return ctx.trace_batch(cams, grids, [S.NU_230], opts, images=images, flux=flux)[2]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    ray_steps = sum(s.ray_steps for s in stats) / args.steps
    samples = sum(s.samples for s in stats) / args.steps
    kern_ms = sum(s.kernel_ms for s in stats) / args.steps
    w = R.work_per_unit()
    fp64_flops = ray_steps * w["step_flops"] + samples * w["sample_flops"]
    if args.prec == "f64":
        fp64_flops += samples * w["freq_flops"]
    achieved = fp64_flops / (kern_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("prec") == args.prec and tj.get("res") == args.res:
            traffic = tj.get("bytes_per_launch")
    out = {
        "metric": "ray-steps/sec and 512^2 images/sec, plain vs MLP-emissivity at <=1e-3 flux err",
        "value": ray_steps / (ms * 1e-3),
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
                               f"FP64 geodesic + {args.prec.upper()} transfer, exact closure",
                   "closure": "exact", "images_per_step": len(cams), "rays_per_step": n_pix},
        "images_per_s": len(cams) / (ms * 1e-3),
        "images_512_per_s": len(cams) * (args.res * args.res) / (512 * 512) / (ms * 1e-3),
        "ray_steps_per_step": ray_steps,
        "samples_per_step": samples,
        "kernel_ms": kern_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "trace_kernel (fused RK4 geodesic + transfer)",
                     "flops_per_ray_step": w["step_flops"], "flops_per_sample": w["sample_flops"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sets, opts)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
