"""Benchmark: stereo multichannel ray casting on one MI355X.

Default workload: 2-channel 12-bit uint16 512x512x64 confocal-like volume
(40 ellipsoidal cells, 10 spline vessels, Poisson noise), perspective stereo
pair 1920x1080 per eye, step 1 voxel, early termination at alpha 0.99, FP32.
One step = one stereo pair (one vr_render launch, both eyes).  Prints one
JSON line: ray-samples/s (composited samples, the method's nominal count),
stereo frames/s, the HBM roofline of the render kernel on effective sampled
bytes (8 taps x channels x bytes per voxel per sample), and the FP64 CPU
oracle timed on a bounded pixel sample of the same frame.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "render_2ch_u16_realistic_stereo_counters.txt")


def _light():
    from paper_1407_2089_amd.synth import Light
    return Light((0.4, -0.3, -0.8), 0.3, 0.7)


def render_kernel_hash():
    """sha256 of the render kernel's source (march.h, params.h and the plain
    render kernel's part of kernels.hip)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1407_2089_amd", "csrc")
    for f in ("march.h", "params.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "kernels.hip")) as fh:
        k = fh.read()
    a = k.index("// ------------------------------------------------------------ plain render")
    b = k.index("// -------------------------------------------------------- batched render")
    h.update(k[a:b].encode())
    return h.hexdigest()


def measured_counters():
    """From the committed rocprofv3 counter summary of the headline kernel:
    HBM-side bytes per launch (FETCH_SIZE and WRITE_SIZE, scaled by a plain
    copy's readings), VALU busy and TA busy fractions; an empty dict once the
    kernel's source has changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            text = fh.read()
    except OSError:
        return {}
    import re
    h = re.search(r"sha256 \(.*\):\s*([0-9a-f]{64})", text)
    if not h or h.group(1) != render_kernel_hash():
        return {}
    out = {}
    t = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    if t:
        out["traffic"] = int(t.group(1))
    v = re.search(r"VALUBusy ([0-9.]+) %", text)
    if v:
        out["valu_busy"] = float(v.group(1)) / 100.0
    a = re.search(r"TA busy ([0-9.]+) %", text)
    if a:
        out["ta_busy"] = float(a.group(1)) / 100.0
    return out


def measured_traffic():
    """HBM-side bytes per launch of the headline kernel (see
    measured_counters), or None."""
    return measured_counters().get("traffic")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(scene, target_s=10.0):
    """Time the FP64 oracle on the host: the whole stereo pair (lit: 2^18
    seeded pixels per eye), repeated until about target_s seconds have
    passed, on every host thread; plus one thread on 2^16 seeded pixels per
    eye."""
    import numpy as np

    import oracle
    cores = os.cpu_count() or 1
    ov = oracle.Volume(scene.volume, scene.bits, scene.spacing, scene.origin)
    tfs = [oracle.Transfer(t.lo, t.hi, t.curve, t.alpha_mul, t.rgb, t.visible) for t in scene.tfs]
    c = scene.cam
    cam = oracle.Camera(c.projection, c.center, c.forward, c.up, c.fov_y, c.ortho_height,
                        c.eye_separation, c.convergence)
    lt = scene.light
    light = None if lt is None else oracle.Light(lt.direction, lt.ambient, lt.diffuse)

    def run(pixels, threads):
        s = 0
        for eye in (-1, 1):
            r = oracle.render(ov, tfs, cam, scene.width, scene.height, eye, scene.step,
                              scene.term_alpha, pixels=pixels, nthreads=threads, light=light)
            s += int(r["samples"].sum())
        return s

    rng = np.random.default_rng(12345)
    npix = scene.width * scene.height
    many = None if light is None else rng.choice(npix, size=min(npix, 1 << 18), replace=False)
    t0 = time.perf_counter()
    samples, reps = 0, 0
    while reps == 0 or time.perf_counter() - t0 < target_s:
        samples += run(many, cores)
        reps += 1
    dt = time.perf_counter() - t0
    pix = rng.choice(npix, size=1 << 16, replace=False)
    t1 = time.perf_counter()
    s1 = run(pix, 1)
    dt1 = time.perf_counter() - t1
    what = (f"the whole stereo pair ({2 * npix} rays)" if many is None
            else f"2 x {many.size} seeded pixels, lit")
    return {"value": samples / dt, "unit": "ray-samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{what} x {reps}, FP64, {dt:.1f} s on {cores} threads",
            "value_1thread": s1 / dt1,
            "sample_1thread": f"2 x 65536 seeded pixels, {dt1:.1f} s"}


def denoise_cpu_baseline(crop=(256, 256, 64)):
    """The denoising oracle (numpy, one thread) on a crop of the same frame:
    bounded CPU work."""
    import numpy as np

    from oracle import denoise as dn
    from paper_1407_2089_amd import workloads
    vol, (wx, wy, wz) = workloads.denoise_setup()
    cx, cy, cz = crop
    v = vol[:cz, :cy, :cx].cpu().numpy().view(np.uint16).copy()
    t0 = time.perf_counter()
    dn.remove_background(v, wx, wy, wz, 16)
    t_bg = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, iters, _, _ = dn.mrf(v, 12, 50)
    t_mrf = time.perf_counter() - t0
    return {"kind": "oracle", "cores": 1, "unit": "voxels/s",
            "sample": f"{cx}x{cy}x{cz} crop of the frame, numpy int64, one thread",
            "background_voxels_per_s": v.size / t_bg,
            "mrf_voxel_steps_per_s": v.size * (iters + 1) / t_mrf, "mrf_iterations": iters}


def montage_cpu_baseline(src, cam, tfs, W, H, target_s=10.0):
    """The oracle on seeded single rays of the montage view, each rendered on
    its ray's crop of the volume (the montage is too large to copy whole):
    one thread, about target_s seconds of oracle time."""
    import numpy as np

    import oracle
    from paper_1407_2089_amd import workloads
    rng = np.random.default_rng(12345)
    otf = [oracle.Transfer(t.lo, t.hi, t.curve, t.alpha_mul, t.rgb, t.visible) for t in tfs]
    ocam = oracle.Camera(cam.projection, cam.center, cam.forward, cam.up, cam.fov_y,
                         cam.ortho_height, cam.eye_separation, cam.convergence)
    dims = (src.shape[3], src.shape[2], src.shape[1])
    samples, rays, spent = 0, 0, 0.0
    while spent < target_s:
        pix = int(rng.integers(W * H))
        eye = -1 if rng.integers(0, 2) == 0 else 1
        box = workloads.ray_crop(cam, W, H, eye, pix % W, pix // W, dims)
        if box is None:
            continue
        lo, hi = box
        crop = src[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        ov = oracle.Volume(crop, 8, (1.0, 1.0, 1.0), tuple(float(x) for x in lo))
        t0 = time.perf_counter()
        r = oracle.render(ov, otf, ocam, W, H, eye, 1.0, 0.99, pixels=[pix], nthreads=1)
        spent += time.perf_counter() - t0
        samples += int(r["samples"].sum())
        rays += 1
    return {"value": samples / spent, "unit": "ray-samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{rays} seeded rays of the stereo view that meet the volume, each on its "
                      f"ray's crop, FP64, one thread, {spent:.1f} s"}


def tiny(args):
    """Launch-bound small case: 1-channel u8 64x64x32, ortho mono 256x256."""
    import numpy as np
    import torch

    import paper_1407_2089_amd as vr
    from paper_1407_2089_amd import synth
    sc = synth.tiny_scene()
    ctx = vr.Context(0)
    vol = vr.Volume(ctx, (64, 64, 32), 1, 1, vr.VR_U8, 8, row_pairs=args.layout == "pairs")
    vol.upload(0, torch.from_numpy(sc.volume).cuda())
    vol.set_transfer(0, sc.tfs[0])
    out = torch.empty((1, 256, 256, 4), dtype=torch.float32, device="cuda")
    smp = torch.empty((1, 256, 256), dtype=torch.int32, device="cuda")
    req = vr.make_request(vol.ptr, 0, sc.cam, 256, 256, False, 0.5, 1.0, out, out_samples=smp)
    vr.vr_render(ctx.ptr, req)
    torch.cuda.synchronize()
    samples = int(smp.sum().item())
    ms = []
    for _ in range(50 + 5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        vr.vr_render(ctx.ptr, req)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    med = float(np.median(ms[5:]))
    vol.destroy()
    ctx.close()
    return {"workload": "tiny: 1ch u8 64x64x32 blobs, ortho mono 256x256, step 0.5",
            "layout": args.layout,
            "samples": samples, "median_ms": med, "samples_per_s": samples / (med * 1e-3),
            "eff_GBps": samples * 8 / (med * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp32", "fp16"], default="fp32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--mode", choices=["render", "copy"], default="render",
                    help="copy: a plain 1 GiB device copy, to calibrate HBM byte counters")
    ap.add_argument("--workload", choices=["realistic", "tiny", "batch", "serve", "precision",
                                           "layout", "denoise", "stream", "montage"],
                    default="realistic",
                    help="realistic (default): one stereo 1920x1080 frame per step; batch: 64 "
                         "mixed requests, batched vs plain launches; serve: Poisson arrivals "
                         "on resident datasets, p50/p99; precision: 48-frame series FP32/FP16; "
                         "denoise: background removal and MRF of a 1024x1024x64 channel; stream: "
                         "playback of the 48-frame series from pinned host memory")
    ap.add_argument("--brick", default="0,0,0", help="brick edge per axis (0,0,0 = default)")
    ap.add_argument("--tile", default="", help="wave_w,wave_h (pixels per wave) of vr_render")
    ap.add_argument("--layout", choices=["bricks", "pairs"], default="pairs",
                    help="voxel layout of the realistic and tiny frames: bricks with row "
                         "pairs (default; two 16-byte loads per sample for the realistic "
                         "frame, 2.2x the storage) or plain bricks (the library's default "
                         "layout)")
    ap.add_argument("--lit", action="store_true",
                    help="light the realistic frame (one directional light, gradients from "
                         "central differences); also times the unlit kernel for the ratio")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-gb", type=float, default=150.0)
    ap.add_argument("--serve-rates", default="25,100,400,1000,1600,2400,3200,4000")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(rays, eyes and requests shard across GPUs with no exchange; see the "
              "design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1407_2089_amd as vr
    from paper_1407_2089_amd import synth

    if args.mode == "copy":
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n,
                          "copies": 5}), flush=True)
        return

    if args.workload != "realistic":
        from paper_1407_2089_amd import workloads
        ctx = vr.Context(0)
        if args.workload == "tiny":
            ctx.close()
            print(json.dumps(dict(tiny(args), n_gpus=1, data="synthetic")), flush=True)
            return
        if args.workload == "batch":
            res = workloads.batching(ctx)
        elif args.workload == "precision":
            res = workloads.precision(ctx)
        elif args.workload == "layout":
            res = workloads.layout_sweep(ctx)
        elif args.workload == "stream":
            res = workloads.streaming(ctx)
        elif args.workload == "montage":
            res = workloads.montage(ctx, cpu=None if args.no_cpu else montage_cpu_baseline)
        elif args.workload == "denoise":
            res = workloads.denoise(ctx)
            if not args.no_cpu:
                res["cpu_baseline"] = denoise_cpu_baseline()
        else:
            rates = tuple(int(r) for r in args.serve_rates.split(","))
            res = workloads.serving(ctx, total_gb=args.serve_gb, seconds=args.serve_seconds,
                                    rates=rates)
        ctx.close()
        res["n_gpus"] = 1
        res["data"] = "synthetic"
        print(json.dumps(res), flush=True)
        return

    log("generating workload")
    sc = synth.realistic_scene()
    if args.lit:
        sc.light = _light()
    ctx = vr.Context(0)
    c, nz, ny, nx = sc.volume.shape
    brick = tuple(int(b) for b in args.brick.split(","))
    pairs = args.layout == "pairs"
    vol = vr.Volume(ctx, (nx, ny, nz), c, 1, vr.VR_U16, sc.bits, brick=brick, row_pairs=pairs)
    if args.tile:
        vr.vr_test_plain_tile(ctx.ptr, *[int(t) for t in args.tile.split(",")])
    stream = torch.cuda.current_stream()
    vol.upload(0, torch.from_numpy(sc.volume.view(np.int16)).cuda(), stream)
    for ch, tf in enumerate(sc.tfs):
        vol.set_transfer(ch, tf)
    prec = vr.VR_FP16 if args.precision == "fp16" else vr.VR_FP32
    out = torch.empty((2, sc.height, sc.width, 4), dtype=torch.float32, device="cuda")
    smp = torch.empty((2, sc.height, sc.width), dtype=torch.int32, device="cuda")

    # Count the composited samples of one step (the frame is the same every step).
    req_count = vr.make_request(vol.ptr, 0, sc.cam, sc.width, sc.height, True, sc.step,
                                sc.term_alpha, out, precision=prec, out_samples=smp,
                                light=sc.light)
    vr.vr_render(ctx.ptr, req_count, stream)
    torch.cuda.synchronize()
    samples_per_step = int(smp.sum().item())
    req = vr.make_request(vol.ptr, 0, sc.cam, sc.width, sc.height, True, sc.step,
                          sc.term_alpha, out, precision=prec, light=sc.light)

    def timed(r):
        log(f"warmup {args.warmup}")
        for _ in range(args.warmup):
            vr.vr_render(ctx.ptr, r, stream)
        torch.cuda.synchronize()
        log(f"timing {args.steps} steps")
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            vr.vr_render(ctx.ptr, r, stream)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, float(np.mean([a.elapsed_time(b) for a, b in ev]))

    wall, kernel_ms = timed(req)
    ms_per_step = 1000.0 * wall / args.steps
    value = samples_per_step * args.steps / wall
    unlit_ms = None
    if args.lit:
        log("unlit kernel for the ratio")
        _, unlit_ms = timed(vr.make_request(vol.ptr, 0, sc.cam, sc.width, sc.height, True,
                                            sc.step, sc.term_alpha, out, precision=prec))

    bytes_per_sample = 8 * c * 2
    alg_bytes = samples_per_step * bytes_per_sample
    headline_layout = (args.precision == "fp32" and brick == (0, 0, 0) and not args.tile
                       and pairs and not args.lit)
    counters = measured_counters() if headline_layout else {}
    traffic = counters.get("traffic")
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    result = {
        "metric": "ray-samples/s",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-sample/f32-composite" if prec == vr.VR_FP16 else "f32",
        "data": "synthetic",
        "config": {"workload": "realistic frame: 2ch u16-12 512x512x64 cells+vessels, "
                               "perspective stereo 1920x1080 per eye, step 1, alpha 0.99"
                               + (", lit (one directional light)" if args.lit else ""),
                   "eyes": 2, "width": sc.width, "height": sc.height, "brick": list(brick),
                   "layout": args.layout, "storage_bytes": vol.bytes,
                   "tile": args.tile or "8,8",
                   "samples_per_step": samples_per_step},
        "stereo_fps": args.steps / wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "traffic_unit": "bytes/launch (L2-to-fabric FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "kernel": f"render_kernel<2ch,u16,{args.precision},{args.layout}"
                               + (",lit>" if args.lit else ">"),
                     "kernel_ms": kernel_ms, "bytes_per_launch": alg_bytes,
                     # effective bytes price every tap as an HBM byte; the measured
                     # fabric-side rate of the same launches, for comparison:
                     "traffic_GBps": (traffic / (kernel_ms * 1e-3) / 1e9
                                      if traffic is not None else None),
                     # what does limit the kernel (rocprofv3 counters of the same launch)
                     "valu_busy": counters.get("valu_busy"),
                     "ta_busy": counters.get("ta_busy")},
    }
    if args.lit:
        result["config"]["light"] = {"direction": list(sc.light.direction),
                                     "ambient": sc.light.ambient, "diffuse": sc.light.diffuse}
        # effective bytes count the sample's own 8 taps only; the six gradient
        # samples of each shaded sample are not priced
        result["roofline"]["bytes_note"] = "8 taps per sample; gradient samples not counted"
        result["unlit_kernel_ms"] = unlit_ms
        result["lit_over_unlit"] = kernel_ms / unlit_ms
    vol.destroy()
    ctx.close()
    if not args.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
