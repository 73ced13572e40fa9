"""Workload runners for the batching, serving, precision and denoising measurements.

Each runner builds its seeded synthetic inputs on the GPU, drives libvr
through the binding and returns a dict of measurements.  No rendering
arithmetic lives here.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import synth
from . import (VR_FP16, VR_FP32, VR_U8, VR_U16, C, Volume, gaussian_weights, make_grid,
               make_lowpass, make_request, vr_denoise_workspace_bytes, vr_mrf_denoise, vr_poll,
               vr_release, vr_remove_background, vr_render, vr_render_batch, vr_stream_frame,
               vr_stream_ready, vr_submit, vr_tune_batch, vr_tune_layout, vr_volume_desc)

SIZES_BATCH = [(960, 540), (1280, 720), (1600, 900), (1920, 1080)]
SIZES_SERVE = [(960, 540), (1920, 1080), (2560, 1440), (3840, 2160)]
# six channel colours (the viewer offers six): green, red, blue, yellow,
# cyan, magenta
PALETTE = [(0.0, 1.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.4, 1.0), (1.0, 1.0, 0.0),
           (0.0, 1.0, 1.0), (1.0, 0.0, 1.0)]


def log(msg):
    import sys
    print(msg, file=sys.stderr, flush=True)


def default_tfs(channels):
    return [synth.TF(300.0 / 4095.0, 3000.0 / 4095.0, 0.0, 1.0, PALETTE[c]) for c in range(channels)]


def pairs_allowed(channels, bits):
    """Row pairs exist for voxel words of at most 4 bytes."""
    return channels <= 2 or (channels <= 4 and bits <= 8)


def tune_layout(ctx, series, tfs, reps=3):
    """(brick, row_pairs) that vr_tune_layout picks for frame 0 of a
    DeviceSeries, timed on a 1920x1080 stereo overview."""
    import torch
    nx, ny, nz = series.dims
    dtype = VR_U8 if series.bits <= 8 else VR_U16
    desc = vr_volume_desc(nx, ny, nz, series.channels, 1, dtype, series.bits,
                          (C.c_float * 3)(1, 1, 1), (C.c_float * 3)(0, 0, 0),
                          (C.c_int32 * 3)(0, 0, 0), 0)
    out = torch.empty((2, 1080, 1920, 4), dtype=torch.float32, device="cuda")
    cam = synth.orbit_camera(series.dims, 30.0, 40.0, 40.0)
    view = make_request(None, 0, cam, 1920, 1080, True, 1.0, 0.99, out)
    vr_tune_layout(ctx.ptr, desc, tfs, series.frame(0), [view], reps=reps)
    return tuple(desc.brick), bool(desc.row_pairs)


def load_series(ctx, series, frames, tfs, stream=None, row_pairs=False, brick=(0, 0, 0)):
    """Create a resident volume and upload every frame of a DeviceSeries."""
    import torch
    nx, ny, nz = series.dims
    dtype = VR_U8 if series.bits <= 8 else VR_U16
    vol = Volume(ctx, (nx, ny, nz), series.channels, frames, dtype, series.bits,
                 brick=brick, row_pairs=row_pairs)
    for t in range(frames):
        f = series.frame(t)
        vol.upload(t, f, stream or torch.cuda.current_stream())
        del f
    for c, tf in enumerate(tfs):
        vol.set_transfer(c, tf)
    return vol


def count_samples(ctx, reqs):
    """Composited samples of each request (one counting render)."""
    import torch
    counts = []
    for r in reqs:
        eyes = 2 if r.stereo else 1
        smp = torch.empty((eyes, r.height, r.width), dtype=torch.int32, device="cuda")
        saved = r.out_samples
        r.out_samples = smp.data_ptr()
        vr_render(ctx.ptr, r, torch.cuda.current_stream())
        torch.cuda.synchronize()
        counts.append(int(smp.sum().item()))
        r.out_samples = saved
    return counts


# ------------------------------------------------------------------ batching

def batching_setup(ctx, n_req=64, n_vol=16, seed=4):
    """The batching workload's volumes and requests: 64 stereo requests over
    16 volumes of uneven size (2^21..2^26 voxels, 1-4 channels, u8 / u16-12 /
    u16-16; each layout chosen by vr_tune_layout), 960x540..1920x1080 per
    eye, random view directions.  Returns (volumes, their DeviceSeries,
    meta [(dims, channels, bits)], requests, outputs, request -> volume
    index, cameras)."""
    import torch
    rng = np.random.default_rng(seed)
    vols, sers, meta = [], [], []
    log("batching: generating volumes")
    for q in range(n_vol):
        voxels = 2.0 ** rng.uniform(21, 26)
        nz = int(8 * round(rng.uniform(64, 128) / 8))
        nxy = int(round(math.sqrt(voxels / nz)))
        ch = int(rng.integers(1, 5))
        kind = int(rng.integers(0, 3))
        bits = (8, 12, 16)[kind]
        ser = synth.DeviceSeries((nxy, nxy, nz), ch, bits, 4000 + q)
        tfs = default_tfs(ch)
        # each dataset's layout chosen by vr_tune_layout on one overview
        brick, pairs = tune_layout(ctx, ser, tfs)
        vols.append(load_series(ctx, ser, 1, tfs, row_pairs=pairs, brick=brick))
        sers.append(ser)
        meta.append(((nxy, nxy, nz), ch, bits))
    reqs, outs, which, cams = [], [], [], []
    for q in range(n_req):
        v = int(rng.integers(0, n_vol))
        dims = meta[v][0]
        w, h = SIZES_BATCH[int(rng.integers(0, len(SIZES_BATCH)))]
        cam = synth.random_view_camera(rng, dims, True)
        out = torch.empty((2, h, w, 4), dtype=torch.float32, device="cuda")
        reqs.append(make_request(vols[v].ptr, 0, cam, w, h, True, 1.0, 0.99, out))
        outs.append(out)
        which.append(v)
        cams.append(cam)
    return vols, sers, meta, reqs, outs, which, cams


def batching(ctx, n_req=64, n_vol=16, seed=4, reps=5):
    """The batching workload (batching_setup): one vr_render_batch call
    against 64 sequential vr_render calls (one launch per stereo request)."""
    import torch
    vols, _, meta, reqs, outs, _, _ = batching_setup(ctx, n_req, n_vol, seed)
    counts = count_samples(ctx, reqs)
    total_samples = sum(counts)
    eff_bytes = sum(c * 8 * meta_bytes(meta, vols, reqs[i]) for i, c in enumerate(counts))
    stream = torch.cuda.current_stream()

    def run_plain():
        for r in reqs:
            vr_render(ctx.ptr, r, stream)

    def run_batch():
        vr_render_batch(ctx.ptr, reqs, stream)

    # warm-up, and the autotuner's choice of wave tile for this shape class
    run_plain()
    tile = vr_tune_batch(ctx.ptr, reqs, stream)
    run_batch()
    torch.cuda.synchronize()
    # bitwise equality of the two paths
    run_plain()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    for o in outs:
        o.fill_(float("nan"))
    run_batch()
    torch.cuda.synchronize()
    equal = all(torch.equal(a, b) for a, b in zip(outs, ref))
    del ref

    def timed(fn):
        best = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best.append(time.perf_counter() - t0)
        return float(np.median(best))

    t_plain = timed(run_plain)
    t_batch = timed(run_batch)
    for v in vols:
        v.destroy()
    return {
        "workload": "batching: 64 stereo requests over 16 volumes (2^21..2^26 voxels, 1-4 "
                    "channels, u8/u16-12/u16-16, each layout chosen by vr_tune_layout), "
                    "960x540..1920x1080 per eye, step 1, alpha 0.99",
        "requests": n_req, "total_samples": total_samples, "bitwise_equal": equal,
        "plain_s": t_plain, "batch_s": t_batch,
        "plain_stereo_fps": n_req / t_plain, "batch_stereo_fps": n_req / t_batch,
        "plain_samples_per_s": total_samples / t_plain,
        "batch_samples_per_s": total_samples / t_batch,
        "batch_eff_GBps": eff_bytes / t_batch / 1e9,
        "speedup": t_plain / t_batch, "tuned_tile": list(tile),
    }


def meta_bytes(meta, vols, req):
    for (dims, ch, bits), v in zip(meta, vols):
        if v.ptr == req.vol:
            return ch * (1 if bits <= 8 else 2)
    return 0


# ------------------------------------------------------------------ precision

def precision_setup(ctx, frames=48, seed=3, upload=None):
    """The 4-channel uint8 1024x1024x48 series (seeded, generated on the GPU),
    its transfer functions (lo 24/255, hi 220/255, green / red / blue /
    yellow) and the orbit cameras (azimuth 7.5 degrees per frame, elevation
    40, fov 40).  `upload` lists the frames to make resident (default all)."""
    dims = (1024, 1024, 48)
    ser = synth.DeviceSeries(dims, 4, 8, seed, frames=frames, density=1.25)
    tfs = [synth.TF(24 / 255, 220 / 255, 0.0, 1.0, PALETTE[c]) for c in range(4)]
    cams = [synth.orbit_camera(dims, 7.5 * t, 40.0, 40.0) for t in range(frames)]
    return dims, ser, tfs, cams


def precision(ctx, frames=48, seed=3, reps=2):
    """48 frames resident in HBM, one stereo 1920x1080 render per frame,
    FP32 against FP16 sampling (throughput; the error against the FP64
    oracle is measured by the test-suite)."""
    import torch
    log("precision: generating series")
    dims, ser, tfs, cams = precision_setup(ctx, frames, seed)
    vol = load_series(ctx, ser, frames, tfs)
    W, H = 1920, 1080
    out = torch.empty((2, H, W, 4), dtype=torch.float32, device="cuda")
    res = {"workload": "precision: 4ch u8 1024x1024x48, 48 frames resident, stereo 1920x1080 "
                       "per frame, orbit, step 1, alpha 0.99",
           "resident_bytes": vol.bytes}
    stream = torch.cuda.current_stream()
    for prec, name in ((VR_FP32, "fp32"), (VR_FP16, "fp16")):
        reqs = [make_request(vol.ptr, t, cams[t], W, H, True, 1.0, 0.99, out, precision=prec)
                for t in range(frames)]
        total = sum(count_samples(ctx, reqs))
        for r in reqs:
            vr_render(ctx.ptr, r, stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            for r in reqs:
                vr_render(ctx.ptr, r, stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        res[name] = {"samples_per_s": total / dt, "stereo_fps": frames / dt,
                     "eff_GBps": total * 32 / dt / 1e9, "samples_per_series": total}
    vol.destroy()
    return res


# ---------------------------------------------------------------- streaming

PCIE_GBS = 64.0   # PCIe 5.0 x16, one direction (published link rate)


def streaming(ctx, frames=48, slots=3, seed=3, reps=2):
    """Playback of the precision series (4-channel uint8 1024x1024x48, 48
    frames = 9.66 GB) kept in pinned host memory, through a ring of `slots`
    device frames: each step streams a later frame in while the current one
    renders (stereo 1920x1080)."""
    import torch
    log("streaming: generating series into pinned host memory")
    dims, ser, tfs, cams = precision_setup(ctx, frames, seed)
    first = ser.frame(0)
    host = torch.empty((frames,) + tuple(first.shape), dtype=first.dtype, pin_memory=True)
    for t in range(frames):
        host[t].copy_(ser.frame(t) if t else first)
    frame_bytes = host[0].numel() * host.element_size()
    vol = Volume(ctx, dims, 4, slots, VR_U8, 8)
    for c, tf in enumerate(tfs):
        vol.set_transfer(c, tf)
    staging = torch.empty(2 * frame_bytes, dtype=torch.uint8, device="cuda")  # two halves
    copy = torch.cuda.Stream()
    stream = torch.cuda.current_stream()
    W, H = 1920, 1080
    out = torch.empty((2, H, W, 4), dtype=torch.float32, device="cuda")

    def play():
        for t in range(min(slots - 1, frames)):
            vr_stream_frame(vol.ptr, t, host[t], staging, 2 * frame_bytes, copy, stream)
        for t in range(frames):
            nxt = t + slots - 1
            if nxt < frames:
                vr_stream_frame(vol.ptr, nxt % slots, host[nxt], staging, 2 * frame_bytes,
                                copy, stream)
            vr_stream_ready(vol.ptr, t % slots, stream)
            vr_render(ctx.ptr, make_request(vol.ptr, t % slots, cams[t], W, H, True, 1.0,
                                            0.99, out), stream)
        torch.cuda.synchronize()

    play()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        play()
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    # the copy alone: pinned host -> device, one frame at a time
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(copy):
        a.record(copy)
        for t in range(8):
            staging[:frame_bytes].copy_(host[t].view(torch.uint8).reshape(-1),
                                        non_blocking=True)
        b.record(copy)
    torch.cuda.synchronize()
    copy_gbs = 8 * frame_bytes / (a.elapsed_time(b) * 1e-3) / 1e9
    # the renders alone (frames already resident in the slots)
    a.record(stream)
    for t in range(frames):
        vr_render(ctx.ptr, make_request(vol.ptr, t % slots, cams[t], W, H, True, 1.0, 0.99,
                                        out), stream)
    b.record(stream)
    torch.cuda.synchronize()
    render_ms = a.elapsed_time(b) / frames
    vol.destroy()
    fps = frames / dt
    return {"workload": f"streaming: 4ch u8 1024x1024x48, {frames} frames in pinned host memory "
                        f"({frames * frame_bytes / 1e9:.2f} GB), {slots} device slots, stereo "
                        "1920x1080 per frame",
            "frame_bytes": frame_bytes, "stereo_fps": fps, "ms_per_frame": 1e3 / fps,
            "h2d_GBps": fps * frame_bytes / 1e9, "copy_only_GBps": copy_gbs,
            "render_only_ms": render_ms,
            "roofline": {"bound": "pcie", "achieved": fps * frame_bytes / 1e9,
                         "peak": PCIE_GBS, "unit": "GB/s",
                         "frac": fps * frame_bytes / 1e9 / PCIE_GBS}}


# ------------------------------------------------------------------ denoise

DENOISE_DIMS = (1024, 1024, 64)
DENOISE_SIGMA = (16.0, 16.0, 4.0)


def denoise_setup(seed=11):
    """One 12-bit uint16 channel (the vessel channel of a generated
    1024x1024x64 confocal-like frame) as a [Z][Y][X] device tensor, and the
    quantised Gaussian weights (sigma 16, 16, 4 voxels; sums 2^16)."""
    frame = synth.DeviceSeries(DENOISE_DIMS, 2, 12, seed).frame(0)
    vol = frame[1].contiguous()
    w = [gaussian_weights(s, 16) for s in DENOISE_SIGMA]
    return vol, w


def denoise(ctx, reps=10, max_iters=500):
    """Background removal (eq. (1)) and the sign-diffusion iteration
    (eqs. (2)-(3)) of one 1024x1024x64 uint16 channel resident in HBM."""
    import torch
    log("denoise: generating frame")
    vol, (wx, wy, wz) = denoise_setup()
    nx, ny, nz = DENOISE_DIMS
    n = nx * ny * nz
    grid = make_grid(nx, ny, nz, VR_U16, 12)
    ws_bytes = vr_denoise_workspace_bytes(grid)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    dst, bg = torch.empty_like(vol), torch.empty_like(vol)
    lp = make_lowpass(wx, wy, wz, 16)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        vr_remove_background(ctx.ptr, grid, lp, vol, dst, bg, ws, ws_bytes, stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        vr_remove_background(ctx.ptr, grid, lp, vol, dst, bg, ws, ws_bytes, stream)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    bg_ms = float(np.median(times))
    taps = [len(wx), len(wy), len(wz)]
    res = {"workload": f"denoise: 1 channel u16-12 {nx}x{ny}x{nz} (vessel channel), "
                       f"Gaussian background sigma {DENOISE_SIGMA} ({taps} taps), 3x3x3 median; "
                       f"sign-diffusion MRF, max {max_iters} iterations",
           "voxels": n,
           "background": {"ms": bg_ms, "voxels_per_s": n / (bg_ms * 1e-3),
                          # per voxel: three passes read + write 2 B each, the
                          # median reads L and B and writes the result
                          "alg_bytes": 18 * n, "eff_GBps": 18 * n / (bg_ms * 1e-3) / 1e9,
                          "macs_per_voxel": sum(taps)}}
    mrf_dst = torch.empty_like(vol)
    vr_mrf_denoise(ctx.ptr, grid, 2, vol, mrf_dst, ws, ws_bytes, stream)  # warm-up
    t0 = time.perf_counter()
    info = vr_mrf_denoise(ctx.ptr, grid, max_iters, vol, mrf_dst, ws, ws_bytes, stream)
    wall = time.perf_counter() - t0
    # steps computed: the kept ones, the rejected one and, when that one was
    # the first of a pair, the pair's second (iterations run two per round
    # trip to the host)
    k = info.iterations
    steps = k
    if k < max_iters:
        steps += 1 + (1 if k % 2 == 0 and k + 2 <= max_iters else 0)
    res["mrf"] = {"iterations": info.iterations, "steps_run": steps, "sigma": info.sigma,
                  "delta": info.delta, "rms": info.rms, "wall_ms": wall * 1e3,
                  "ms_per_step": wall * 1e3 / max(steps, 1),
                  "voxel_steps_per_s": n * steps / wall,
                  # per voxel and step: read the current and the original
                  # image, write the next one
                  "alg_bytes_per_step": 6 * n}
    del ws
    return res


# ------------------------------------------------------------------- layout

def layout_sweep(ctx, reps=30):
    """Render time of one stereo 1920x1080 pair of a 512x512x64 frame for
    each brick shape and voxel-word size (1-channel u8: 1 B; 2-channel
    u16-12 and 4-channel u8: 4 B; 4-channel u16: 8 B), for a view entering
    through the top face and a grazing view entering through the sides."""
    import torch
    W, H = 1920, 1080
    dims = (512, 512, 64)
    views = {"top": synth.orbit_camera(dims, 30.0, 50.0, 45.0),
             "side": synth.orbit_camera(dims, 75.0, 10.0, 45.0)}
    bricks = [(4, 4, 4), (8, 8, 8), (16, 16, 16), (4, 8, 8), (8, 4, 8), (8, 8, 4), (8, 16, 8),
              (16, 8, 8), (16, 16, 8), (32, 8, 8), (0, 0, 0)]
    # row pairs exist for words of up to 4 bytes
    pair_bricks = [(0, 0, 0), (4, 16, 8), (8, 16, 8), (16, 16, 16), (8, 32, 8), (4, 32, 8)]
    out = torch.empty((2, H, W, 4), dtype=torch.float32, device="cuda")
    rows = []
    for ch, bits in ((1, 8), (2, 12), (4, 8), (4, 16)):
        frame = synth.DeviceSeries(dims, ch, bits, 77).frame(0)
        cases = [(b, False) for b in bricks] + (
            [(b, True) for b in pair_bricks] if pairs_allowed(ch, bits) else [])
        for b, pairs in cases:
            vol = Volume(ctx, dims, ch, 1, VR_U8 if bits == 8 else VR_U16, bits, brick=b,
                         row_pairs=pairs)
            vol.upload(0, frame)
            for c, tf in enumerate(default_tfs(ch)):
                vol.set_transfer(c, tf)
            for name, cam in views.items():
                req = make_request(vol.ptr, 0, cam, W, H, True, 1.0, 0.99, out)
                for _ in range(5):
                    vr_render(ctx.ptr, req)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    vr_render(ctx.ptr, req)
                e1.record()
                torch.cuda.synchronize()
                rows.append({"channels": ch, "bits": bits, "brick": list(b), "row_pairs": pairs,
                             "view": name, "ms": e0.elapsed_time(e1) / reps,
                             "storage_bytes": vol.bytes})
                log(f"  ch {ch} bits {bits} brick {b} pairs {pairs} {name}: "
                    f"{rows[-1]['ms']:.4f} ms")
            vol.destroy()
    return {"workload": "layout sweep: 512x512x64, stereo 1920x1080, step 1, alpha 0.99",
            "rows": rows}


# ------------------------------------------------------------------- serving

class _Pool:
    """Reusable output buffers per image size (client side)."""

    def __init__(self, per_size=6):
        self.free = {}
        self.per_size = per_size

    def take(self, w, h):
        import torch
        lst = self.free.setdefault((w, h), [])
        if lst:
            return lst.pop()
        return torch.empty((2, h, w, 4), dtype=torch.float32, device="cuda")

    def give(self, w, h, t):
        self.free.setdefault((w, h), []).append(t)


def serving(ctx, total_gb=150.0, seconds=10.0, warm=1.0,
            rates=(25, 100, 400, 1000, 1600, 2400, 3200, 4000), seed=5, n_datasets=16, check=32,
            max_inflight=128):
    """16 resident datasets (2-4 channels, 24-96 frames of up to
    1024x1024x64 uint16-12, frame counts scaled to `total_gb` resident);
    Poisson arrivals of stereo requests (960x540..3840x2160) served by the
    continuous-batching loop, against the same arrivals on a FIFO server of
    plain per-request launches.  Latency = completion - scheduled arrival
    (a client holds at most `max_inflight` requests; arrivals beyond that
    wait, and their wait counts in their latency).  Frames/s = completed
    requests over the span from the first arrival to the last completion."""
    import torch
    rng = np.random.default_rng(seed)
    specs = []
    for q in range(n_datasets):
        ch = int(rng.integers(2, 5))
        nxy = int(rng.choice([512, 768, 1024]))
        nz = int(rng.choice([32, 48, 64]))
        frames = int(rng.integers(24, 97))
        specs.append([(nxy, nxy, nz), ch, frames])
    from . import vr_volume_desc, vr_volume_storage_bytes
    import ctypes as C

    def stored(dims, ch, frames):
        d = vr_volume_desc(dims[0], dims[1], dims[2], ch, frames, VR_U16, 12,
                           (C.c_float * 3)(1, 1, 1), (C.c_float * 3)(0, 0, 0),
                           (C.c_int32 * 3)(0, 0, 0))
        return vr_volume_storage_bytes(d)

    tot = sum(stored(*s) for s in specs)
    scale = total_gb * 1e9 / tot
    for s in specs:
        s[2] = max(1, int(round(s[2] * scale)))
    resident = sum(stored(*s) for s in specs)
    log(f"serving: generating {resident / 1e9:.1f} GB of resident series")
    vols = []
    for q, (dims, ch, frames) in enumerate(specs):
        ser = synth.DeviceSeries(dims, ch, 12, 5000 + q, frames=frames)
        vols.append(load_series(ctx, ser, frames, default_tfs(ch)))
        torch.cuda.synchronize()
        log(f"  dataset {q}: {dims} x {ch} ch x {frames} frames")
    pool = _Pool()
    results = {"workload": "serving: 16 resident datasets (2-4 ch, u16-12, up to 1024x1024x64, "
                           "24-96 frames scaled to the total), Poisson arrivals, stereo "
                           "960x540..3840x2160, step 1, alpha 0.99",
               "resident_bytes": resident, "seconds_per_rate": seconds, "rates": {}}

    def make_arrivals(lam):
        t, arr = 0.0, []
        while t < seconds:
            t += rng.exponential(1.0 / lam)
            if t >= seconds:
                break
            q = int(rng.integers(0, n_datasets))
            dims, ch, frames = specs[q]
            w, h = SIZES_SERVE[int(rng.integers(0, len(SIZES_SERVE)))]
            arr.append((t, q, int(rng.integers(0, frames)), synth.random_view_camera(rng, dims),
                        w, h))
        return arr

    def summarize(lat, n_done, span):
        lat = np.sort(np.asarray(lat))
        if lat.size == 0:
            return {}
        pick = lambda p: float(lat[min(lat.size - 1, max(0, int(math.ceil(p * lat.size)) - 1))])
        return {"p50_ms": pick(0.50) * 1e3, "p99_ms": pick(0.99) * 1e3,
                "stereo_fps": n_done / span, "completed": int(n_done)}

    for lam in rates:
        arr = make_arrivals(lam)
        # ---- served (continuous batching)
        torch.cuda.synchronize()
        t0 = time.monotonic_ns()
        pending = []  # (ticket, index, scheduled ns, w, h, out), in submission order
        lat, keep = [], {}
        check_ids = set(rng.choice(len(arr), size=min(check, len(arr)), replace=False).tolist())
        k = 0
        while k < len(arr) or pending:
            now = time.monotonic_ns()
            while k < len(arr) and t0 + int(arr[k][0] * 1e9) <= now and len(pending) < max_inflight:
                ta, q, fr, cam, w, h = arr[k]
                out = pool.take(w, h)
                req = make_request(vols[q].ptr, fr, cam, w, h, True, 1.0, 0.99, out)
                pending.append((vr_submit(ctx.ptr, req), k, t0 + int(ta * 1e9), w, h, out))
                k += 1
            # completions, oldest first (a later one is seen once those before it are)
            while pending:
                tk, idx, sched, w, h, out = pending[0]
                info = vr_poll(ctx.ptr, tk)
                if info.state < 2:
                    break
                if info.state == 3:
                    raise RuntimeError(f"served request failed: status {info.err}")
                if arr[idx][0] >= warm:
                    lat.append((info.t_done_ns - sched) * 1e-9)
                if idx in check_ids:
                    keep[idx] = out.clone()
                    # the copy runs on torch's stream: let it finish before the
                    # buffer can be handed to a later request on a serving stream
                    torch.cuda.current_stream().synchronize()
                pool.give(w, h, out)
                vr_release(ctx.ptr, tk)
                pending.pop(0)
        span = (time.monotonic_ns() - t0) * 1e-9
        served = summarize(lat, sum(1 for a in arr if a[0] >= warm), span - warm)
        # ---- same arrivals, FIFO server of plain per-request launches
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t0 = time.monotonic_ns()
        lat2 = []
        same = True
        for idx, (ta, q, fr, cam, w, h) in enumerate(arr):
            sched = t0 + int(ta * 1e9)
            while time.monotonic_ns() < sched:
                pass
            out = pool.take(w, h)
            vr_render(ctx.ptr, make_request(vols[q].ptr, fr, cam, w, h, True, 1.0, 0.99, out),
                      stream)
            torch.cuda.synchronize()
            if ta >= warm:
                lat2.append((time.monotonic_ns() - sched) * 1e-9)
            if idx in keep:
                same = same and torch.equal(keep[idx], out)
            pool.give(w, h, out)
        span2 = (time.monotonic_ns() - t0) * 1e-9
        fifo = summarize(lat2, sum(1 for a in arr if a[0] >= warm), span2 - warm)
        results["rates"][str(lam)] = {"served": served, "fifo_plain": fifo,
                                      "alone_equals_mix": same, "checked": len(keep),
                                      "requests": len(arr)}
        log(f"  rate {lam}: served {served} fifo {fifo} same {same}")
    for v in vols:
        v.destroy()
    return results


# ------------------------------------------------------------------ montage

MONTAGE_DIMS = (10173, 3858, 74)   # stitched SVZ montage, 5 channels, 8 bit
MONTAGE_CHANNELS = 5


def montage_setup(ctx, seed=3, brick=(0, 0, 0), tune=False, row_pairs=False):
    """The five-channel uint8 montage resident in HBM (large-volume
    addressing: 2.9 G voxels per channel, 37.7 GB of default bricks) with the
    default transfer functions; with tune, its layout is chosen by
    vr_tune_layout on the overview (vol.layout_choice says which).  Returns
    (volume, source tensor, tfs)."""
    log("montage: generating 10173x3858x74x5 uint8")
    src = synth.montage(MONTAGE_DIMS, MONTAGE_CHANNELS, seed, log=log)
    tfs = [synth.TF(20.0 / 255.0, 200.0 / 255.0, 0.0, 1.0, PALETTE[c])
           for c in range(MONTAGE_CHANNELS)]
    import torch
    pairs, choice = row_pairs, f"given: brick {list(brick)}, row pairs {row_pairs}"
    if tune:
        desc = vr_volume_desc(*MONTAGE_DIMS, MONTAGE_CHANNELS, 1, VR_U8, 8,
                              (C.c_float * 3)(1, 1, 1), (C.c_float * 3)(0, 0, 0),
                              (C.c_int32 * 3)(0, 0, 0), 0)
        out = torch.empty((2, 1080, 1920, 4), dtype=torch.float32, device="cuda")
        view = make_request(None, 0, montage_camera(), 1920, 1080, True, 1.0, 0.99, out)
        t0 = time.time()
        ms = vr_tune_layout(ctx.ptr, desc, tfs, src, [view], reps=5)
        del out
        brick, pairs = tuple(desc.brick), bool(desc.row_pairs)
        choice = (f"vr_tune_layout: brick {list(brick)}, row pairs {pairs} ({ms:.3f} ms on "
                  f"the overview, {time.time() - t0:.1f} s of tuning)")
        log(choice)
    vol = Volume(ctx, MONTAGE_DIMS, MONTAGE_CHANNELS, 1, VR_U8, 8, brick=brick, row_pairs=pairs)
    vol.layout_choice = choice
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    a.record(stream)
    vol.upload(0, src, stream)
    b.record(stream)
    torch.cuda.synchronize()
    vol.relayout_ms = a.elapsed_time(b)
    for c, tf in enumerate(tfs):
        vol.set_transfer(c, tf)
    return vol, src, tfs


def montage_camera():
    return synth.orbit_camera(MONTAGE_DIMS, 30.0, 55.0, 40.0, 0.6)


def montage(ctx, reps=10, W=1920, H=1080, cpu=None, layout=None):
    """Stereo 1920x1080 views of the montage (perspective, elevation 55
    degrees, the montage's long side filling the view).  `cpu`, if given, is
    called as cpu(src, cam, tfs, W, H) while the source is still on the GPU
    and its result is returned as cpu_baseline.  layout: None to let
    vr_tune_layout choose, else (brick, row_pairs)."""
    import torch
    if layout is None:
        vol, src, tfs = montage_setup(ctx, tune=True)
    else:
        vol, src, tfs = montage_setup(ctx, brick=tuple(layout[0]), row_pairs=bool(layout[1]))
    cam = montage_camera()
    base = cpu(src, cam, tfs, W, H) if cpu is not None else None
    del src
    stream = torch.cuda.current_stream()
    out = torch.empty((2, H, W, 4), dtype=torch.float32, device="cuda")
    smp = torch.empty((2, H, W), dtype=torch.int32, device="cuda")
    req = make_request(vol.ptr, 0, cam, W, H, True, 1.0, 0.99, out, out_samples=smp)
    vr_render(ctx.ptr, req, stream)
    torch.cuda.synchronize()
    samples = int(smp.to(torch.int64).sum().item())
    req = make_request(vol.ptr, 0, cam, W, H, True, 1.0, 0.99, out)
    for _ in range(2):
        vr_render(ctx.ptr, req, stream)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        vr_render(ctx.ptr, req, stream)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    word = 8   # five uint8 channels per voxel word
    eff = samples * 8 * word / (ms * 1e-3) / 1e9
    frame_bytes = vol.bytes
    relayout_ms = vol.relayout_ms
    choice = vol.layout_choice
    vol.destroy()
    return {"workload": "montage: 5ch u8 10173x3858x74 (one frame, 14.5 GB of voxels, "
                        f"{frame_bytes / 1e9:.1f} GB of bricks), stereo {W}x{H}, step 1.0, "
                        "tau 0.99, perspective elevation 55 deg",
            "frame_bytes": frame_bytes, "layout_choice": choice, "samples": samples,
            "ms_per_step": ms,
            # upload: read 5 B per voxel, write the bricks
            "relayout_ms": relayout_ms,
            "relayout_GBps": (5 * 10173 * 3858 * 74 + frame_bytes) / (relayout_ms * 1e-3) / 1e9,
            "value": samples / (ms * 1e-3), "unit": "ray-samples/s",
            "roofline": {"bound": "hbm", "achieved": eff, "peak": 8000.0, "unit": "GB/s",
                         "frac": eff / 8000.0,
                         "note": "effective bytes: 8 taps x 8-byte words per sample"},
            "cpu_baseline": base}
