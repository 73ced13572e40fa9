"""GPU parity of the workloads at their own sizes, against the FP64 oracle on
seeded pixels:
  - batching: the 64-request batch over 16 volumes of 2^21..2^26 voxels at
    960x540..1920x1080 per eye, one vr_render_batch call, 2^14 seeded pixels
    per request;
  - serving: a mix of stereo requests on resident multi-frame datasets
    submitted to the serving loop while earlier ones run, 4096 seeded pixels
    per eye of sampled requests, each also equal to the same request
    rendered alone;
  - precision: the resident 48-frame 4-channel series (15.5 GB of bricks),
    frames 0, 16, 32 and 47 rendered from it in FP32 and FP16.
The max-abs RGBA errors are printed per case."""
import time

import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
from paper_1407_2089_amd import synth, workloads
from paper_1407_2089_amd.synth import Scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    c = vr.Context(0)
    yield c
    try:
        c.close()
    except vr.VrError:
        pass


def log(msg):
    print(msg, flush=True)


def host_frame(t):
    """A device frame [C][Z][Y][X] (uint8, or int16 holding uint16) as numpy."""
    a = t.cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a


def check_pixels(sc, rgba, smp, pixels, tol):
    """Compare a stereo image's seeded pixels (the same per eye) with the
    oracle; returns the comparison stats."""
    img = rgba.reshape(2, -1, 4)[:, pixels]
    ss = smp.reshape(2, -1)[:, pixels] if smp is not None else None
    ref = orc.render_all(sc, band_eps=tol, pixels=pixels)
    return gpu.compare(img, ss, ref, tol)


def test_batching_workload_against_oracle(ctx):
    import torch
    vols, sers, meta, reqs, outs, which, cams = workloads.batching_setup(ctx)
    smps = []
    for r, o in zip(reqs, outs):
        s = torch.full((2, r.height, r.width), -1, dtype=torch.int32, device="cuda")
        r.out_samples = s.data_ptr()
        o.fill_(float("nan"))
        smps.append(s)
    vr.vr_render_batch(ctx.ptr, reqs, torch.cuda.current_stream())
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    worst = 0.0
    hosts = {}
    try:
        for q, (r, o, s) in enumerate(zip(reqs, outs, smps)):
            v = which[q]
            if v not in hosts:
                hosts[v] = host_frame(sers[v].frame(0))
            dims, ch, bits = meta[v]
            sc = Scene("c4", hosts[v], bits, workloads.default_tfs(ch), cams[q], r.width,
                       r.height, True, 1.0, 0.99)
            pix = rng.choice(r.width * r.height, size=1 << 13, replace=False)
            st = check_pixels(sc, o.cpu().numpy(), s.cpu().numpy(), pix, 1e-3)
            worst = max(worst, st["max_err_accept"])
            if q % 16 == 0:
                log(f"request {q}: {dims} {ch} ch {bits} bit {r.width}x{r.height}: {st}")
        log(f"batching workload: 64 requests x 2 x 8192 seeded pixels, max-abs error "
            f"{worst:.2e}")
    finally:
        for v in vols:
            v.destroy()


def test_serving_mix_against_oracle(ctx):
    """Four resident datasets (2-4 channels, u16-12, 3-5 frames each); 40
    stereo requests at 960x540..1920x1080 with random frames and views,
    submitted in bursts while earlier ones run; 8 of them checked on 4096
    seeded pixels per eye against the oracle and bitwise against the same
    request rendered alone."""
    import torch
    rng = np.random.default_rng(55)
    specs = [((384, 384, 48), 2, 4), ((512, 512, 32), 3, 3), ((256, 256, 64), 4, 5),
             ((448, 448, 40), 2, 3)]
    sers, vols = [], []
    try:
        for q, (dims, ch, frames) in enumerate(specs):
            ser = synth.DeviceSeries(dims, ch, 12, 700 + q, frames=frames)
            sers.append(ser)
            vols.append(workloads.load_series(ctx, ser, frames, workloads.default_tfs(ch)))
        torch.cuda.synchronize()
        reqs, outs, meta = [], [], []
        for k in range(40):
            q = int(rng.integers(0, len(specs)))
            dims, ch, frames = specs[q]
            fr = int(rng.integers(0, frames))
            w, h = workloads.SIZES_BATCH[int(rng.integers(0, len(workloads.SIZES_BATCH)))]
            cam = synth.random_view_camera(rng, dims, True)
            out = torch.full((2, h, w, 4), float("nan"), device="cuda")
            smp = torch.full((2, h, w), -1, dtype=torch.int32, device="cuda")
            reqs.append(vr.make_request(vols[q].ptr, fr, cam, w, h, True, 1.0, 0.99, out,
                                        out_samples=smp))
            outs.append((out, smp))
            meta.append((q, fr, cam))
        tickets = []
        for k, r in enumerate(reqs):
            tickets.append(vr.vr_submit(ctx.ptr, r))
            if k % 5 == 4:
                time.sleep(0.002)  # the next burst arrives while these run
        t0 = time.time()
        infos = {}
        for t in tickets:
            while True:
                i = vr.vr_poll(ctx.ptr, t)
                if i.state >= 2:
                    infos[t] = i
                    break
                assert time.time() - t0 < 60.0, f"ticket {t} stuck"
                time.sleep(0.0002)
        assert all(infos[t].state == 2 for t in tickets)
        checked = rng.choice(len(reqs), size=8, replace=False)
        worst = 0.0
        for k in checked:
            q, fr, cam = meta[k]
            o, s = outs[k]
            served = (o.cpu().numpy(), s.cpu().numpy())
            # the served ticket reports the samples its request composited
            assert infos[tickets[k]].samples == int(served[1].sum())
            o.fill_(float("nan"))
            vr.vr_render(ctx.ptr, reqs[k], torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert np.array_equal(o.cpu().numpy().view(np.uint32), served[0].view(np.uint32))
            dims, ch, frames = specs[q]
            sc = Scene("c5", host_frame(sers[q].frame(fr)), 12, workloads.default_tfs(ch), cam,
                       reqs[k].width, reqs[k].height, True, 1.0, 0.99)
            pix = rng.choice(sc.width * sc.height, size=4096, replace=False)
            st = check_pixels(sc, served[0], served[1], pix, 1e-3)
            worst = max(worst, st["max_err_accept"])
        log(f"served mix: 8 of 40 requests x 2 x 4096 seeded pixels, max-abs error {worst:.2e}")
        for t in tickets:
            vr.vr_release(ctx.ptr, t)
    finally:
        for v in vols:
            v.destroy()


def test_precision_series_resident_against_oracle(ctx):
    import torch
    frames = 48
    dims, ser, tfs, cams = workloads.precision_setup(ctx, frames)
    vol = workloads.load_series(ctx, ser, frames, tfs)
    torch.cuda.synchronize()
    log(f"precision series resident: {vol.bytes / 1e9:.2f} GB")
    W, H = 1920, 1080
    rng = np.random.default_rng(33)
    worst = {vr.VR_FP32: 0.0, vr.VR_FP16: 0.0}
    accept = {vr.VR_FP32: 0.0, vr.VR_FP16: 0.0}
    try:
        for t in (0, 16, 32, 47):
            sc = Scene("precision", host_frame(ser.frame(t)), 8, tfs, cams[t], W, H, True,
                       1.0, 0.99)
            pix = rng.choice(W * H, size=1 << 14, replace=False)
            for prec, tol in ((vr.VR_FP32, 1e-3), (vr.VR_FP16, 4e-3)):
                out, smp = gpu.alloc_out(sc)
                req = gpu.request_for(vol, sc, out, smp, prec, frame=t)
                vr.vr_render(ctx.ptr, req, torch.cuda.current_stream())
                torch.cuda.synchronize()
                st = check_pixels(sc, out.cpu().numpy(), smp.cpu().numpy(), pix, tol)
                worst[prec] = max(worst[prec], st["max_err"])
                accept[prec] = max(accept[prec], st["max_err_accept"])
                log(f"frame {t} {'fp16' if prec else 'fp32'}: {st}")
    finally:
        vol.destroy()
    log(f"precision series (resident, 48 frames) max-abs RGBA error against the oracle, "
        f"every checked pixel against the oracle's own stop: fp32 {worst[vr.VR_FP32]:.3e} "
        f"fp16 {worst[vr.VR_FP16]:.3e}; against the nearest admissible stop: "
        f"fp32 {accept[vr.VR_FP32]:.3e} fp16 {accept[vr.VR_FP16]:.3e}")


@pytest.mark.parametrize("lit,prec", [(True, vr.VR_FP32), (False, vr.VR_FP16), (True, vr.VR_FP16)])
def test_realistic_frame_bench_configurations_against_oracle(ctx, lit, prec):
    """The realistic stereo pair at its full 1920x1080 per eye, in the
    configurations bench.py times beside the headline (lit, FP16 sampling),
    with the layout vr_tune_layout picks there: 2^14 seeded pixels per eye
    against the oracle."""
    import torch
    sc = synth.realistic_scene()
    if lit:
        sc.light = synth.Light((0.4, -0.3, -0.8), 0.3, 0.7)
    c, nz, ny, nx = sc.volume.shape
    src = torch.from_numpy(sc.volume.view(np.int16)).cuda()
    out, smp = gpu.alloc_out(sc)
    desc = vr.vr_volume_desc(nx, ny, nz, c, 1, vr.VR_U16, sc.bits, (vr.C.c_float * 3)(1, 1, 1),
                             (vr.C.c_float * 3)(0, 0, 0), (vr.C.c_int32 * 3)(0, 0, 0), 0)
    view = vr.make_request(None, 0, sc.cam, sc.width, sc.height, True, sc.step, sc.term_alpha,
                           out, sc.background, prec, smp, sc.light)
    vr.vr_tune_layout(ctx.ptr, desc, sc.tfs, src, [view], reps=3)
    v = vr.Volume(ctx, (nx, ny, nz), c, 1, vr.VR_U16, sc.bits, brick=tuple(desc.brick),
                  row_pairs=bool(desc.row_pairs))
    try:
        v.upload(0, src)
        for ch, tf in enumerate(sc.tfs):
            v.set_transfer(ch, tf)
        out, smp = gpu.alloc_out(sc)
        vr.vr_render(ctx.ptr, gpu.request_for(v, sc, out, smp, prec), torch.cuda.current_stream())
        torch.cuda.synchronize()
        rng = np.random.default_rng(71 + 2 * lit + prec)
        pix = rng.choice(sc.width * sc.height, size=1 << 14, replace=False)
        tol = 4e-3 if prec == vr.VR_FP16 else 1e-3
        st = check_pixels(sc, out.cpu().numpy(), smp.cpu().numpy(), pix, tol)
        log(f"realistic 1920x1080 lit={lit} {'fp16' if prec else 'fp32'} layout "
            f"{list(desc.brick)} pairs={desc.row_pairs}: {st}")
    finally:
        v.destroy()
