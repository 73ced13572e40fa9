"""GPU parity at the documented limits: frames larger than 2 GiB (byte
offsets above 2^31 in the 32-bit buffer addressing), frames above 4 GiB and
axes of 16384 voxels (large-volume addressing), the longest axis of the
32-bit path (8192 voxels) and the widest and tallest images (16384
pixels)."""
import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
import scenes
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Cam, Scene

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


COEF = ((16, 16, 32, 7), (3, 29, 41, 1000))  # per channel: a i + b j + c k + d < 2^16


def linear_2ch(nx, ny, nz, coef=COEF):
    """Two-channel linear uint16 field, built on the GPU, [C][Z][Y][X]."""
    import torch
    i = torch.arange(nx, device="cuda", dtype=torch.int32)
    j = torch.arange(ny, device="cuda", dtype=torch.int32)
    k = torch.arange(nz, device="cuda", dtype=torch.int32)
    chans = []
    for a, b, c, d in coef:
        v = a * i[None, None, :] + b * j[None, :, None] + c * k[:, None, None] + d
        chans.append((v - 65536 * (v >= 32768).to(torch.int32)).to(torch.int16))  # uint16 bits
    return torch.stack(chans).contiguous()


@pytest.mark.parametrize("row_pairs,dims", [(False, (1024, 1024, 512)), (True, (1024, 1024, 256))])
def test_frame_above_2_gib(ctx, row_pairs, dims):
    """A frame of 2.1-4.3 GB: samples whose taps lie past byte 2^31 of the
    frame reproduce the linear field exactly (as on small volumes)."""
    import torch
    nx, ny, nz = dims
    v = vr.Volume(ctx, dims, 2, 1, vr.VR_U16, 16, row_pairs=row_pairs)
    frame_bytes = v.bytes
    assert 2 ** 31 < frame_bytes < 2 ** 32, frame_bytes
    try:
        v.upload(0, linear_2ch(nx, ny, nz))
        torch.cuda.synchronize()
        rng = np.random.default_rng(1)
        n = 1 << 16
        # the last quarter of the z range lies past 2^31 bytes in brick order
        lo = np.array([0, 0, 0.75 * (nz - 1)])
        hi = np.array([nx - 1, ny - 1, nz - 1])
        pts = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
        pts[:8] = [[nx - 1, ny - 1, nz - 1], [0, 0, nz - 1], [nx - 1, 0, nz - 1],
                   [0, ny - 1, nz - 1], [nx - 1.5, ny - 1.5, nz - 1.5], [nx / 2, ny / 2, nz - 1],
                   [0, 0, 0], [nx - 1, ny - 1, 0]]
        out = torch.zeros(n * 2, dtype=torch.float32, device="cuda")
        vr.vr_debug_sample(v.ptr, 0, torch.from_numpy(pts).cuda(), n, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(n, 2).astype(np.float64)
        p = pts.astype(np.float64)
        for c, (a, b, g, d) in enumerate(COEF):
            exp = a * p[:, 0] + b * p[:, 1] + g * p[:, 2] + d
            np.testing.assert_allclose(got[:, c], exp, rtol=2e-6, atol=0)
    finally:
        v.destroy()


def test_2_to_the_24_bricks(ctx):
    """2048 x 2048 x 255 uint8 voxels in 4 x 4 x 4 bricks: 513 x 513 x 64
    bricks (above 2^24) in a 2.1 GB frame (under 2^31 words).  The volume
    takes the large-volume addressing, and samples in the last brick layer,
    whose brick indices pass 2^24, reproduce the field v = k (a brick index
    wrapped modulo 2^24 would read the first layer's values instead)."""
    import torch
    nx, ny, nz = dims = (2048, 2048, 255)
    v = vr.Volume(ctx, dims, 1, 1, vr.VR_U8, 8, brick=(4, 4, 4))
    assert v.bytes < 2 ** 31
    try:
        assert vr.vr_test_volume_large(v.ptr)
        k = torch.arange(nz, device="cuda", dtype=torch.uint8)
        src = k[None, :, None, None].expand(1, nz, ny, nx).contiguous()
        v.upload(0, src)
        del src
        torch.cuda.synchronize()
        rng = np.random.default_rng(3)
        n = 1 << 16
        # brick (bx, by, 63) has index >= 2^24 once 513 by + bx >= 197569
        lo = np.array([0, 1560, 251.5])
        hi = np.array([nx - 1, ny - 1, nz - 1])
        pts = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
        pts[:2] = [[nx - 1, ny - 1, nz - 1], [0, ny - 1, nz - 1.5]]
        out = torch.zeros(n, dtype=torch.float32, device="cuda")
        vr.vr_debug_sample(v.ptr, 0, torch.from_numpy(pts).cuda(), n, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, pts[:, 2].astype(np.float64), rtol=2e-6, atol=0)
    finally:
        v.destroy()


COEF_4G = ((16, 16, 32, 7), (3, 29, 30, 1000))  # < 2^16 on 1024 x 1024 x 800


def test_frame_above_4_gib(ctx):
    """A frame of 4.5 GB (two uint16 channels, 1024 x 1024 x 800): samples
    whose taps lie past byte 2^32 of the frame reproduce the linear field, and
    a stereo render through the whole depth matches the oracle."""
    import torch
    nx, ny, nz = dims = (1024, 1024, 800)
    v = vr.Volume(ctx, dims, 2, 1, vr.VR_U16, 16)
    assert v.bytes > 2 ** 32, v.bytes
    try:
        src = linear_2ch(nx, ny, nz, COEF_4G)
        v.upload(0, src)
        torch.cuda.synchronize()
        rng = np.random.default_rng(2)
        n = 1 << 16
        lo = np.array([0, 0, 0.8 * (nz - 1)])  # past 2^32 bytes in brick order
        hi = np.array([nx - 1, ny - 1, nz - 1])
        pts = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
        pts[:4] = [[nx - 1, ny - 1, nz - 1], [0, 0, nz - 1], [nx - 1.5, ny - 1.5, nz - 1.5],
                   [nx / 2, ny / 2, nz - 1]]
        out = torch.zeros(n * 2, dtype=torch.float32, device="cuda")
        vr.vr_debug_sample(v.ptr, 0, torch.from_numpy(pts).cuda(), n, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(n, 2).astype(np.float64)
        p = pts.astype(np.float64)
        for c, (a, b, g, d) in enumerate(COEF_4G):
            exp = a * p[:, 0] + b * p[:, 1] + g * p[:, 2] + d
            np.testing.assert_allclose(got[:, c], exp, rtol=2e-6, atol=0)
        host = src.cpu().numpy().view(np.uint16)
        del src
        tfs = [TF(0.55, 0.95, 0.0, 0.03, (0.0, 1.0, 0.0)), TF(0.4, 0.9, 0.3, 0.03, (1.0, 0.0, 1.0))]
        for c, tf in enumerate(tfs):
            v.set_transfer(c, tf)
        cam = synth.orbit_camera(dims, 30.0, 50.0, 40.0, stereo=True)
        sc = Scene("4gib", host, 16, tfs, cam, 24, 18, True, 2.0, 0.99)
        out, smp = gpu.alloc_out(sc)
        vr.vr_render(ctx.ptr, gpu.request_for(v, sc, out, smp), torch.cuda.current_stream())
        torch.cuda.synchronize()
        rgba, smp = out.cpu().numpy(), smp.cpu().numpy()
        gpu.compare(rgba, smp, orc.render_all(sc), 1e-3)
        assert float(rgba[..., 3].max()) > 0.1 and int(smp.max()) > 300
    finally:
        v.destroy()


@pytest.mark.parametrize("length", [8192, 16384])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_longest_axis(ctx, axis, length):
    """Volumes 8192 (32-bit path) and 16384 (large-volume path) voxels long
    along one axis, viewed along and across it."""
    n = [3, 4, 2]
    n[axis] = length
    nx, ny, nz = n
    vol = scenes.random_volume(40 + axis, (1, nz, ny, nx), np.uint8)
    c = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    fwd = [0.0, 0.0, 0.0]
    fwd[axis] = 1.0
    up = (0.0, 0.0, 1.0) if axis != 2 else (0.0, 1.0, 0.0)
    along = Cam("ortho", c, tuple(fwd), up, ortho_height=6.0)
    across = synth.orbit_camera((nx, ny, nz), 20.0 + 30 * axis, 30.0, 40.0, stereo=True)
    for cam, stereo, tau in ((along, False, 1.0), (across, True, 0.99)):
        sc = Scene("long", vol, 8, [TF(0.2, 0.9, 0.0, 0.05)], cam, 16, 12, stereo, 1.0, tau)
        rgba, smp = gpu.render(ctx, sc)
        gpu.compare(rgba, smp, orc.render_all(sc), 1e-3)


@pytest.mark.parametrize("w,h", [(16384, 2), (2, 16384)])
def test_widest_and_tallest_images(ctx, w, h):
    nx, ny, nz = 20, 18, 12
    vol = scenes.random_volume(77, (2, nz, ny, nx), np.uint16, 4096)
    cam = synth.orbit_camera((nx, ny, nz), 35.0, 25.0, 45.0)
    sc = Scene("wide", vol, 12, [TF(0.1, 0.8), TF(0.3, 0.9, 0.2, 1.5, (0, 1, 0))], cam, w, h,
               True, 0.8, 0.995)
    rgba, smp = gpu.render(ctx, sc)
    gpu.compare(rgba, smp, orc.render_all(sc), 1e-3)


# ------------------------------------------------------- the montage frame

def oracle_pixels_on_crops(src, sc, eye, pixels):
    """Oracle results of single pixels of one eye, each rendered on its ray's
    crop of the device volume `src` [C][Z][Y][X]."""
    import oracle
    from oracle.crop import ray_crop
    res = []
    for pix in pixels:
        px, py = int(pix) % sc.width, int(pix) // sc.width
        box = ray_crop(sc.cam, sc.width, sc.height, eye, px, py,
                       (src.shape[3], src.shape[2], src.shape[1]))
        lo, hi = box if box is not None else (np.zeros(3, int), np.ones(3, int))
        crop = src[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        vol = oracle.Volume(crop, sc.bits, (1.0, 1.0, 1.0), tuple(float(x) for x in lo))
        res.append(oracle.render(vol, orc.transfers(sc.tfs), orc.camera(sc.cam), sc.width,
                                 sc.height, eye, sc.step, sc.term_alpha, 1e-3, sc.background,
                                 [int(pix)], 1, None))
    return orc.concat(res)


@pytest.fixture(scope="module")
def montage(ctx):
    """The five-channel 10173 x 3858 x 74 uint8 montage (one frame, 33 GB of
    bricks, large-volume addressing) and its source."""
    import torch
    from paper_1407_2089_amd import workloads
    vol, src, tfs = workloads.montage_setup(ctx)
    torch.cuda.synchronize()
    yield vol, src, tfs
    vol.destroy()


@pytest.mark.parametrize("view", ["bench", "top"])
def test_montage_sampled_pixels_match_the_oracle(ctx, montage, view):
    """Full-size montage renders (the benchmark's stereo 1920 x 1080 view, and
    an orthographic top view): seeded pixels, half of them on rays that take
    samples, against the oracle on each ray's crop."""
    import torch
    from paper_1407_2089_amd import workloads
    vol, src, tfs = montage
    nx, ny, nz = workloads.MONTAGE_DIMS
    if view == "bench":
        cam, W, H, stereo = workloads.montage_camera(), 1920, 1080, True
    else:
        cam = Cam("ortho", ((nx - 1) / 2, (ny - 1) / 2, nz + 10.0), (0.0, 0.0, -1.0),
                  (0.0, 1.0, 0.0), ortho_height=float(ny))
        W, H, stereo = 2637, 1000, False
    sc = Scene("montage", None, 8, tfs, cam, W, H, stereo, 1.0, 0.99)
    out, smp = gpu.alloc_out(sc)
    vr.vr_render(ctx.ptr, gpu.request_for(vol, sc, out, smp), torch.cuda.current_stream())
    torch.cuda.synchronize()
    rgba, smp = out.cpu().numpy(), smp.cpu().numpy()
    assert np.isfinite(rgba).all() and (smp >= 0).all()
    rng = np.random.default_rng(17)
    for e, eye in enumerate(orc.eyes(sc)):
        s = smp[e].reshape(-1)
        hit = np.flatnonzero(s > 0)
        assert hit.size > W * H // 10
        pix = np.concatenate([rng.choice(hit, 24, replace=False),
                              rng.choice(W * H, 24, replace=False), [0, W * H - 1]])
        print(f"montage {view} eye {eye}: {hit.size} rays hit, max {int(s.max())} samples",
              flush=True)
        ref = oracle_pixels_on_crops(src, sc, eye, pix)
        gpu.compare(rgba[e].reshape(-1, 4)[pix], s[pix], ref, 1e-3)
    assert float(rgba[..., 3].max()) > 0.3
