"""GPU parity at the documented limits: frames larger than 2 GiB (byte
offsets above 2^31 in the 32-bit buffer addressing), the longest volume axis
(8192 voxels) and the widest and tallest images (16384 pixels)."""
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


def linear_2ch(nx, ny, nz):
    """Two-channel linear uint16 field, built on the GPU, [C][Z][Y][X]."""
    import torch
    i = torch.arange(nx, device="cuda", dtype=torch.int32)
    j = torch.arange(ny, device="cuda", dtype=torch.int32)
    k = torch.arange(nz, device="cuda", dtype=torch.int32)
    chans = []
    for a, b, c, d in COEF:
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


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_longest_axis_8192(ctx, axis):
    """Volumes 8192 voxels long along one axis, viewed along and across it."""
    n = [3, 4, 2]
    n[axis] = 8192
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
