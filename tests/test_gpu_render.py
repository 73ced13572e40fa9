"""GPU parity: libvr (HIP, gfx950) against the FP64 oracle and the closed
forms, through the C ABI.  FP32 tolerance 1e-3, FP16 sampling 4e-3 (max abs
RGBA error), with the termination-band acceptance rule of tests/gpu.py."""
import math

import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
import scenes
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Cam, Scene

pytestmark = pytest.mark.gpu
TOL32, TOL16 = 1e-3, 4e-3


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    c = vr.Context(0)
    yield c
    try:
        c.close()
    except vr.VrError:
        pass  # a failed test may leave volumes alive


@pytest.fixture(scope="module")
def realistic():
    return synth.realistic_scene()


def log(msg):
    print(msg, flush=True)


# ------------------------------------------------------------ sampling

@pytest.mark.parametrize("brick", [(4, 4, 4), (8, 8, 8), (16, 16, 16), (32, 32, 32),
                                   (8, 16, 4), (32, 4, 16)])
def test_linear_field_and_voxel_centres(ctx, brick):
    import torch
    log(f"linear field brick {brick}")
    nx, ny, nz = 37, 29, 21
    coef = (3, 5, 7, 11)
    data = scenes.linear_field(nx, ny, nz, coef)
    sc = Scene("lin", data, 16, [TF()], scenes.ortho_down_z(nx, ny, 8, 8, 8.0), 8, 8,
               False, 1.0, 1.0)
    v = gpu.make_volume(ctx, sc, brick)
    rng = np.random.default_rng(3)
    pts = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(4096, 3))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    centres = np.stack([i.ravel(), j.ravel(), k.ravel()], -1)
    allp = np.concatenate([pts, centres]).astype(np.float32)
    d_pts = torch.from_numpy(allp).cuda()
    out = torch.zeros(allp.shape[0], dtype=torch.float32, device="cuda")
    vr.vr_debug_sample(v.ptr, 0, d_pts, allp.shape[0], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    p = allp.astype(np.float64)
    exp = coef[0] * p[:, 0] + coef[1] * p[:, 1] + coef[2] * p[:, 2] + coef[3]
    np.testing.assert_allclose(got[:4096], exp[:4096], rtol=1e-6, atol=0)
    assert np.array_equal(got[4096:], data.reshape(-1).astype(np.float64))
    v.destroy()


SAMPLER_CASES = [(1, np.uint8, 8, False), (2, np.uint8, 8, False), (3, np.uint8, 8, False),
                 (4, np.uint8, 8, False), (1, np.uint16, 16, False), (2, np.uint16, 12, False),
                 (3, np.uint16, 12, False), (4, np.uint16, 16, False),
                 (3, np.uint8, 8, True), (4, np.uint8, 8, True), (2, np.uint16, 12, True),
                 (2, np.uint16, 16, True), (1, np.uint8, 8, True), (2, np.uint8, 8, True),
                 (1, np.uint16, 16, True), (5, np.uint8, 8, False), (6, np.uint8, 8, False),
                 (5, np.uint16, 12, False), (6, np.uint16, 16, False)]


@pytest.mark.parametrize("ch,dtype,bits,row_pairs", SAMPLER_CASES)
def test_sampler_matches_oracle_everywhere_in_box(ctx, ch, dtype, bits, row_pairs):
    import oracle
    import torch
    log(f"sampler ch={ch} {dtype.__name__} row_pairs={row_pairs}")
    nx, ny, nz = 19, 13, 11
    data = scenes.random_volume(ch, (ch, nz, ny, nx), dtype, 1 << bits)
    sc = Scene("rnd", data, bits, [TF()] * ch, scenes.ortho_down_z(nx, ny, 8, 8, 8.0), 8, 8,
               False, 1.0, 1.0)
    v = gpu.make_volume(ctx, sc, (8, 4, 8), row_pairs=row_pairs)
    rng = np.random.default_rng(ch)
    pts = rng.uniform([-1, -1, -1], [nx, ny, nz], size=(8192, 3)).astype(np.float32)
    # faces and corners of the extended box
    pts[:6] = [[-1, 3, 3], [nx, 3, 3], [4, -1, 2], [4, ny, 2], [5, 5, -1], [5, 5, nz]]
    d_pts = torch.from_numpy(pts).cuda()
    out = torch.zeros(pts.shape[0] * ch, dtype=torch.float32, device="cuda")
    vr.vr_debug_sample(v.ptr, 0, d_pts, pts.shape[0], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(-1, ch)
    exp = oracle.sample(orc.volume(sc), pts.astype(np.float64))
    np.testing.assert_allclose(got, exp, rtol=0, atol=2e-6 * (1 << bits))
    # faces of [-1, n]: exactly 0 on the lower faces; an upper face is
    # evaluated one float step inside it (at the largest float below n + 1 in
    # stored coordinates), where the field is at most that step times full scale
    assert np.all(got[[0, 2, 4]] == 0)
    for row, n in zip((1, 3, 5), (nx, ny, nz)):
        step = float(np.spacing(np.float32(n + 1)))
        assert np.all(np.abs(got[row]) <= 1.01 * step * ((1 << bits) - 1))
    v.destroy()


# ------------------------------------------------------- whole workloads

def test_tiny_workload_full_frame(ctx):
    log("tiny workload")
    sc = synth.tiny_scene()
    rgba, smp = gpu.render(ctx, sc)
    ref = orc.render_all(sc)
    st = gpu.compare(rgba, smp, ref, TOL32)
    log(f"tiny stats {st}")
    # with tau = 1, FP32 opacity may round to exactly 1 on near-opaque rays
    # (inside the band); every other ray takes exactly the oracle's samples
    assert st["count_exact"] >= st["pixels"] - st["band_pixels"]


def test_realistic_stereo_pair_full_frame(ctx, realistic):
    log("realistic stereo 1920x1080")
    rgba, smp = gpu.render(ctx, realistic)
    ref = orc.render_all(realistic)
    st = gpu.compare(rgba, smp, ref, TOL32)
    log(f"realistic stats {st}")
    assert st["count_exact"] >= 0.999 * st["pixels"]


@pytest.mark.parametrize("w,h", [(37, 29), (1, 1), (200, 3), (3, 130), (64, 64)])
def test_ragged_sizes_stereo(ctx, w, h):
    log(f"ragged {w}x{h}")
    nx, ny, nz = 45, 38, 27
    vol = scenes.random_volume(11, (2, nz, ny, nx), np.uint16, 4096)
    cam = synth.orbit_camera((nx, ny, nz), 70.0, 25.0, 40.0)
    tfs = [TF(0.1, 0.9, 0.4, 0.3, (0.2, 0.8, 0.4)), TF(0.3, 0.95, -0.5, 0.7, (1.0, 0.2, 0.1))]
    sc = Scene("ragged", vol, 12, tfs, cam, w, h, True, 0.7, 0.97, (0.1, 0.2, 0.3, 0.4))
    rgba, smp = gpu.render(ctx, sc)
    assert not np.isnan(rgba).any() and (smp >= 0).all()
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)


def test_empty_image_is_a_no_op(ctx):
    import torch
    sc = synth.tiny_scene()
    v = gpu.make_volume(ctx, sc)
    req = vr.make_request(v.ptr, 0, sc.cam, 0, 0, False, 0.5, 1.0, None)
    vr.vr_render(ctx.ptr, req)
    vr.vr_render_batch(ctx.ptr, [req, req])
    torch.cuda.synchronize()
    v.destroy()


def test_rays_that_miss_return_background(ctx):
    sc = synth.tiny_scene()
    away = Cam("perspective", (31.5, 31.5, -50.0), (0, 0, -1), (0, -1, 0), 0.5, 1, 2.0, 50.0)
    s2 = Scene("miss", sc.volume, 8, sc.tfs, away, 40, 30, True, 0.5, 1.0, (0.3, 0.2, 0.1, 0.6))
    rgba, smp = gpu.render(ctx, s2)
    assert (smp == 0).all()
    f = np.float32  # the request carries float32 background components
    bg = [float(f(x)) for x in (0.3, 0.2, 0.1, 0.6)]
    exp = np.array([bg[3] * bg[0], bg[3] * bg[1], bg[3] * bg[2], bg[3]], np.float32)
    assert np.array_equal(rgba.reshape(-1, 4), np.broadcast_to(exp, (2 * 40 * 30, 4)))


def test_single_voxel_volume(ctx):
    vol = np.full((1, 1, 1, 1), 180, np.uint8)
    cam = synth.orbit_camera((1, 1, 1), 20.0, 30.0, 50.0)
    sc = Scene("one", vol, 8, [TF(0.0, 1.0, 0.0, 1.5, (1.0, 0.5, 0.0))], cam, 33, 17, True,
               0.1, 1.0)
    rgba, smp = gpu.render(ctx, sc)
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)
    assert rgba[..., 3].max() > 0.1


# ---------------------------------------------------------- pins on GPU

def test_p1_empty_volume_bitwise_background(ctx):
    vol = np.zeros((2, 12, 10, 14), np.uint16)
    bg = (0.2, 0.3, 0.4, 0.5)
    sc = Scene("p1", vol, 12, [TF(), TF(0.1, 0.9, 0.5)], scenes.mirror_camera(14, 10, 12), 21,
               13, True, 0.7, 0.95, bg)
    rgba, _ = gpu.render(ctx, sc)
    exp = np.array([bg[3] * bg[0], bg[3] * bg[1], bg[3] * bg[2], bg[3]], np.float32)
    assert np.array_equal(rgba.reshape(-1, 4), np.broadcast_to(exp, (rgba.size // 4, 4)))


@pytest.mark.parametrize("dtype,bits,v", [(np.uint8, 8, 200), (np.uint16, 12, 2500)])
def test_p2_slab_closed_form_on_gpu(ctx, dtype, bits, v):
    sc = scenes.slab_scene(dtype, bits, v, z_a=5, z_b=15)
    exp, a, _ = scenes.slab_closed_form(sc, v, 5, 15)
    rgba, smp = gpu.render(ctx, sc)
    np.testing.assert_allclose(rgba.reshape(-1, 4), np.broadcast_to(exp, (64, 4)), atol=2e-6)
    assert (smp == sc.volume.shape[1] + 1).all()


def test_p2_slab_termination_count_on_gpu(ctx):
    sc = scenes.slab_scene(alpha_mul=1.0, curve=0.0, term_alpha=0.9, z_a=3, z_b=20, nz=26)
    exp, a, stop = scenes.slab_closed_form(sc, 200, 3, 20)
    rgba, smp = gpu.render(ctx, sc)
    assert (smp == stop).all()
    np.testing.assert_allclose(rgba.reshape(-1, 4), np.broadcast_to(exp, (64, 4)), atol=2e-6)


def test_p4_mirror_stereo_on_gpu(ctx):
    nx, ny, nz = 33, 24, 20
    vol = scenes.mirror_volume(4, nx, ny, nz)
    tfs = [TF(0.1, 0.9, 0.2, 0.6, (0.2, 0.9, 0.1)), TF(0.3, 0.8, -0.4, 1.3, (0.9, 0.1, 0.5))]
    sc = Scene("p4", vol, 8, tfs, scenes.mirror_camera(nx, ny, nz, 3.0), 40, 30, True, 0.8, 1.0)
    rgba, smp = gpu.render(ctx, sc)
    np.testing.assert_allclose(rgba[0], rgba[1][:, ::-1], atol=1e-4)
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)


def test_p6_opaque_first_sample_on_gpu(ctx):
    vol = np.full((1, 6, 8, 8), 255, np.uint8)
    sc = Scene("p6", vol, 8, [TF(0.0, 0.5, 0.0, 1.0, (0.3, 0.6, 0.9))],
               scenes.ortho_down_z(8, 8, 4, 4, 4.0), 4, 4, False, 1.0, 1.0)
    rgba, smp = gpu.render(ctx, sc)
    assert (smp == 1).all()
    np.testing.assert_allclose(rgba.reshape(-1, 4), np.broadcast_to([0.3, 0.6, 0.9, 1.0],
                                                                     (16, 4)), atol=1e-7)


def test_p7_channel_permutation_on_gpu(ctx):
    nx, ny, nz = 18, 15, 12
    vol = scenes.random_volume(7, (4, nz, ny, nx), np.uint16, 4096)
    tfs = [TF(0.1, 0.8, 0.3, 0.7, (1, 0, 0)), TF(0.2, 0.9, -0.5, 1.5, (0, 1, 0)),
           TF(0.05, 0.6, 0.0, 0.3, (0, 0, 1)), TF(0.3, 0.7, 1.0, 2.0, (1, 1, 0))]
    sc = Scene("p7", vol, 12, tfs, scenes.mirror_camera(nx, ny, nz, 2.0), 16, 12, True, 0.9,
               0.95)
    base, _ = gpu.render(ctx, sc)
    perm = [2, 0, 3, 1]
    sc2 = Scene("p7p", np.ascontiguousarray(vol[perm]), 12, [tfs[p] for p in perm], sc.cam, 16,
                12, True, 0.9, 0.95)
    got, _ = gpu.render(ctx, sc2)
    np.testing.assert_allclose(got, base, atol=1e-6)


# --------------------------------------------------------- layouts

@pytest.mark.parametrize("ch,dtype,bits", [(3, np.uint8, 8), (4, np.uint8, 8), (2, np.uint16, 12),
                                           (2, np.uint16, 16), (1, np.uint8, 8), (2, np.uint8, 8),
                                           (1, np.uint16, 12)])
@pytest.mark.parametrize("brick", [(0, 0, 0), (4, 8, 16), (16, 4, 8), (32, 32, 4)])
def test_row_pair_layout_gives_the_same_images(ctx, ch, dtype, bits, brick):
    """Row pairs change where the taps are stored, not their values: images
    and sample counts are bitwise those of the default layout, FP32 and FP16."""
    nx, ny, nz = 45, 38, 27
    vol = np.zeros((ch, nz, ny, nx), dtype)
    for c in range(ch):
        vol[c] = synth.cells_and_vessels((nx, ny, nz), 1, bits, 30 + c, n_cells=6, n_tubes=2)[0]
    tfs = [TF(0.08 + 0.03 * c, 0.8, 0.1 * c, 1.0, (1.0 - 0.2 * c, 0.3 * c, 0.5)) for c in range(ch)]
    cam = synth.orbit_camera((nx, ny, nz), 35.0 + 20 * ch, 25.0, 45.0)
    sc = Scene("pairs", vol, bits, tfs, cam, 70, 52, True, 0.9, 0.99)
    for precision in (vr.VR_FP32, vr.VR_FP16):
        a = gpu.render(ctx, sc, precision, brick)
        b = gpu.render(ctx, sc, precision, brick, row_pairs=True)
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))


@pytest.mark.parametrize("brick", [(4, 4, 4), (16, 16, 16), (32, 32, 32), (16, 16, 4)])
def test_brick_shape_does_not_change_the_image(ctx, realistic, brick):
    sc = Scene("small", realistic.volume[:, :32, :160, :192].copy(), 12, realistic.tfs,
               synth.orbit_camera((192, 160, 32), 30.0, 50.0, 45.0), 160, 96, True, 1.0, 0.99)
    a, sa = gpu.render(ctx, sc, brick=(0, 0, 0))
    b, sb = gpu.render(ctx, sc, brick=brick)
    assert np.array_equal(a, b) and np.array_equal(sa, sb)


# ------------------------------------------------ spacing, frames, clamping

def test_anisotropic_spacing_and_origin(ctx):
    # confocal stacks: 0.8 um pixels, 1 um z steps (Methods, acquisition)
    nx, ny, nz = 48, 40, 20
    vol = synth.cells_and_vessels((nx, ny, nz), 2, 12, 31, n_cells=5, n_tubes=2)
    spacing, origin = (0.8, 0.8, 1.0), (-10.0, 5.0, 3.0)
    ext = np.array([nx * 0.8, ny * 0.8, nz * 1.0])
    centre = np.array(origin) + ext / 2
    eye = centre + np.array([30.0, -55.0, 40.0])
    fwd = centre - eye
    dist = float(np.linalg.norm(fwd))
    cam = Cam("perspective", tuple(eye), tuple(fwd / dist), (0, 0, 1), math.radians(35), 1.0,
              dist / 30, dist)
    tfs = [TF(0.05, 0.6, 0.2, 1.2, (0, 1, 0)), TF(0.08, 0.7, -0.3, 0.9, (1, 0, 0))]
    sc = Scene("aniso", vol, 12, tfs, cam, 96, 72, True, 0.6, 0.99, spacing=spacing,
               origin=origin)
    rgba, smp = gpu.render(ctx, sc)
    assert rgba[..., 3].max() > 0.2
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)


def test_time_series_frames_are_independent(ctx):
    import torch
    nx, ny, nz = 30, 26, 14
    frames = [scenes.random_volume(40 + t, (2, nz, ny, nx), np.uint8) for t in range(3)]
    cam = synth.orbit_camera((nx, ny, nz), 40.0, 30.0, 40.0)
    tfs = [TF(0.2, 0.9, 0.0, 0.5, (0, 1, 0)), TF(0.3, 0.8, 0.5, 0.7, (1, 0, 1))]
    v = vr.Volume(ctx, (nx, ny, nz), 2, 3, vr.VR_U8, 8)
    try:
        for t in (2, 0, 1):  # any upload order
            v.upload(t, gpu.to_device(frames[t]))
        for c, tf in enumerate(tfs):
            v.set_transfer(c, tf)
        for t in range(3):
            sc = Scene("series", frames[t], 8, tfs, cam, 40, 30, True, 0.8, 0.98)
            out, smp = gpu.alloc_out(sc)
            vr.vr_render(ctx.ptr, gpu.request_for(v, sc, out, smp, frame=t),
                         torch.cuda.current_stream())
            torch.cuda.synchronize()
            gpu.compare(out.cpu().numpy(), smp.cpu().numpy(), orc.render_all(sc), TOL32)
    finally:
        v.destroy()


def test_values_above_the_bit_depth_are_clamped(ctx):
    nx, ny, nz = 24, 20, 12
    raw = scenes.random_volume(50, (1, nz, ny, nx), np.uint16, 65536)  # up to 65535
    clamped = np.minimum(raw, 4095).astype(np.uint16)
    cam = synth.orbit_camera((nx, ny, nz), 10.0, 60.0, 40.0)
    sc = Scene("clamp", raw, 12, [TF(0.3, 0.9)], cam, 32, 24, True, 0.7, 1.0)
    rgba, smp = gpu.render(ctx, sc)
    ref = orc.render_all(Scene("clamp", clamped, 12, [TF(0.3, 0.9)], cam, 32, 24, True, 0.7,
                               1.0))
    gpu.compare(rgba, smp, ref, TOL32)


def test_invisible_channel_and_oblique_orthographic_view(ctx):
    nx, ny, nz = 36, 28, 18
    vol = scenes.random_volume(60, (3, nz, ny, nx), np.uint8)
    tfs = [TF(0.1, 0.8, 0.0, 0.4, (1, 0, 0)), TF(0.0, 1.0, 0.0, 2.0, (0, 1, 0), visible=False),
           TF(0.2, 0.9, 0.6, 0.6, (0, 0, 1))]
    c = ((nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2)
    cam = Cam("ortho", c, (0.4, -0.5, 0.77), (0, 0, 1), ortho_height=40.0)
    sc = Scene("ortho", vol, 8, tfs, cam, 50, 40, False, 0.5, 0.995, (0.1, 0.1, 0.1, 1.0))
    rgba, smp = gpu.render(ctx, sc)
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)
    # the invisible channel contributes nothing: zeroing it changes no pixel
    vol2 = vol.copy()
    vol2[1] = 0
    rgba2, _ = gpu.render(ctx, Scene("ortho", vol2, 8, tfs, cam, 50, 40, False, 0.5, 0.995,
                                     (0.1, 0.1, 0.1, 1.0)))
    assert np.array_equal(rgba, rgba2)


LAYOUTS = [((4, 4, 4), False), ((4, 16, 8), False), ((8, 8, 8), False), ((16, 4, 4), False),
           ((32, 8, 4), False), ((4, 4, 4), True), ((8, 16, 8), True), ((16, 4, 32), True)]


@pytest.mark.parametrize("ch,dtype", [(1, np.uint8), (2, np.uint16), (4, np.uint8), (5, np.uint8),
                                      (6, np.uint16)])
def test_relayout_forms_store_the_same_voxels(ctx, ch, dtype):
    # Bricks 4 voxels wide take the scatter form of the relayout, wider ones
    # the gather form; with and without row pairs.  Sampling the same points
    # must give the same values bit for bit in every layout (the taps and
    # the interpolation arithmetic do not depend on the layout).
    import torch
    nx, ny, nz = 37, 29, 23
    bits = 8 if dtype == np.uint8 else 12
    vol = scenes.random_volume(90 + ch, (ch, nz, ny, nx), dtype, 1 << bits)
    rng = np.random.default_rng(ch)
    n = 4096
    pts = torch.from_numpy(rng.uniform([-1, -1, -1], [nx, ny, nz], size=(n, 3))
                           .astype(np.float32)).cuda()
    word = {1: 1, 2: 2, 3: 4, 4: 4, 5: 8, 6: 8}[ch] * (2 if dtype == np.uint16 else 1)
    got = []
    for brick, pairs in LAYOUTS:
        if pairs and word > 4:
            continue
        v = vr.Volume(ctx, (nx, ny, nz), ch, 1, vr.VR_U8 if dtype == np.uint8 else vr.VR_U16,
                      bits, brick=brick, row_pairs=pairs)
        try:
            v.upload(0, gpu.to_device(vol))
            out = torch.zeros(n * ch, dtype=torch.float32, device="cuda")
            vr.vr_debug_sample(v.ptr, 0, pts, n, out)
            torch.cuda.synchronize()
            got.append(out.cpu().numpy().view(np.uint32))
        finally:
            v.destroy()
    assert len(got) >= 5
    for g in got[1:]:
        assert np.array_equal(g, got[0])
