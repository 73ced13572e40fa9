"""Seeded random configurations against the FP64 oracle: volume shape, channel
count, voxel type and bit depth, brick shape and row pairs, spacing and
origin, camera (perspective stereo or orthographic mono, any direction),
transfer functions (floor, ceiling, curve, multiplier, colour, visibility),
step, termination threshold, background and sampling precision.  Each case
must pass the acceptance rule and render the same bits with the
transparent-sample skip on and off."""

import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Cam, Scene

pytestmark = pytest.mark.gpu

EDGES = (4, 8, 16, 32)


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


def random_case(seed):
    rng = np.random.default_rng(10_000 + seed)
    nx, ny, nz = (int(rng.integers(1, 41)) for _ in range(3))
    ch = int(rng.integers(1, 7))
    u16 = bool(rng.integers(0, 2))
    bits = int(rng.integers(9, 17)) if u16 else 8
    dtype = np.uint16 if u16 else np.uint8
    full = (1 << bits) - 1
    # smooth blobs plus noise, so that floors fall inside the data
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = np.zeros((ch, nz, ny, nx), np.float64)
    for c in range(ch):
        for _ in range(int(rng.integers(1, 4))):
            cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
            s = rng.uniform(1.0, 6.0)
            vol[c] += rng.uniform(0.3, 1.0) * full * np.exp(
                -((i - cx) ** 2 + (j - cy) ** 2 + (k - cz) ** 2) / (2 * s * s))
        vol[c] += rng.uniform(0, 0.08 * full, size=(nz, ny, nx))
    vol = np.clip(np.rint(vol), 0, full).astype(dtype)
    word = {1: 1, 2: 2, 3: 4, 4: 4, 5: 8, 6: 8}[ch] * (2 if u16 else 1)
    pairs = word <= 4 and bool(rng.integers(0, 2))
    brick = (0, 0, 0) if rng.integers(0, 3) == 0 else tuple(int(rng.choice(EDGES)) for _ in range(3))
    spacing = tuple(float(x) for x in rng.uniform(0.5, 2.0, 3))
    origin = tuple(float(x) for x in rng.uniform(-5, 5, 3))
    precision = vr.VR_FP16 if rng.integers(0, 3) == 0 else vr.VR_FP32
    # FP16 rounds a normalised value x by up to 2^-11 x; the transfer function
    # scales that by up to 2 / (hi - lo) (curve slope) times the multiplier,
    # so FP16 cases keep windows of 0.4 and more and multipliers up to 1.
    fp16 = precision == vr.VR_FP16
    min_window, max_mul = (0.4, 1.0) if fp16 else (0.02, 2.0)
    tfs = []
    for c in range(ch):
        lo = float(rng.uniform(0.0, 0.6))
        hi = float(min(1.0, lo + rng.uniform(min_window, 0.8)))
        tfs.append(TF(lo, hi, float(rng.uniform(-1, 1)), float(rng.uniform(0, max_mul)),
                      tuple(float(x) for x in rng.uniform(0, 1, 3)),
                      visible=bool(rng.integers(0, 5) != 0)))
    ext = np.array([nx - 1, ny - 1, nz - 1]) * np.array(spacing)
    centre = np.array(origin) + ext / 2
    if rng.integers(0, 3) == 0:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        up = np.cross(v, rng.normal(size=3))
        radius = 0.5 * float(np.linalg.norm(ext + np.array(spacing)))
        cam = Cam("ortho", tuple(centre), tuple(v), tuple(up),
                  ortho_height=float(2.2 * radius + 1.0))
        stereo = False
    else:
        base = synth.random_view_camera(rng, (nx, ny, nz), True)
        # re-centre on the volume as placed (spacing and origin)
        scale = float(np.linalg.norm(ext + np.array(spacing))) / float(
            np.linalg.norm([nx, ny, nz]))
        off = (np.array(base.center) - (np.array([nx, ny, nz]) - 1) / 2) * scale
        cam = Cam("perspective", tuple(centre + off), base.forward, base.up, base.fov_y, 1.0,
                  base.eye_separation * scale, base.convergence * scale)
        stereo = True
    w, h = int(rng.integers(1, 49)), int(rng.integers(1, 41))
    step = float(rng.uniform(0.3, 1.5)) * float(min(spacing))
    tau = float(rng.choice([1.0, 0.99, 0.9, 0.5]))
    bg = tuple(float(x) for x in rng.uniform(0, 1, 4)) if rng.integers(0, 2) else (0, 0, 0, 0)
    sc = Scene(f"random {seed}", vol, bits, tfs, cam, w, h, stereo, step, tau, bg)
    sc.spacing, sc.origin = spacing, origin
    return sc, brick, pairs, precision


@pytest.mark.parametrize("seed", range(160))
def test_random_configuration_against_the_oracle(ctx, seed):
    sc, brick, pairs, precision = random_case(seed)
    tol = 4e-3 if precision == vr.VR_FP16 else 1e-3
    vol = gpu.make_volume(ctx, sc, brick, row_pairs=pairs)
    try:
        vr.vr_test_clear_skip(ctx.ptr, False)
        full = gpu.render(ctx, sc, precision, vol=vol)
        vr.vr_test_clear_skip(ctx.ptr, True)
        rgba, smp = gpu.render(ctx, sc, precision, vol=vol)
    finally:
        vr.vr_test_clear_skip(ctx.ptr, True)
        vol.destroy()
    assert np.array_equal(full[1], smp)
    assert np.array_equal(full[0].view(np.uint32), rgba.view(np.uint32))
    gpu.compare(rgba, smp, orc.render_all(sc, band_eps=tol), tol)
