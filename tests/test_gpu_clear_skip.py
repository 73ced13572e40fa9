"""The transparent-sample skip of vr_render (a wave leaves out the arithmetic
of samples whose taps all lie below every channel's transfer-function floor)
must not change a single output bit; and FP16 sampling of 16-bit data stays
finite at the top of the range."""
import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
import scenes
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Scene

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


def render_both(ctx, sc, precision, cells=True):
    """Render with the skips on and off; restore the default.  With cells the
    skipping render also jumps over transparent macro cells; it is compared
    with the per-sample skip alone as well."""
    vol = gpu.make_volume(ctx, sc)
    try:
        vr.vr_test_clear_skip(ctx.ptr, False)
        full = gpu.render(ctx, sc, precision, vol=vol)
        vr.vr_test_clear_skip(ctx.ptr, 2)
        sample_only = gpu.render(ctx, sc, precision, vol=vol)
        vr.vr_test_clear_skip(ctx.ptr, True)
        skip = gpu.render(ctx, sc, precision, vol=vol)
    finally:
        vr.vr_test_clear_skip(ctx.ptr, True)
        vol.destroy()
    assert_same_bits(full, sample_only)
    return full, skip


def assert_same_bits(a, b):
    (ra, sa), (rb, sb) = a, b
    assert np.array_equal(sa, sb)
    assert np.array_equal(ra.view(np.uint32), rb.view(np.uint32))


CASES = [(1, np.uint8, 8), (2, np.uint8, 8), (3, np.uint8, 8), (4, np.uint8, 8),
         (1, np.uint16, 12), (2, np.uint16, 12), (3, np.uint16, 16), (4, np.uint16, 16),
         (5, np.uint8, 8), (6, np.uint8, 8), (5, np.uint16, 12), (6, np.uint16, 16)]


@pytest.mark.parametrize("precision", [vr.VR_FP32, vr.VR_FP16])
@pytest.mark.parametrize("ch,dtype,bits", CASES)
def test_skip_is_bitwise_neutral_with_floors_inside_the_data(ctx, ch, dtype, bits, precision):
    """Floors at data quantiles, so many samples have taps on both sides of
    the threshold; channel 0 integer-aligned floor, others fractional."""
    full = (1 << bits) - 1
    nx, ny, nz = 40, 34, 22
    rng = np.random.default_rng(100 + ch + bits)
    vol = np.zeros((ch, nz, ny, nx), dtype)
    for c in range(ch):
        # sparse bright voxels over a low noise floor: wide transparent regions
        base = rng.integers(0, max(2, full // 12), size=(nz, ny, nx))
        blobs = scenes.random_volume(7 + c, (1, nz, ny, nx), dtype, full + 1)[0] \
            * (rng.random((nz, ny, nx)) < 0.05)
        vol[c] = np.minimum(base + blobs, full).astype(dtype)
    tfs = []
    for c in range(ch):
        q = float(np.quantile(vol[c], 0.85 if c else 0.9))
        lo = (np.floor(q) if c == 0 else q + 0.37) / full
        lo = min(lo, 0.95)
        tfs.append(TF(lo, min(1.0, lo + 0.3), 0.2 * c - 0.2, 1.0 + 0.2 * c,
                      (1.0, 0.5 * c / 3, 0.3), visible=True))
    cam = synth.orbit_camera((nx, ny, nz), 25.0 + 40 * ch, 35.0, 45.0)
    sc = Scene("skip", vol, bits, tfs, cam, 72, 56, True, 0.8, 0.99)
    full_img, skip_img = render_both(ctx, sc, precision)
    assert_same_bits(full_img, skip_img)


@pytest.mark.parametrize("precision", [vr.VR_FP32, vr.VR_FP16])
@pytest.mark.parametrize("dtype,bits,q", [(np.uint8, 8, 1), (np.uint8, 8, 37), (np.uint8, 8, 200),
                                          (np.uint16, 12, 300), (np.uint16, 12, 4000),
                                          (np.uint16, 16, 65000)])
def test_skip_threshold_at_a_plateau_exactly_on_the_floor(ctx, dtype, bits, q, precision):
    """Plateaus of exactly q, q - 1 and q + 1 with the floor at q / full: a
    sample whose taps all equal q may have u = 0 or a rounding-sized u > 0;
    either way the skip must give the same bits as the full arithmetic."""
    full = (1 << bits) - 1
    nx, ny, nz = 30, 24, 16
    vol = np.zeros((1, nz, ny, nx), dtype)
    vol[0, 2:14, 2:12, 2:10] = q
    vol[0, 2:14, 12:22, 2:10] = max(q - 1, 0)
    vol[0, 2:14, 2:22, 10:20] = min(q + 1, full)
    vol[0, 2:14, 2:22, 20:28] = np.clip(np.arange(8) + q - 4, 0, full)[None, None, :]
    tf = TF(q / full, min(1.0, q / full + 0.01), 0.0, 2.0, (1.0, 1.0, 1.0))
    cam = synth.orbit_camera((nx, ny, nz), 30.0, 50.0, 45.0)
    sc = Scene("plateau", vol, bits, [tf], cam, 64, 48, True, 0.7, 1.0)
    full_img, skip_img = render_both(ctx, sc, precision)
    assert_same_bits(full_img, skip_img)


def test_skip_on_the_realistic_content(ctx):
    sc = synth.realistic_scene(width=240, height=136, dims=(128, 128, 32))
    for precision in (vr.VR_FP32, vr.VR_FP16):
        full_img, skip_img = render_both(ctx, sc, precision)
        assert_same_bits(full_img, skip_img)


@pytest.mark.parametrize("ch,bits", [(1, 15), (2, 15), (3, 15), (1, 16), (2, 16)])
def test_fp16_sampling_at_the_top_of_the_bit_depth(ctx, ch, bits):
    """Taps at the full scale 2^bits - 1: 15-bit data converts to FP16
    without the clamp at 65504 that 16-bit data takes; both match the oracle
    within the FP16 tolerance."""
    nx, ny, nz = 26, 22, 14
    vol = scenes.random_volume(72 + ch, (ch, nz, ny, nx), np.uint16, 1 << bits)
    vol[:, 3:11, 4:18, 5:20] = (1 << bits) - 1
    tfs = [TF(0.5, 1.0, 0.0, 0.3, tuple(float(x) for x in np.roll((1.0, 0.3, 0.0), c)))
           for c in range(ch)]
    cam = synth.orbit_camera((nx, ny, nz), 20.0, 40.0, 45.0)
    sc = Scene("top", vol, bits, tfs, cam, 40, 30, True, 0.6, 0.995)
    rgba, smp = gpu.render(ctx, sc, vr.VR_FP16)
    assert np.isfinite(rgba).all()
    gpu.compare(rgba, smp, orc.render_all(sc), 4e-3)


def test_fp16_sampling_of_saturated_16_bit_taps_is_finite(ctx):
    """16-bit taps at 65535 exceed the largest finite half (65504); FP16
    sampling clamps them and stays within the FP16 tolerance of the oracle.
    (FP16 rounds a normalised value x by up to 2^-11 x, which the transfer
    function scales by 1 / (hi - lo): the windows here are wide enough for
    the 4e-3 tolerance; a 0.1-wide window at the top of the range is not.)"""
    nx, ny, nz = 26, 22, 14
    vol = scenes.random_volume(71, (2, nz, ny, nx), np.uint16, 65536)
    vol[:, 3:11, 4:18, 5:20] = 65535
    tfs = [TF(0.5, 1.0, 0.0, 0.3, (1, 0, 0)), TF(0.6, 1.0, 0.4, 0.5, (0, 1, 0))]
    cam = synth.orbit_camera((nx, ny, nz), 20.0, 40.0, 45.0)
    sc = Scene("sat16", vol, 16, tfs, cam, 40, 30, True, 0.6, 0.995)
    rgba, smp = gpu.render(ctx, sc, vr.VR_FP16)
    assert np.isfinite(rgba).all()
    gpu.compare(rgba, smp, orc.render_all(sc), 4e-3)
