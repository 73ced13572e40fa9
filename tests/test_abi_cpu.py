"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/vr.h, sizes storage by the documented brick
layout, and rejects invalid arguments with the documented status before
touching a device (validation-only context, device = -1)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import paper_1407_2089_amd as vr
from paper_1407_2089_amd.synth import Cam, Light

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="vr.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = vr.lib()
    names = declared_symbols()
    assert "vr_render" in names and "vr_submit" in names and len(names) == 19
    assert "vr_tune_batch" in names
    assert "vr_stream_frame" in names and "vr_stream_ready" in names
    dn = declared_symbols("vr_denoise.h")
    assert dn == ["vr_denoise_workspace_bytes", "vr_gaussian_weights", "vr_mrf_denoise",
                  "vr_remove_background"]
    for n in names + declared_symbols("vr_test.h") + dn:
        assert hasattr(L, n), n


def desc(nx=64, ny=48, nz=20, ch=2, frames=3, dtype=vr.VR_U16, bits=12, brick=(0, 0, 0),
         spacing=(1.0, 1.0, 1.0), row_pairs=0):
    return vr.vr_volume_desc(nx, ny, nz, ch, frames, dtype, bits, (C.c_float * 3)(*spacing),
                             (C.c_float * 3)(0, 0, 0), (C.c_int32 * 3)(*brick), row_pairs)


WORD = {1: 1, 2: 2, 3: 4, 4: 4, 5: 8, 6: 8}   # bytes per voxel word of uint8 channels


def with_cells(brick_bytes, dims, word):
    """Frame bytes: the bricks padded to 256 bytes, then one word per macro
    cell of 8 x 8 x 8 sample corners (floor(n / 8) + 1 cells per axis),
    padded to 256 bytes."""
    cells = 1
    for n in dims:
        cells *= n // 8 + 1
    return (brick_bytes + 255) // 256 * 256 + (cells * word + 255) // 256 * 256


@pytest.mark.parametrize("dims,ch,dtype,brick", [
    ((64, 48, 20), 2, vr.VR_U16, (16, 16, 16)),
    ((1, 1, 1), 1, vr.VR_U8, (4, 4, 4)),
    ((100, 37, 9), 3, vr.VR_U8, (8, 16, 4)),
    ((512, 512, 64), 4, vr.VR_U16, (32, 32, 8)),
    ((40, 30, 20), 5, vr.VR_U8, (8, 8, 8)),
    ((40, 30, 20), 6, vr.VR_U16, (4, 8, 16)),
])
def test_storage_bytes_follow_brick_layout(dims, ch, dtype, brick):
    d = desc(*dims, ch=ch, frames=3, dtype=dtype, bits=8 if dtype == vr.VR_U8 else 16,
             brick=brick)
    word = WORD[ch] * (1 if dtype == vr.VR_U8 else 2)
    nb = [math.ceil((n + 1) / b) for n, b in zip(dims, brick)]
    per_brick = (brick[0] + 1) * (brick[1] + 1) * (brick[2] + 1)
    frame = with_cells(nb[0] * nb[1] * nb[2] * per_brick * word, dims, word)
    assert vr.vr_volume_storage_bytes(d) == 3 * frame


@pytest.mark.parametrize("dims,ch,dtype,brick", [
    ((64, 48, 20), 2, vr.VR_U16, (16, 16, 16)),
    ((100, 37, 9), 3, vr.VR_U8, (8, 16, 4)),
    ((512, 512, 64), 2, vr.VR_U16, (0, 0, 0)),
    ((7, 5, 3), 4, vr.VR_U8, (4, 4, 4)),
    ((33, 20, 11), 1, vr.VR_U8, (0, 0, 0)),
    ((33, 20, 11), 2, vr.VR_U8, (8, 4, 16)),
    ((9, 70, 5), 1, vr.VR_U16, (32, 4, 4)),
])
def test_storage_bytes_of_the_row_pair_layout(dims, ch, dtype, brick):
    """Row pairs: a brick plane holds By pairs of rows, 2 (Bx + 1) words each."""
    d = desc(*dims, ch=ch, frames=2, dtype=dtype, bits=8 if dtype == vr.VR_U8 else 16,
             brick=brick, row_pairs=1)
    word = WORD[ch] * (1 if dtype == vr.VR_U8 else 2)
    if brick == (0, 0, 0):
        brick = {1: (16, 16, 16), 2: (8, 32, 8), 4: (4, 16, 16)}[word]
    nb = [math.ceil((n + 1) / b) for n, b in zip(dims, brick)]
    per_brick = brick[1] * 2 * (brick[0] + 1) * (brick[2] + 1)
    frame = with_cells(nb[0] * nb[1] * nb[2] * per_brick * word, dims, word)
    assert vr.vr_volume_storage_bytes(d) == 2 * frame


@pytest.mark.parametrize("ch,dtype,bits,row_pairs", [
    (2, vr.VR_U16, 12, 2), (4, vr.VR_U8, 8, -1), (5, vr.VR_U16, 16, 1), (6, vr.VR_U16, 12, 1)])
def test_row_pairs_need_words_of_at_most_8_bytes_and_a_flag(ch, dtype, bits, row_pairs):
    with pytest.raises(vr.VrError):
        vr.vr_volume_storage_bytes(desc(ch=ch, dtype=dtype, bits=bits, row_pairs=row_pairs))


@pytest.mark.parametrize("ch,dtype,bits", [(3, vr.VR_U16, 16), (4, vr.VR_U16, 12),
                                           (5, vr.VR_U8, 8), (6, vr.VR_U8, 8)])
def test_row_pairs_of_8_byte_words_need_a_large_volume(ch, dtype, bits):
    ctx = vr.vr_init(-1, 1 << 40)
    try:
        d = desc(ch=ch, dtype=dtype, bits=bits, row_pairs=1, frames=1)
        n = vr.vr_volume_storage_bytes(d)  # sized like any pair layout
        with pytest.raises(vr.VrError, match="need a large volume") as e:
            vr.vr_create_volume(ctx, d, FAKE, n)
        assert e.value.status == vr.VR_ERR_INVALID_ARG
        vr.vr_test_large_addressing(ctx, True)
        vr.vr_destroy_volume(vr.vr_create_volume(ctx, d, FAKE, n))
        vr.vr_test_large_addressing(ctx, False)
        big = desc(16384, 8, 8, ch=ch, dtype=dtype, bits=bits, row_pairs=1, frames=1)
        vr.vr_destroy_volume(vr.vr_create_volume(ctx, big, FAKE, vr.vr_volume_storage_bytes(big)))
    finally:
        vr.vr_shutdown(ctx)


@pytest.mark.parametrize("ch,dtype,bits,brick", [
    (1, vr.VR_U8, 8, (16, 16, 8)), (2, vr.VR_U8, 8, (8, 16, 8)), (1, vr.VR_U16, 12, (8, 16, 8)),
    (2, vr.VR_U16, 12, (8, 16, 8)), (4, vr.VR_U8, 8, (8, 16, 8)), (3, vr.VR_U8, 8, (8, 16, 8)),
    (3, vr.VR_U16, 16, (8, 8, 8)), (4, vr.VR_U16, 16, (8, 8, 8)), (5, vr.VR_U8, 8, (8, 8, 8)),
    (6, vr.VR_U8, 8, (8, 8, 8)), (5, vr.VR_U16, 12, (8, 8, 8)), (6, vr.VR_U16, 16, (8, 8, 8))])
def test_default_brick_depends_on_word_size(ch, dtype, bits, brick):
    assert vr.vr_volume_storage_bytes(desc(ch=ch, dtype=dtype, bits=bits, brick=(0, 0, 0))) == \
        vr.vr_volume_storage_bytes(desc(ch=ch, dtype=dtype, bits=bits, brick=brick))


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("nz", 16385), ("channels", 0), ("channels", 7), ("frames", 0), ("dtype", 3),
    ("bits", 7),
])
def test_invalid_descriptions(field, value):
    d = desc()
    setattr(d, field, value)
    with pytest.raises(vr.VrError) as e:
        vr.vr_volume_storage_bytes(d)
    assert e.value.status == vr.VR_ERR_INVALID_ARG


def test_invalid_spacing_bits_and_brick():
    for d in (desc(spacing=(1, 0, 1)), desc(spacing=(1, float("nan"), 1)),
              desc(dtype=vr.VR_U8, bits=12), desc(dtype=vr.VR_U16, bits=17),
              desc(brick=(16, 12, 16)), desc(brick=(64, 64, 64))):
        with pytest.raises(vr.VrError) as e:
            vr.vr_volume_storage_bytes(d)
        assert e.value.status == vr.VR_ERR_INVALID_ARG


@pytest.mark.parametrize("dims,large", [((2048, 2048, 255), True), ((2044, 2044, 255), True),
                                        ((2040, 2044, 255), False), ((1024, 1024, 64), False)])
def test_2_to_the_24_bricks_take_the_large_addressing(dims, large):
    # 4 x 4 x 4 bricks of 1-byte words: 2044 x 2044 x 255 voxels give
    # 512 x 512 x 64 = 2^24 bricks (2.1e9 words, under 2^31 and 4 GiB), where
    # the 32-bit sampler's 24-bit brick products would wrap; one brick column
    # less stays on the 32-bit path
    ctx = vr.vr_init(-1, 1 << 40)
    try:
        d = desc(*dims, ch=1, frames=1, dtype=vr.VR_U8, bits=8, brick=(4, 4, 4))
        nb = [math.ceil((n + 1) / 4) for n in dims]
        assert (nb[0] * nb[1] * nb[2] >= 1 << 24) == large
        assert nb[0] * nb[1] * nb[2] * 125 < 1 << 31
        v = vr.vr_create_volume(ctx, d, FAKE, vr.vr_volume_storage_bytes(d))
        assert vr.vr_test_volume_large(v) == large
        vr.vr_destroy_volume(v)
    finally:
        vr.vr_shutdown(ctx)


def test_large_volume_limits():
    # a frame of 2^31 words or more, 4 GiB or more, or an axis above 8192
    # voxels takes the large-volume addressing: accepted, sized as any other
    for dims, ch, dt in (((8192, 8192, 64), 1, vr.VR_U8), ((1024, 1024, 800), 2, vr.VR_U16),
                         ((16384, 3, 2), 1, vr.VR_U8), ((10173, 3858, 74), 5, vr.VR_U8)):
        d = desc(*dims, ch=ch, frames=2, dtype=dt, bits=8 if dt == vr.VR_U8 else 16)
        word = WORD[ch] * (1 if dt == vr.VR_U8 else 2)
        assert vr.vr_volume_storage_bytes(d) >= 2 * word * dims[0] * dims[1] * dims[2]
    # the default brick of a large volume with 8-byte words is 4 x 16 x 8;
    # smaller volumes with 8-byte words keep 8 x 8 x 8
    def frame(dims, b, word):
        nb = [math.ceil((n + 1) / e) for n, e in zip(dims, b)]
        return with_cells(nb[0] * nb[1] * nb[2] * (b[0] + 1) * (b[1] + 1) * (b[2] + 1) * word,
                          dims, word)
    mont = (10173, 3858, 74)
    assert vr.vr_volume_storage_bytes(desc(*mont, ch=5, frames=1, dtype=vr.VR_U8, bits=8)) == \
        frame(mont, (4, 16, 8), 8)
    assert vr.vr_volume_storage_bytes(desc(512, 512, 64, ch=5, frames=1, dtype=vr.VR_U8, bits=8)) \
        == frame((512, 512, 64), (8, 8, 8), 8)
    # row pairs too; not beyond 16384 voxels per axis
    for d in (desc(8192, 8192, 64, ch=1, frames=1, dtype=vr.VR_U8, bits=8, row_pairs=1),
              desc(8193, 4, 4, ch=2, frames=1, dtype=vr.VR_U16, bits=12, row_pairs=1)):
        assert vr.vr_volume_storage_bytes(d) > 0
    for dims in ((16385, 4, 4), (4, 16385, 4), (4, 4, 16385)):
        with pytest.raises(vr.VrError, match="1..16384") as e:
            vr.vr_volume_storage_bytes(desc(*dims))
        assert e.value.status == vr.VR_ERR_INVALID_ARG
    # storage of every frame must fit 64 bits
    with pytest.raises(vr.VrError, match="bricks"):
        vr.vr_volume_storage_bytes(desc(16384, 16384, 16384, ch=6, frames=1 << 30,
                                        dtype=vr.VR_U16, bits=16))


@pytest.fixture
def vctx():
    ctx = vr.vr_init(-1, 1 << 30)
    yield ctx
    vr.vr_shutdown(ctx)


FAKE = 0x7f0000000000  # never dereferenced by a validation-only context


def test_validation_context_budget(vctx):
    d = desc(frames=1)
    need = vr.vr_volume_storage_bytes(d)
    with pytest.raises(vr.VrError) as e:
        vr.vr_create_volume(vctx, d, FAKE, need - 1)
    assert e.value.status == vr.VR_ERR_OUT_OF_MEMORY
    with pytest.raises(vr.VrError) as e:
        vr.vr_create_volume(vctx, d, FAKE + 16, need)
    assert e.value.status == vr.VR_ERR_INVALID_ARG and "aligned" in str(e.value)
    vols = []
    n = (1 << 30) // need
    for _ in range(n):
        vols.append(vr.vr_create_volume(vctx, d, FAKE, need))
    with pytest.raises(vr.VrError) as e:
        vr.vr_create_volume(vctx, d, FAKE, need)
    assert e.value.status == vr.VR_ERR_OUT_OF_MEMORY
    with pytest.raises(vr.VrError) as e:
        vr.vr_shutdown(vctx)
    assert e.value.status == vr.VR_ERR_BUSY
    for v in vols:
        vr.vr_destroy_volume(v)


def lit(r, direction, ambient=0.3, diffuse=0.7):
    r.light = vr.make_light(Light(direction, ambient, diffuse))


def good_request(vol):
    cam = Cam("perspective", (10, 20, 30), (0, 0, -1), (0, 1, 0), 0.8, 1.0, 1.0, 30.0)
    return vr.make_request(vol, 0, cam, 64, 32, True, 1.0, 0.99, FAKE)


@pytest.fixture
def vvol(vctx):
    d = desc(frames=2)
    v = vr.vr_create_volume(vctx, d, FAKE, vr.vr_volume_storage_bytes(d))
    yield vctx, v
    vr.vr_destroy_volume(v)


def expect(status, fn, *a):
    with pytest.raises(vr.VrError) as e:
        fn(*a)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_large_addressing_hook(vctx):
    # forced large-volume addressing takes row pairs as well; a large
    # volume's requests pass validation like any other
    d = desc(frames=1, row_pairs=1)
    n = vr.vr_volume_storage_bytes(d)
    vr.vr_test_large_addressing(vctx, True)
    try:
        vr.vr_destroy_volume(vr.vr_create_volume(vctx, d, FAKE, n))
        v = vr.vr_create_volume(vctx, desc(frames=1), FAKE, n * 4)
        expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, vctx, good_request(v))
        vr.vr_destroy_volume(v)
    finally:
        vr.vr_test_large_addressing(vctx, False)
    vr.vr_destroy_volume(vr.vr_create_volume(vctx, d, FAKE, n))
    big = desc(16384, 8, 8, ch=6, frames=1, dtype=vr.VR_U16, bits=16)
    v = vr.vr_create_volume(vctx, big, FAKE, vr.vr_volume_storage_bytes(big))
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, vctx, good_request(v))
    vr.vr_destroy_volume(v)


def test_valid_request_reaches_the_device_check(vvol):
    ctx, v = vvol
    msg = expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, ctx, good_request(v))
    assert "validation-only" in msg
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render_batch, ctx, [good_request(v)] * 3)


@pytest.mark.parametrize("mutate", [
    lambda r: setattr(r, "frame", 2), lambda r: setattr(r, "frame", -1),
    lambda r: setattr(r, "width", -1), lambda r: setattr(r, "height", 20000),
    lambda r: setattr(r, "stereo", 2), lambda r: setattr(r, "step", 0.0),
    lambda r: setattr(r, "step", float("inf")), lambda r: setattr(r, "term_alpha", 0.0),
    lambda r: setattr(r, "term_alpha", 1.5), lambda r: r.background.__setitem__(3, 2.0),
    lambda r: setattr(r, "precision", 7), lambda r: setattr(r, "out_rgba", None),
    lambda r: setattr(r, "vol", None),
    lambda r: setattr(r.cam, "projection", 5),
    lambda r: setattr(r.cam, "projection", vr.VR_ORTHO),  # stereo needs perspective
    lambda r: setattr(r.cam, "fov_y", 0.0), lambda r: setattr(r.cam, "fov_y", 3.2),
    lambda r: setattr(r.cam, "convergence", 0.0),
    lambda r: setattr(r.cam, "eye_separation", -1.0),
    lambda r: r.cam.forward.__setitem__(2, 0.0),                   # forward = 0
    lambda r: [r.cam.up.__setitem__(i, r.cam.forward[i]) for i in range(3)],  # parallel
    lambda r: r.cam.center.__setitem__(0, float("nan")),
    lambda r: setattr(r.light, "enabled", 2),
    lambda r: lit(r, (0.0, 0.0, 0.0)),
    lambda r: lit(r, (float("nan"), 0.0, 1.0)),
    lambda r: lit(r, (0.0, float("inf"), 1.0)),
    lambda r: lit(r, (0.0, 0.0, 1.0), ambient=-0.1),
    lambda r: lit(r, (0.0, 0.0, 1.0), diffuse=1.5),
    lambda r: lit(r, (0.0, 0.0, 1.0), ambient=float("nan")),
])
def test_invalid_requests_are_rejected_before_enqueue(vvol, mutate):
    ctx, v = vvol
    r = good_request(v)
    mutate(r)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_render, ctx, r)
    msg = expect(vr.VR_ERR_INVALID_ARG, vr.vr_render_batch, ctx, [good_request(v), r])
    assert msg.split(": ", 1)[1].startswith("request 1")


def test_lit_requests_are_valid(vvol):
    # any non-zero direction (not unit length), ambient and diffuse in [0, 1]
    ctx, v = vvol
    for d, ka, kd in [((0.0, 0.0, -3.0), 0.0, 1.0), ((1e-3, 2.0, 0.5), 1.0, 0.0),
                      ((-1.0, 0.0, 0.0), 0.3, 0.7)]:
        r = good_request(v)
        lit(r, d, ka, kd)
        expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, ctx, r)
        expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render_batch, ctx, [good_request(v), r])
    # a disabled light is ignored whatever its other fields hold
    r = good_request(v)
    r.light.direction[0] = float("nan")
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, ctx, r)


def test_ortho_mono_and_empty_image_are_valid(vvol):
    ctx, v = vvol
    r = good_request(v)
    r.stereo = 0
    r.cam.projection = vr.VR_ORTHO
    r.cam.ortho_height = 10.0
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, ctx, r)
    r.width = 0
    r.out_rgba = None  # nothing to write
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_render, ctx, r)


def test_transfer_validation(vvol):
    ctx, v = vvol
    vr.vr_set_transfer(v, 1, vr.make_transfer(0.1, 0.9, -1.0, 2.0, (0, 0.5, 1)))
    for tf in (vr.make_transfer(0.5, 0.5), vr.make_transfer(-0.1, 0.5),
               vr.make_transfer(0.0, 1.1), vr.make_transfer(curve=1.5),
               vr.make_transfer(alpha_mul=2.5), vr.make_transfer(rgb=(0, 2, 0))):
        expect(vr.VR_ERR_INVALID_ARG, vr.vr_set_transfer, v, 0, tf)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_set_transfer, v, 2, vr.make_transfer())
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_upload_frame, v, 5, FAKE)
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_upload_frame, v, 1, FAKE)


def test_tune_layout_validation(vctx):
    L = vr.lib()
    d = desc(frames=1)
    tfs = (vr.vr_transfer * 1)(vr.make_transfer())
    reqs = (vr.vr_render_req * 1)()
    ms = C.c_float()
    args = lambda **k: dict(dict(ctx=vctx, desc=C.byref(d), tfs=tfs, frame=FAKE, views=reqs,
                                 n=1, reps=5, max_bytes=0, stream=None, ms=C.byref(ms)), **k)
    def call(**k):
        a = args(**k)
        return L.vr_tune_layout(a["ctx"], a["desc"], a["tfs"], a["frame"], a["views"], a["n"],
                                a["reps"], a["max_bytes"], a["stream"], a["ms"])
    assert call(ctx=None) == vr.VR_ERR_INVALID_ARG
    assert call(desc=None) == vr.VR_ERR_INVALID_ARG
    assert call(tfs=None) == vr.VR_ERR_INVALID_ARG
    assert call(frame=None) == vr.VR_ERR_INVALID_ARG
    assert call(n=0) == vr.VR_ERR_INVALID_ARG
    assert call(views=None) == vr.VR_ERR_INVALID_ARG
    assert call(reps=0) == vr.VR_ERR_INVALID_ARG
    assert call(reps=1001) == vr.VR_ERR_INVALID_ARG
    assert call() == vr.VR_ERR_UNSUPPORTED  # validation-only context
    assert list(d.brick) == [0, 0, 0] and d.row_pairs == 0  # untouched on failure


def test_null_arguments_do_not_crash():
    L = vr.lib()
    assert L.vr_init(0, 0, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_shutdown(None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_volume_storage_bytes(None, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_render(None, None, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_render_batch(None, None, 0, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_destroy_volume(None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_set_transfer(None, 0, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_upload_frame(None, 0, None, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_debug_sample(None, 0, None, 0, None, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_submit(None, None, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_poll(None, 0, None) == vr.VR_ERR_INVALID_ARG
    assert L.vr_release(None, 0) == vr.VR_ERR_INVALID_ARG
    assert vr.vr_last_error() != ""


def test_block_map_is_a_permutation_that_deals_super_tiles_to_xcds():
    """Launches remap hardware block b (dispatched to XCD b mod 8) to a
    position in their tile order: a bijection on every grid size, runs of 16
    consecutive positions (one 4 x 4 super-tile) per XCD dealt in turn, and
    the tail past the last whole round of 8 runs unchanged."""
    R = 16
    for n in list(range(0, 300)) + [16320, 16321, 16384 + 37, 65536 * 3 + 5]:
        m = vr.vr_test_block_map(n)
        assert np.array_equal(np.sort(m), np.arange(n)), n
    n = 8 * R * 2 + 5
    m = vr.vr_test_block_map(n)
    # First deal of runs: XCD x takes positions R x .. R x + R - 1 as its blocks 0..R-1.
    for xcd in range(8):
        blocks = np.arange(xcd, 8 * R * 8, 8)[:R]
        assert list(m[blocks]) == list(range(R * xcd, R * xcd + R))
    assert list(m[8 * R * 2:]) == list(range(8 * R * 2, n))  # the tail keeps its order
    # Work spread: every XCD holds positions from every deal of 8 runs.
    m = vr.vr_test_block_map(8 * R * 10)
    for xcd in range(8):
        rounds = set((m[np.arange(xcd, 8 * R * 10, 8)] // (8 * R)).tolist())
        assert rounds == set(range(10))
    with pytest.raises(vr.VrError):
        vr.vr_test_block_map(-1)


def test_tile_hooks_validate_wave_tiles(vctx):
    for hook in (vr.vr_test_plain_tile, vr.vr_test_batch_tile):
        hook(vctx, 16, 4)
        hook(vctx, 1, 64)
        hook(vctx)  # back to the default / the autotuner
        for bad in ((8, 4), (0, 64), (-8, -8), (65, 1), (128, 0)):
            with pytest.raises(vr.VrError):
                hook(vctx, *bad)


def _f32_up(x):
    """Smallest float32 >= x (x a Fraction or float)."""
    from fractions import Fraction
    f = np.float32(float(x))
    if Fraction(float(f)) < Fraction(x):
        f = np.nextafter(f, np.float32(np.inf))
    return f


@pytest.mark.parametrize("lo,hi,bits", [(0.0, 1.0, 8), (300 / 4095, 3000 / 4095, 12),
                                        (24 / 255, 220 / 255, 8), (0.5, 0.6, 16),
                                        (0.013, 0.9, 12), (0.999, 1.0, 16), (0.2, 0.21, 8)])
def test_transparent_threshold_is_safe_and_tight(lo, hi, bits):
    """The largest tap value T whose samples are skipped: every value up to
    T (1 + 2^-6) (the interpolation error margin) gives u <= 0 in exact
    arithmetic with the kernels' folded constants; T + 1 does not pass the
    same test; and T sits just below the floor lo (2^bits - 1) of the
    transfer-function definition."""
    from fractions import Fraction as F
    scale, bias, t = vr.vr_test_transparent_max(lo, hi, bits)
    full = (1 << bits) - 1
    s, b = F(float(np.float32(scale))), F(float(np.float32(bias)))
    assert t >= 0
    margin = F(1) + F(1, 64)
    assert F(t) * margin * s + b <= 0
    if t < full:
        x = _f32_up(F(t + 1) * margin)
        assert F(float(x)) * s + b > 0
    floor_raw = F(float(np.float32(lo))) * full
    assert t <= floor_raw
    assert t >= floor_raw / margin - 2


# ------------------------------------------------------------- denoising

def test_denoise_workspace_bytes():
    g = vr.make_grid(100, 37, 9, vr.VR_U16, 12)
    vol = (100 * 37 * 9 * 2 + 255) // 256 * 256
    tables = 256 + 65536 + (1 << 20)
    assert vr.vr_denoise_workspace_bytes(g) == 2 * vol + tables
    g = vr.make_grid(1, 1, 1, vr.VR_U8, 8)
    assert vr.vr_denoise_workspace_bytes(g) == 2 * 256 + tables


@pytest.mark.parametrize("grid", [(0, 4, 4, 1, 8), (4, 4, 4, 3, 8), (4, 4, 4, 1, 12),
                                  (4, 4, 4, 2, 8), (4, 4, 4, 2, 17), (2048, 2048, 512, 1, 8)])
def test_denoise_rejects_bad_grids(grid):
    g = vr.make_grid(*grid)
    with pytest.raises(vr.VrError) as e:
        vr.vr_denoise_workspace_bytes(g)
    assert e.value.status == vr.VR_ERR_INVALID_ARG


BASE = 1 << 40
GOOD_W = [1, 2, 1]


def bg_call(vctx, g, lp, src=BASE, dst=BASE + (1 << 30), bg=None, ws=BASE + (2 << 30), n=None):
    n = vr.vr_denoise_workspace_bytes(g) if n is None else n
    return vr.vr_remove_background(vctx, g, lp, src, dst, bg, ws, n)


def test_remove_background_validation(vctx):
    g = vr.make_grid(40, 30, 20, vr.VR_U16, 12)
    ok = vr.make_lowpass(GOOD_W, [4], vr.gaussian_weights(2.0, 2), 2)
    expect(vr.VR_ERR_UNSUPPORTED, lambda: bg_call(vctx, g, ok))
    expect(vr.VR_ERR_UNSUPPORTED, lambda: bg_call(vctx, g, ok, bg=BASE + (3 << 30)))
    bad = [vr.make_lowpass([1, 2, 2], GOOD_W, GOOD_W, 2),      # sum 5
           vr.make_lowpass([1, 3], GOOD_W, GOOD_W, 2),         # even taps
           vr.make_lowpass([1] * 131, GOOD_W, GOOD_W, 2),      # too many taps
           vr.make_lowpass([0, 2 ** 17, 0], [2 ** 17], [2 ** 17], 17)]  # shift > 16
    for lp in bad:
        expect(vr.VR_ERR_INVALID_ARG, lambda: bg_call(vctx, g, lp))
    expect(vr.VR_ERR_INVALID_ARG, lambda: bg_call(vctx, g, ok, n=1000))             # small workspace
    expect(vr.VR_ERR_INVALID_ARG, lambda: bg_call(vctx, g, ok, dst=BASE + 100))     # overlaps src
    expect(vr.VR_ERR_INVALID_ARG, lambda: bg_call(vctx, g, ok, bg=BASE + (2 << 30) + 512))  # in ws
    expect(vr.VR_ERR_INVALID_ARG, lambda: bg_call(vctx, g, ok, src=None))
    # buffers that only touch are fine
    expect(vr.VR_ERR_UNSUPPORTED, lambda: bg_call(vctx, g, ok, dst=BASE + 40 * 30 * 20 * 2))


@pytest.mark.parametrize("sigma,shift,radius", [(0.5, 8, None), (0.6, 3, 2), (0.6, 4, 2),
                                                (1.0, 8, 3), (1.0, 14, None),
                                                (2.5, 16, None), (4.0, 16, None),
                                                (16.0, 16, None), (20.0, 16, None),
                                                (30.0, 16, None), (7.3, 12, 9)])
def test_gaussian_weights_match_the_oracle(sigma, shift, radius):
    # the library's host computation against the oracle's, integer for integer
    from oracle import denoise as dn
    assert vr.gaussian_weights(sigma, shift, radius) == dn.gaussian_weights(sigma, shift, radius)


def test_gaussian_weights_validation():
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, 0.0, 8)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, float("nan"), 8)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, 1.0, 0)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, 1.0, 17)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, 1.0, 8, 65)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_gaussian_weights, 100.0, 3, 5)  # cannot normalise
    buf = (C.c_uint32 * 4)()
    taps = C.c_int32()
    assert vr.lib().vr_gaussian_weights(2.0, 8, -1, buf, 4, C.byref(taps)) == vr.VR_ERR_INVALID_ARG


def test_mrf_validation(vctx):
    g = vr.make_grid(16, 16, 16, vr.VR_U8, 8)
    n = vr.vr_denoise_workspace_bytes(g)
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_mrf_denoise, vctx, g, 10, BASE, BASE + 8192,
           BASE + 65536, n)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_mrf_denoise, vctx, g, -1, BASE, BASE + 8192,
           BASE + 65536, n)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_mrf_denoise, vctx, g, 10, BASE, BASE + 100,
           BASE + 65536, n)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_mrf_denoise, vctx, g, 10, BASE, BASE + 8192,
           BASE + 65536, n - 1)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_mrf_denoise, vctx, g, 10, BASE, None, BASE + 65536, n)


def test_stream_frame_validation(vvol):
    ctx, v = vvol
    raw = 64 * 48 * 20 * 2 * 2   # desc(): 64 x 48 x 20, 2 channels, uint16
    host = C.create_string_buffer(16)
    hp = C.addressof(host)
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_stream_frame, v, 1, hp, BASE, raw, 1, 2)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_frame, v, 2, hp, BASE, raw, 1, 2)   # slot
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_frame, v, -1, hp, BASE, raw, 1, 2)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_frame, v, 0, hp, BASE, raw - 1, 1, 2)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_frame, v, 0, hp, None, raw, 1, 2)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_frame, v, 0, hp, BASE, raw, 3, 3)   # same stream
    expect(vr.VR_ERR_UNSUPPORTED, vr.vr_stream_ready, v, 1, 2)
    expect(vr.VR_ERR_INVALID_ARG, vr.vr_stream_ready, v, 5, 2)
