"""GPU tests of vr_tune_layout: the layout it picks is one of its candidates
and within the storage limit, a volume created with it renders the same bits
as the default layout, and the image matches the FP64 oracle."""
import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Scene

pytestmark = pytest.mark.gpu

CANDIDATES = {((0, 0, 0), 0), ((8, 8, 8), 0), ((8, 16, 8), 0), ((16, 16, 8), 0),
              ((16, 8, 8), 0), ((8, 8, 4), 0), ((4, 16, 8), 0), ((16, 16, 16), 0),
              ((0, 0, 0), 1), ((4, 16, 8), 1), ((8, 16, 8), 1), ((8, 32, 8), 1),
              ((4, 32, 8), 1), ((16, 16, 16), 1)}


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


def scene_for(ch, bits, seed, dims=(96, 80, 40)):
    vol = synth.cells_and_vessels(dims, ch, bits, seed, n_cells=10, n_tubes=3)
    rng = np.random.default_rng(seed)
    tfs = [TF(float(rng.uniform(0.03, 0.1)), float(rng.uniform(0.5, 0.9)), 0.0,
              float(rng.uniform(0.5, 1.0)), tuple(float(x) for x in rng.uniform(0.2, 1.0, 3)))
           for _ in range(ch)]
    cam = synth.orbit_camera(dims, 30.0, 40.0, 40.0)
    return Scene("tune", vol, bits, tfs, cam, 200, 150, True, 0.8, 0.99)


def tuned_desc(ctx, sc, max_bytes=0):
    c, nz, ny, nx = sc.volume.shape
    dtype = vr.VR_U8 if sc.volume.dtype == np.uint8 else vr.VR_U16
    desc = vr.vr_volume_desc(nx, ny, nz, c, 1, dtype, sc.bits, (vr.C.c_float * 3)(*sc.spacing),
                             (vr.C.c_float * 3)(*sc.origin), (vr.C.c_int32 * 3)(0, 0, 0), 0)
    out, smp = gpu.alloc_out(sc)
    view = vr.make_request(None, 0, sc.cam, sc.width, sc.height, True, sc.step, sc.term_alpha,
                           out, sc.background, vr.VR_FP32, smp)
    ms = vr.vr_tune_layout(ctx.ptr, desc, sc.tfs, gpu.to_device(sc.volume), [view], reps=3,
                           max_bytes=max_bytes)
    return desc, ms


@pytest.mark.parametrize("ch,bits,seed", [(2, 12, 5), (1, 8, 6), (5, 8, 7)])
def test_tuned_layout_is_a_candidate_with_the_same_bits(ctx, ch, bits, seed):
    sc = scene_for(ch, bits, seed)
    print(f"tune layout ch={ch} bits={bits}", flush=True)
    desc, ms = tuned_desc(ctx, sc)
    choice = (tuple(desc.brick), desc.row_pairs)
    print(f"  chose {choice} in {ms:.4f} ms", flush=True)
    assert choice in CANDIDATES and ms > 0
    if ch == 5:
        assert desc.row_pairs == 0  # 8-byte words take row pairs only in large volumes
    base = gpu.render(ctx, sc)
    tuned = gpu.render(ctx, sc, brick=tuple(desc.brick), row_pairs=bool(desc.row_pairs))
    assert np.array_equal(base[1], tuned[1])
    assert np.array_equal(base[0].view(np.uint32), tuned[0].view(np.uint32))
    rng = np.random.default_rng(seed)
    pix = rng.choice(sc.width * sc.height, size=2048, replace=False)
    ref = orc.render_all(sc, band_eps=1e-3, pixels=pix)
    img = tuned[0].reshape(2, -1, 4)[:, pix]
    smp = tuned[1].reshape(2, -1)[:, pix]
    gpu.compare(img, smp, ref, 1e-3)


def test_tuned_layout_respects_the_storage_limit(ctx):
    sc = scene_for(2, 12, 8)
    c, nz, ny, nx = sc.volume.shape
    plain = vr.vr_volume_desc(nx, ny, nz, c, 1, vr.VR_U16, 12, (vr.C.c_float * 3)(1, 1, 1),
                              (vr.C.c_float * 3)(0, 0, 0), (vr.C.c_int32 * 3)(0, 0, 0), 0)
    limit = vr.vr_volume_storage_bytes(plain)
    desc, _ = tuned_desc(ctx, sc, max_bytes=limit)
    assert vr.vr_volume_storage_bytes(desc) <= limit
    assert desc.row_pairs == 0  # row pairs store about twice the words


def test_tuning_with_no_admissible_layout_fails_cleanly(ctx):
    sc = scene_for(2, 12, 9, dims=(40, 36, 20))
    desc, _ = tuned_desc(ctx, sc)  # a working call first
    c, nz, ny, nx = sc.volume.shape
    d = vr.vr_volume_desc(nx, ny, nz, c, 1, vr.VR_U16, 12, (vr.C.c_float * 3)(1, 1, 1),
                          (vr.C.c_float * 3)(0, 0, 0), (vr.C.c_int32 * 3)(0, 0, 0), 0)
    out, smp = gpu.alloc_out(sc)
    view = vr.make_request(None, 0, sc.cam, sc.width, sc.height, True, sc.step, sc.term_alpha,
                           out, sc.background, vr.VR_FP32, smp)
    with pytest.raises(vr.VrError) as e:
        vr.vr_tune_layout(ctx.ptr, d, sc.tfs, gpu.to_device(sc.volume), [view], reps=1,
                          max_bytes=4096)  # below every candidate's storage
    assert e.value.status == vr.VR_ERR_OUT_OF_MEMORY
    assert list(d.brick) == [0, 0, 0] and d.row_pairs == 0
    # the context still works afterwards
    tuned = gpu.render(ctx, sc, brick=tuple(desc.brick), row_pairs=bool(desc.row_pairs))
    assert np.isfinite(tuned[0]).all()
