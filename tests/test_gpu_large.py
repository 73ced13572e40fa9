"""GPU parity of the large-volume addressing (64-bit byte offsets, FP64 ray
set-up and sample positions) that a volume with an axis above 8192 voxels or
a frame of 2^31 stored words or 4 GiB and more takes.  Here it is forced onto
small volumes (test hook) so every data variant, lit and unlit, runs against
the FP64 oracle, also through batches and the serving loop; the full-size
cases (a frame above 4 GiB, 16384-voxel axes, the five-channel montage) are
in the limits tests."""
import time

import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
import scenes
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Light, Scene

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
        pass


def log(msg):
    print(msg, flush=True)


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


WORD = {1: 1, 2: 2, 3: 4, 4: 4, 5: 8, 6: 8}   # bytes per voxel word of uint8 channels


def word_bytes(ch, dtype):
    return WORD[ch] * (2 if dtype == np.uint16 else 1)


def large_volume(ctx, sc, brick=(0, 0, 0), row_pairs=False):
    vr.vr_test_large_addressing(ctx.ptr, True)
    try:
        return gpu.make_volume(ctx, sc, brick, row_pairs=row_pairs)
    finally:
        vr.vr_test_large_addressing(ctx.ptr, False)


def render_both_skips(ctx, sc, precision, v):
    try:
        vr.vr_test_clear_skip(ctx.ptr, False)
        full = gpu.render(ctx, sc, precision, vol=v)
        vr.vr_test_clear_skip(ctx.ptr, True)
        rgba, smp = gpu.render(ctx, sc, precision, vol=v)
    finally:
        vr.vr_test_clear_skip(ctx.ptr, True)
    assert np.array_equal(full[1], smp) and same_bits(full[0], rgba)
    return rgba, smp


VARIANTS = [(ch, dt, bits, prec) for ch in range(1, 7)
            for dt, bits in ((np.uint8, 8), (np.uint16, 12))
            for prec in (vr.VR_FP32, vr.VR_FP16)]


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("ch,dtype,bits,precision", VARIANTS)
def test_every_large_variant_matches_the_oracle(ctx, ch, dtype, bits, precision, lit, pairs):
    if pairs and word_bytes(ch, dtype) > 8:
        pytest.skip("row pairs exist for voxel words of at most 8 bytes")
    log(f"large variant ch {ch} {dtype.__name__}-{bits} prec {precision} lit {lit} pairs {pairs}")
    dims = (52, 44, 30)
    data = synth.cells_and_vessels(dims, ch, bits, 60 + ch, n_cells=8, n_tubes=3)
    rng = np.random.default_rng(ch * 10 + bits)
    tfs = [TF(float(rng.uniform(0.03, 0.1)), float(rng.uniform(0.5, 0.9)),
              float(rng.uniform(-0.4, 0.4)), float(rng.uniform(0.5, 1.0)),
              tuple(float(x) for x in rng.uniform(0.2, 1.0, 3))) for _ in range(ch)]
    cam = synth.orbit_camera(dims, float(rng.uniform(0, 360)), float(rng.uniform(-60, 60)), 40.0)
    sc = Scene("large", data, bits, tfs, cam, 64, 48, True, 0.8, 0.98, (0.1, 0.2, 0.3, 0.5),
               spacing=(1.0, 1.2, 1.6))
    if lit:
        sc.light = Light(tuple(float(x) for x in rng.normal(size=3)), 0.3, 0.7)
    tol = TOL16 if precision == vr.VR_FP16 else TOL32
    v = large_volume(ctx, sc, row_pairs=pairs)
    try:
        rgba, smp = render_both_skips(ctx, sc, precision, v)
    finally:
        v.destroy()
    stats = gpu.compare(rgba, smp, orc.render_all(sc, band_eps=tol), tol)
    assert float(rgba[..., 3].max()) > 0.1
    log(f"  {stats}")


@pytest.mark.parametrize("seed", range(64))
def test_large_random_configuration_against_the_oracle(ctx, seed):
    # the seeded random configurations of the 32-bit path (their row-pair
    # choice; 8-byte words take pairs on even seeds); every fourth one lit
    from test_gpu_random import random_case
    sc, brick, pairs, precision = random_case(seed)
    if word_bytes(sc.volume.shape[0], sc.volume.dtype) == 8 and seed % 2 == 0:
        pairs = True
    if seed % 4 == 3:
        rng = np.random.default_rng(1300 + seed)
        sc.light = Light(tuple(float(x) for x in rng.normal(size=3)),
                         float(rng.uniform(0, 1)), float(rng.uniform(0, 1)))
    tol = TOL16 if precision == vr.VR_FP16 else TOL32
    v = large_volume(ctx, sc, brick, row_pairs=pairs)
    try:
        rgba, smp = render_both_skips(ctx, sc, precision, v)
    finally:
        v.destroy()
    gpu.compare(rgba, smp, orc.render_all(sc, band_eps=tol), tol)


@pytest.mark.parametrize("pairs", [False, True])
def test_large_sampler_reproduces_a_linear_field(ctx, pairs):
    # trilinear interpolation of a linear field is exact up to FP32 rounding
    import torch
    nx, ny, nz = 37, 29, 23
    vol = scenes.linear_field(nx, ny, nz)
    sc = Scene("lin", vol, 16, [TF()], None, 1, 1, False, 1.0, 1.0)
    v = large_volume(ctx, sc, row_pairs=pairs)
    try:
        rng = np.random.default_rng(5)
        pts = rng.uniform([-1, -1, -1], [nx, ny, nz], size=(4096, 3)).astype(np.float32)
        out = torch.zeros(4096, dtype=torch.float32, device="cuda")
        vr.vr_debug_sample(v.ptr, 0, torch.from_numpy(pts).cuda(), 4096, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
    finally:
        v.destroy()
    import oracle
    exp = oracle.sample(orc.volume(sc), pts.astype(np.float64))[:, 0]
    np.testing.assert_allclose(got, exp, rtol=2e-6, atol=2e-3)


def test_large_volumes_in_batches_and_serving_equal_alone(ctx):
    # large volumes take plain launches inside a batch; the images equal
    # vr_render's bit for bit, next to requests on 32-bit addressed volumes
    import torch
    rng = np.random.default_rng(77)
    vols = []
    for q, (ch, dt, bits, large) in enumerate([(2, np.uint16, 12, True), (4, np.uint8, 8, False),
                                               (5, np.uint8, 8, True), (1, np.uint8, 8, False)]):
        dims = (int(rng.integers(24, 60)), int(rng.integers(24, 60)), int(rng.integers(10, 30)))
        data = synth.cells_and_vessels(dims, ch, bits, 40 + q, n_cells=6, n_tubes=2)
        tfs = [TF(0.05, 0.7, 0.0, 1.0, tuple(rng.uniform(0.2, 1, 3))) for _ in range(ch)]
        sc = Scene("m", data, bits, tfs, None, 1, 1, False, 1.0, 1.0)
        vols.append((large_volume(ctx, sc) if large else gpu.make_volume(ctx, sc), dims))
    reqs, outs = [], []
    for q in range(16):
        v, dims = vols[q % len(vols)]
        w, h = int(rng.integers(1, 120)), int(rng.integers(1, 90))
        stereo = bool(rng.integers(0, 2))
        cam = synth.random_view_camera(rng, dims, stereo)
        light = Light(tuple(rng.normal(size=3)), 0.25, 0.75) if q % 3 == 0 else None
        eyes = 2 if stereo else 1
        out = torch.full((eyes, h, w, 4), float("nan"), device="cuda")
        smp = torch.full((eyes, h, w), -1, dtype=torch.int32, device="cuda")
        reqs.append(vr.make_request(v.ptr, 0, cam, w, h, stereo, 1.0, 0.99, out,
                                    (0.0, 0.0, 0.0, 0.0), vr.VR_FP32, smp, light))
        outs.append((out, smp))
    try:
        ref = []
        for r, (o, s) in zip(reqs, outs):
            vr.vr_render(ctx.ptr, r, torch.cuda.current_stream())
            torch.cuda.synchronize()
            ref.append((o.clone(), s.clone()))

        def reset():
            for o, s in outs:
                o.fill_(float("nan"))
                s.fill_(-1)
            torch.cuda.synchronize()

        reset()
        vr.vr_render_batch(ctx.ptr, reqs, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for (o, s), (ro, rs) in zip(outs, ref):
            assert torch.equal(o, ro) and torch.equal(s, rs)
        reset()
        tickets = [vr.vr_submit(ctx.ptr, r) for r in reqs]
        t0 = time.time()
        for t in tickets:
            while vr.vr_poll(ctx.ptr, t).state < 2:
                assert time.time() - t0 < 60, "ticket stuck"
                time.sleep(0.0002)
            assert vr.vr_poll(ctx.ptr, t).state == 2
            vr.vr_release(ctx.ptr, t)
        for (o, s), (ro, rs) in zip(outs, ref):
            assert torch.equal(o, ro) and torch.equal(s, rs)
    finally:
        for v, _ in vols:
            v.destroy()
