"""GPU parity of the lit path (one global directional light, per-channel
normals from central differences of the trilinear field): every data variant
and layout against the FP64 oracle, the thin-slab closed form, the
colour-only invariants bit for bit, the transparent-sample skip, random
configurations, and lit requests inside batches and the serving loop."""
import time

import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
from paper_1407_2089_amd import synth
from paper_1407_2089_amd.synth import TF, Cam, Light, Scene

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


def test_lit_thin_slab_matches_the_closed_form(ctx):
    # The oracle's result here equals the hand-derived two-sample closed form
    # (oracle pin P14); the GPU must reproduce it to FP32 rounding.
    nx, ny = 8, 5
    V = np.zeros((1, 1, ny, nx), np.uint8)
    V[0, 0] = (20 * np.arange(nx) + 10)[None, :]
    cam = Cam("ortho", (7.0, 2.0, -3.0), (0, 0, 1), (0, -1, 0), ortho_height=1.0)
    sc = Scene("lit slab", V, 8, [TF(0.0, 1.0, 0.0, 0.9, (1.0, 0.5, 0.25))], cam, 6, 2, False,
               0.5, 1.0, spacing=(2.0, 1.0, 0.5))
    sc.light = Light((0.2, 0.0, -1.0), 0.25, 0.6)
    rgba, smp = gpu.render(ctx, sc)
    ref = orc.render_all(sc)
    assert (smp == 2).all()
    np.testing.assert_allclose(rgba.reshape(-1, 4), ref["rgba"].reshape(-1, 4), rtol=0,
                               atol=2e-6)


VARIANTS = [(1, np.uint8, 8, False), (2, np.uint8, 8, False), (3, np.uint8, 8, False),
            (4, np.uint8, 8, False), (1, np.uint16, 12, False), (2, np.uint16, 12, False),
            (3, np.uint16, 12, False), (4, np.uint16, 16, False), (1, np.uint8, 8, True),
            (2, np.uint8, 8, True), (4, np.uint8, 8, True), (1, np.uint16, 16, True),
            (2, np.uint16, 12, True), (5, np.uint8, 8, False), (6, np.uint16, 12, False)]


@pytest.mark.parametrize("precision", [vr.VR_FP32, vr.VR_FP16])
@pytest.mark.parametrize("ch,dtype,bits,pairs", VARIANTS)
def test_every_lit_variant_matches_the_oracle(ctx, ch, dtype, bits, pairs, precision):
    log(f"lit variant ch={ch} {dtype.__name__} bits={bits} pairs={pairs} prec={precision}")
    dims = (44, 38, 22)
    seed = 100 * ch + bits + (7 if pairs else 0)
    vol = synth.cells_and_vessels(dims, ch, bits, seed, n_cells=8, n_tubes=2)
    rng = np.random.default_rng(seed)
    tfs = [TF(float(rng.uniform(0.03, 0.1)), float(rng.uniform(0.5, 0.9)),
              float(rng.uniform(-0.4, 0.4)), float(rng.uniform(0.5, 1.0)),
              tuple(float(x) for x in rng.uniform(0.2, 1.0, 3))) for _ in range(ch)]
    cam = synth.orbit_camera(dims, float(rng.uniform(0, 360)), float(rng.uniform(-60, 60)), 40.0)
    sc = Scene("lit", vol, bits, tfs, cam, 72, 56, True, 0.8, 0.98, (0.1, 0.2, 0.3, 0.5),
               spacing=(1.0, 1.2, 1.6))
    sc.light = Light(tuple(float(x) for x in rng.normal(size=3)), 0.3, 0.7)
    v = gpu.make_volume(ctx, sc, row_pairs=pairs)
    try:
        vr.vr_test_clear_skip(ctx.ptr, False)
        full = gpu.render(ctx, sc, precision, vol=v)
        vr.vr_test_clear_skip(ctx.ptr, True)
        rgba, smp = gpu.render(ctx, sc, precision, vol=v)
    finally:
        vr.vr_test_clear_skip(ctx.ptr, True)
        v.destroy()
    assert np.array_equal(full[1], smp) and same_bits(full[0], rgba)
    tol = TOL16 if precision == vr.VR_FP16 else TOL32
    ref = orc.render_all(sc, band_eps=tol)
    st = gpu.compare(rgba, smp, ref, tol)
    log(f"  {st}, lit margin max {ref['lit_margin'].max():.2e}")
    # The allowance for FP32 gradient rounding stays below the tolerance
    # itself, so the widened bound stays meaningful.
    assert ref["lit_margin"].max() < tol
    assert rgba[..., :3].max() > 0.05  # something was lit


def test_lighting_changes_colour_only(ctx):
    # Same kernel arithmetic for opacity: lit and unlit renders share alpha
    # and sample counts bit for bit; ambient 1 without diffuse is the unlit
    # image bit for bit (the shade is exactly 1).
    sc = synth.realistic_scene(width=480, height=270)
    v = gpu.make_volume(ctx, sc)
    try:
        base = gpu.render(ctx, sc, vol=v)
        sc.light = Light((0.4, -0.3, -0.8), 0.3, 0.7)
        lit = gpu.render(ctx, sc, vol=v)
        sc.light = Light((0.4, -0.3, -0.8), 1.0, 0.0)
        unit = gpu.render(ctx, sc, vol=v)
    finally:
        v.destroy()
    assert np.array_equal(lit[1], base[1])
    assert same_bits(lit[0][..., 3], base[0][..., 3])
    assert same_bits(unit[0], base[0]) and np.array_equal(unit[1], base[1])
    assert not np.allclose(lit[0][..., :3], base[0][..., :3], atol=1e-2)
    sc.light = Light((0.4, -0.3, -0.8), 0.3, 0.7)
    ref = orc.render_all(sc)
    st = gpu.compare(lit[0], lit[1], ref, TOL32)
    log(f"lit realistic 480x270 {st}, lit margin max {ref['lit_margin'].max():.2e}")
    assert ref["lit_margin"].max() < TOL32


def test_lit_random_configurations(ctx):
    # 40 seeded random configurations (as in the unlit random test) with a
    # random light, each against the oracle and bitwise with the skip off.
    from test_gpu_random import random_case
    for seed in range(40):
        sc, brick, pairs, precision = random_case(500 + seed)
        rng = np.random.default_rng(900 + seed)
        sc.light = Light(tuple(float(x) for x in rng.normal(size=3)),
                         float(rng.uniform(0, 1)), float(rng.uniform(0, 1)))
        tol = TOL16 if precision == vr.VR_FP16 else TOL32
        log(f"lit random {500 + seed}")
        v = gpu.make_volume(ctx, sc, brick, row_pairs=pairs)
        try:
            vr.vr_test_clear_skip(ctx.ptr, False)
            full = gpu.render(ctx, sc, precision, vol=v)
            vr.vr_test_clear_skip(ctx.ptr, True)
            rgba, smp = gpu.render(ctx, sc, precision, vol=v)
        finally:
            vr.vr_test_clear_skip(ctx.ptr, True)
            v.destroy()
        assert np.array_equal(full[1], smp) and same_bits(full[0], rgba)
        ref = orc.render_all(sc, band_eps=tol)
        assert ref["lit_margin"].max() < tol
        gpu.compare(rgba, smp, ref, tol)


def lit_and_unlit_requests(ctx, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    vols, reqs, outs = [], [], []
    for q, (ch, dt, bits, pairs) in enumerate([(2, np.uint16, 12, True), (4, np.uint8, 8, False),
                                                (1, np.uint8, 8, True)]):
        dims = (int(rng.integers(24, 60)), int(rng.integers(24, 60)), int(rng.integers(10, 30)))
        data = synth.cells_and_vessels(dims, ch, bits, seed + q, n_cells=6, n_tubes=2)
        tfs = [TF(0.05, 0.7, 0.0, 1.0, tuple(rng.uniform(0.2, 1, 3))) for _ in range(ch)]
        sc = Scene("m", data, bits, tfs, None, 1, 1, False, 1.0, 1.0)
        vols.append((gpu.make_volume(ctx, sc, row_pairs=pairs), dims))
    for q in range(n):
        v, dims = vols[q % len(vols)]
        w, h = int(rng.integers(1, 120)), int(rng.integers(1, 90))
        stereo = bool(rng.integers(0, 2))
        cam = synth.random_view_camera(rng, dims, stereo)
        light = Light(tuple(rng.normal(size=3)), 0.25, 0.75) if q % 2 == 0 else None
        eyes = 2 if stereo else 1
        out = torch.full((eyes, h, w, 4), float("nan"), device="cuda")
        smp = torch.full((eyes, h, w), -1, dtype=torch.int32, device="cuda")
        reqs.append(vr.make_request(v.ptr, 0, cam, w, h, stereo, 1.0, 0.99, out,
                                    (0.0, 0.0, 0.0, 0.0), vr.VR_FP32, smp, light))
        outs.append((out, smp))
    return vols, reqs, outs


def test_lit_requests_in_batches_and_serving_equal_alone(ctx):
    import torch
    vols, reqs, outs = lit_and_unlit_requests(ctx, 18, 31)
    ref = []
    for r, (o, s) in zip(reqs, outs):
        vr.vr_render(ctx.ptr, r, torch.cuda.current_stream())
        torch.cuda.synchronize()
        ref.append((o.clone(), s.clone()))
    for o, s in outs:
        o.fill_(float("nan"))
        s.fill_(-1)
    vr.vr_render_batch(ctx.ptr, reqs, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for (o, s), (ro, rs) in zip(outs, ref):
        assert torch.equal(o, ro) and torch.equal(s, rs)
    for o, s in outs:
        o.fill_(float("nan"))
        s.fill_(-1)
    torch.cuda.synchronize()
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
    for v, _ in vols:
        v.destroy()


@pytest.mark.parametrize("ch", [3, 4, 6])
def test_lit_flat_plateaus_have_no_gradient(ctx, ch):
    # A saturated cube per channel: inside it every gradient sample reads
    # equal voxels, so the gradient is exactly zero and the shade is
    # ambient + diffuse (the FP32 weighted-sum interpolation of many channels
    # would leave rounding noise there, with a random normal).
    nx, ny, nz = 30, 26, 20
    rng = np.random.default_rng(ch)
    vol = rng.integers(0, 30, size=(ch, nz, ny, nx)).astype(np.uint8)
    for c in range(ch):
        vol[c, 4 + c:16, 5:20, 6 + c:24] = 255
    tfs = [TF(0.3, 0.9, 0.0, 0.3, tuple(float(x) for x in rng.uniform(0.2, 1.0, 3)))
           for _ in range(ch)]
    cam = synth.orbit_camera((nx, ny, nz), 40.0, 30.0, 40.0)
    sc = Scene("plateau", vol, 8, tfs, cam, 64, 48, True, 0.7, 0.99)
    sc.light = Light((0.3, -0.4, 0.9), 0.2, 0.8)
    rgba, smp = gpu.render(ctx, sc)
    gpu.compare(rgba, smp, orc.render_all(sc), TOL32)


@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 5, 3), (2, 2, 2), (3, 1, 7), (6, 4, 1)])
@pytest.mark.parametrize("large", [False, True])
@pytest.mark.parametrize("pairs", [False, True])
def test_lit_thin_and_tiny_volumes(ctx, dims, large, pairs):
    # Volumes one or two voxels thick along some axis: every shaded sample
    # sits at a face there, and the gradient layers of the other axes are
    # loaded from clamped corners next to those faces (bricks of 4 and the
    # default shapes; the large-volume path addresses them with plain loads).
    log(f"lit tiny dims={dims} large={large} pairs={pairs}")
    rng = np.random.default_rng(sum(dims) * 7 + large + 2 * pairs)
    nx, ny, nz = dims
    vol = rng.integers(0, 4096, size=(2, nz, ny, nx)).astype(np.uint16)
    tfs = [TF(0.05, 0.8, 0.2, 1.0, (0.9, 0.3, 0.1)), TF(0.1, 0.9, -0.2, 0.8, (0.1, 0.6, 0.9))]
    cam = synth.orbit_camera(dims, 35.0, 25.0, 40.0, 2.5)
    sc = Scene("lit-tiny", vol, 12, tfs, cam, 40, 30, True, 0.25, 0.99, (0.1, 0.1, 0.2, 0.3),
               spacing=(1.0, 1.3, 0.7))
    sc.light = Light((0.3, -0.6, 0.5), 0.3, 0.7)
    for brick in ((0, 0, 0), (4, 4, 4)):
        if large:
            vr.vr_test_large_addressing(ctx.ptr, True)
        try:
            v = gpu.make_volume(ctx, sc, brick, row_pairs=pairs)
        finally:
            if large:
                vr.vr_test_large_addressing(ctx.ptr, False)
        try:
            rgba, smp = gpu.render(ctx, sc, vr.VR_FP32, vol=v)
        finally:
            v.destroy()
        gpu.compare(rgba, smp, orc.render_all(sc, band_eps=TOL32), TOL32)


def word_bytes(ch, dtype):
    w = 1 if ch == 1 else 2 if ch == 2 else 4 if ch <= 4 else 8
    return w * (2 if dtype == np.uint16 else 1)


@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 4, 2), (3, 1, 5), (2, 3, 1)])
@pytest.mark.parametrize("ch,dtype,bits", [(1, np.uint8, 8), (5, np.uint8, 8), (6, np.uint16, 12)])
@pytest.mark.parametrize("large", [False, True])
@pytest.mark.parametrize("lit", [False, True])
def test_thin_volumes_every_word_size(ctx, dims, ch, dtype, bits, large, lit):
    # As above for 1-, 8- and 16-byte words (the wide words take the
    # one-axis-at-a-time gradient), lit and unlit, FP32 and FP16 sampling.
    log(f"thin dims={dims} ch={ch} large={large} lit={lit}")
    rng = np.random.default_rng(sum(dims) * 11 + ch + 2 * large + 4 * lit)
    nx, ny, nz = dims
    full = (1 << bits) - 1
    vol = rng.integers(0, full + 1, size=(ch, nz, ny, nx)).astype(dtype)
    tfs = [TF(float(rng.uniform(0.02, 0.1)), float(rng.uniform(0.6, 0.9)), 0.0,
              float(rng.uniform(0.5, 1.0)), tuple(float(x) for x in rng.uniform(0.2, 1, 3)))
           for _ in range(ch)]
    cam = synth.orbit_camera(dims, 200.0, -30.0, 40.0, 2.5)
    sc = Scene("thin", vol, bits, tfs, cam, 36, 28, True, 0.3, 0.98)
    if lit:
        sc.light = Light((-0.4, 0.2, 0.7), 0.25, 0.75)
    pairs = word_bytes(ch, dtype) <= (8 if large else 4)
    for row_pairs in sorted({False, pairs}):
        if large:
            vr.vr_test_large_addressing(ctx.ptr, True)
        try:
            v = gpu.make_volume(ctx, sc, row_pairs=row_pairs)
        finally:
            if large:
                vr.vr_test_large_addressing(ctx.ptr, False)
        try:
            for prec, tol in ((vr.VR_FP32, TOL32), (vr.VR_FP16, TOL16)):
                rgba, smp = gpu.render(ctx, sc, prec, vol=v)
                gpu.compare(rgba, smp, orc.render_all(sc, band_eps=tol), tol)
        finally:
            v.destroy()
