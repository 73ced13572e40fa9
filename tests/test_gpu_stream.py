"""GPU: playback of a series kept in pinned host memory through a ring of
device slots (vr_stream_frame / vr_stream_ready) renders every frame exactly
as the resident series does, bit for bit, with copies overlapping renders,
and streamed frames match the oracle on the frames' own voxels."""
import numpy as np
import pytest

import gpu
import orc
import paper_1407_2089_amd as vr
from paper_1407_2089_amd import synth, workloads

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


def host_series(dims, ch, bits, frames, seed):
    """[F][C][Z][Y][X] pinned host tensor (uint8, or int16 holding uint16)."""
    import torch
    ser = synth.DeviceSeries(dims, ch, bits, seed, frames=frames)
    out = None
    for t in range(frames):
        f = ser.frame(t)
        if out is None:
            out = torch.empty((frames,) + tuple(f.shape), dtype=f.dtype, pin_memory=True)
        out[t].copy_(f)
    return out


def render_all(ctx, vol, frames, slots, cams, W, H, stream, host=None, staging=None,
               copy_stream=None):
    """Renders frame t from slot t % slots; with `host`, streams frames in."""
    import torch
    outs = [torch.full((2, H, W, 4), float("nan"), device="cuda") for _ in range(frames)]
    smps = [torch.full((2, H, W), -1, dtype=torch.int32, device="cuda") for _ in range(frames)]
    if host is not None:
        for t in range(min(slots - 1, frames)):
            vr.vr_stream_frame(vol.ptr, t, host[t], staging, staging.numel(), copy_stream,
                               stream)
    for t in range(frames):
        slot = t % slots
        if host is not None:
            nxt = t + slots - 1
            if nxt < frames:
                vr.vr_stream_frame(vol.ptr, nxt % slots, host[nxt], staging, staging.numel(),
                                   copy_stream, stream)
            vr.vr_stream_ready(vol.ptr, slot, stream)
        req = vr.make_request(vol.ptr, slot, cams[t], W, H, True, 1.0, 0.99, outs[t],
                              out_samples=smps[t])
        vr.vr_render(ctx.ptr, req, stream)
    torch.cuda.synchronize()
    return outs, smps


@pytest.mark.parametrize("ch,bits,pairs,slots,halves,large", [
    (2, 12, True, 2, 1, False), (2, 12, True, 2, 2, False), (4, 8, False, 3, 2, False),
    (1, 8, True, 2, 1, False), (3, 16, False, 4, 2, False), (5, 8, False, 3, 2, True)])
def test_streamed_playback_equals_resident(ctx, ch, bits, pairs, slots, halves, large):
    # large: both volumes take the large-volume addressing (test hook)
    import torch
    vr.vr_test_large_addressing(ctx.ptr, large)
    try:
        _streamed_playback(ctx, ch, bits, pairs, slots, halves)
    finally:
        vr.vr_test_large_addressing(ctx.ptr, False)


def _streamed_playback(ctx, ch, bits, pairs, slots, halves):
    import torch
    dims, F = (96, 80, 40), 7
    W, H = 160, 120
    host = host_series(dims, ch, bits, F, 3 + ch)
    dt = vr.VR_U8 if bits == 8 else vr.VR_U16
    tfs = workloads.default_tfs(ch)
    cams = [synth.orbit_camera(dims, 20.0 * t, 35.0, 40.0) for t in range(F)]
    stream = torch.cuda.current_stream()
    res = vr.Volume(ctx, dims, ch, F, dt, bits, row_pairs=pairs)
    for t in range(F):
        res.upload(t, host[t].cuda())
    for c, tf in enumerate(tfs):
        res.set_transfer(c, tf)
    # resident: frame t is slot t of the resident volume
    ref = render_all(ctx, res, F, F, cams, W, H, stream)
    res.destroy()
    ring = vr.Volume(ctx, dims, ch, slots, dt, bits, row_pairs=pairs)
    for c, tf in enumerate(tfs):
        ring.set_transfer(c, tf)
    staging = torch.empty(halves * host[0].numel() * host.element_size(), dtype=torch.uint8,
                          device="cuda")
    copy = torch.cuda.Stream()
    got = render_all(ctx, ring, F, slots, cams, W, H, stream, host, staging, copy)
    ring.destroy()
    for t in range(F):
        assert torch.equal(got[1][t], ref[1][t]), t
        assert torch.equal(got[0][t].view(torch.int32), ref[0][t].view(torch.int32)), t
    assert float(ref[0][F - 1][..., 3].max()) > 0.1
    # streamed frames against the oracle on the frame's own voxels
    for t in (0, F // 2, F - 1):
        data = host[t].numpy()
        if data.dtype == np.int16:
            data = data.view(np.uint16)
        sc = synth.Scene("stream", data, bits, tfs, cams[t], W, H, True, 1.0, 0.99)
        st = gpu.compare(got[0][t].cpu().numpy(), got[1][t].cpu().numpy(), orc.render_all(sc),
                         1e-3)
        print(f"streamed frame {t}: {st}", flush=True)
