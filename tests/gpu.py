"""Helpers that drive libvr through its C ABI from tests, and the acceptance
rule that compares a GPU image with the oracle's."""
import numpy as np

import paper_1407_2089_amd as vr


def to_device(vol_np):
    import torch
    arr = np.ascontiguousarray(vol_np)
    if arr.dtype == np.uint16:
        arr = arr.view(np.int16)
    return torch.from_numpy(arr).cuda()


def make_volume(ctx, scene, brick=(0, 0, 0), data=None, frames=1, row_pairs=False):
    data = scene.volume if data is None else data
    c, nz, ny, nx = data.shape
    dtype = vr.VR_U8 if data.dtype == np.uint8 else vr.VR_U16
    v = vr.Volume(ctx, (nx, ny, nz), c, frames, dtype, scene.bits, scene.spacing, scene.origin,
                  brick, row_pairs)
    v.upload(0, to_device(data))
    for ch, tf in enumerate(scene.tfs):
        v.set_transfer(ch, tf)
    return v


def request_for(vol, scene, out, samples=None, precision=vr.VR_FP32, frame=0, cam=None,
                term_alpha=None):
    return vr.make_request(vol.ptr, frame, cam or scene.cam, scene.width, scene.height,
                           scene.stereo, scene.step,
                           scene.term_alpha if term_alpha is None else term_alpha, out,
                           scene.background, precision, samples, scene.light)


def alloc_out(scene):
    import torch
    eyes = 2 if scene.stereo else 1
    out = torch.full((eyes, scene.height, scene.width, 4), float("nan"), dtype=torch.float32,
                     device="cuda")
    smp = torch.full((eyes, scene.height, scene.width), -1, dtype=torch.int32, device="cuda")
    return out, smp


def render(ctx, scene, precision=vr.VR_FP32, brick=(0, 0, 0), vol=None, row_pairs=False):
    """Render a scene through vr_render; returns (rgba [eyes][H][W][4],
    samples [eyes][H][W]) as numpy."""
    import torch
    own = vol is None
    if own:
        vol = make_volume(ctx, scene, brick, row_pairs=row_pairs)
    try:
        out, smp = alloc_out(scene)
        req = request_for(vol, scene, out, smp, precision)
        vr.vr_render(ctx.ptr, req, torch.cuda.current_stream())
        torch.cuda.synchronize()
    finally:
        if own:
            vol.destroy()
    return out.cpu().numpy(), smp.cpu().numpy()


def compare(rgba, samples, ref, tol, count_slack=2e-3, pixels=None):
    """Acceptance rule: a pixel passes when its max-abs RGBA error against
    the oracle is within tol, or, for a pixel whose FP64 opacity came within
    tol of the termination threshold, when it lies within tol of one member
    of the oracle's band (R_k, the result of the ray stopped after exactly k
    samples, for each admissible stop k).  Sample counts must equal the
    oracle's, except by one where the real-valued count is within
    count_slack of an integer, and anywhere inside the band's count range.
    Lit renders widen each pixel's colour tolerance by the oracle's
    lit_margin (the reach of FP32 gradient rounding).
    Returns a stats dict (max_err: against the oracle's own stop, every
    pixel; max_err_accept: against the nearest admissible result, i.e. the
    figure the rule bounds; max_err_outside_band; band_pixels); raises
    AssertionError on failure."""
    rgba = np.asarray(rgba, np.float64).reshape(-1, 4)
    ref_rgba = ref["rgba"].reshape(-1, 4)
    bk = ref["band_k"].reshape(-1, 2)
    tolv = np.full(rgba.shape, float(tol))
    if "lit_margin" in ref:
        tolv[:, :3] += ref["lit_margin"].reshape(-1)[:, None]
    err_c = np.abs(rgba - ref_rgba)
    err = err_c.max(-1)
    in_band = bk[:, 0] >= 0
    passed = np.all(err_c <= tolv, axis=-1)
    accept_err = err.copy()
    bidx = ref["band_idx"]
    if bidx.size:
        # distance of each band pixel to each member; NaN padding never matches
        d = np.abs(rgba[bidx][:, None, :] - ref["band_rgba"])
        with np.errstate(invalid="ignore"):
            fits = np.all(d <= tolv[bidx][:, None, :], axis=-1)
            dist = np.where(np.isnan(d).any(-1), np.inf, d.max(-1))
        passed[bidx] |= fits.any(-1)
        accept_err[bidx] = np.minimum(accept_err[bidx], dist.min(-1))
    n_fail = int((~passed).sum())
    stats = {"max_err": float(err.max()) if err.size else 0.0,
             "max_err_accept": float(accept_err.max()) if err.size else 0.0,
             "max_err_outside_band": float(err[~in_band].max()) if (~in_band).any() else 0.0,
             "band_pixels": int(in_band.sum()),
             "band_used": int((in_band & passed & (err > tol)).sum()),
             "fail": n_fail, "pixels": int(err.size)}
    if n_fail:
        idx = np.flatnonzero(~passed)[:5]
        raise AssertionError(f"{n_fail} pixels exceed tol {tol}: first {idx.tolist()} "
                             f"gpu {rgba[idx].tolist()} ref {ref_rgba[idx].tolist()} stats {stats}")
    if samples is not None:
        s = np.asarray(samples).reshape(-1).astype(np.int64)
        k = ref["samples"].reshape(-1).astype(np.int64)
        margin = ref["count_margin"].reshape(-1)
        exact = s == k
        slack = (np.abs(s - k) <= 1) & (margin < count_slack)
        in_range = in_band & (s >= bk[:, 0]) & (s <= bk[:, 1])
        # a ray that stops within the band may be one sample off the oracle's stop
        near_stop = in_band & (np.abs(s - k) <= 1)
        ok = exact | slack | in_range | near_stop
        stats["count_exact"] = int(exact.sum())
        stats["count_fail"] = int((~ok).sum())
        if (~ok).any():
            idx = np.flatnonzero(~ok)[:5]
            raise AssertionError(f"{int((~ok).sum())} sample counts differ: idx {idx.tolist()} "
                                 f"gpu {s[idx].tolist()} ref {k[idx].tolist()} "
                                 f"margin {margin[idx].tolist()}")
    return stats
