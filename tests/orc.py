"""Glue between synth.Scene records and the FP64 oracle (tests only)."""
import numpy as np

import oracle


def volume(scene, data=None):
    return oracle.Volume(scene.volume if data is None else data, scene.bits,
                         scene.spacing, scene.origin)


def transfers(tfs):
    return [oracle.Transfer(t.lo, t.hi, t.curve, t.alpha_mul, t.rgb, t.visible) for t in tfs]


def camera(cam):
    return oracle.Camera(cam.projection, cam.center, cam.forward, cam.up, cam.fov_y,
                         cam.ortho_height, cam.eye_separation, cam.convergence)


def light(lt):
    return None if lt is None else oracle.Light(lt.direction, lt.ambient, lt.diffuse)


def eyes(scene):
    return (-1, 1) if scene.stereo else (0,)


def render(scene, eye=None, pixels=None, band_eps=1e-3, data=None, tfs=None, cam=None,
           term_alpha=None, nthreads=None, lit=None, stop_at=None):
    """Oracle result for one eye of a scene (eye defaults to the first);
    lit overrides the scene's light (False: unlit)."""
    if eye is None:
        eye = eyes(scene)[0]
    lt = scene.light if lit is None else (lit or None)
    return oracle.render(volume(scene, data), transfers(tfs or scene.tfs),
                         camera(cam or scene.cam), scene.width, scene.height, eye,
                         scene.step, scene.term_alpha if term_alpha is None else term_alpha,
                         band_eps, scene.background, pixels, nthreads, light(lt),
                         stop_at=stop_at)


def concat(results):
    """One result dict from several (eyes, or single-pixel renders): per-pixel
    arrays stacked (same shapes) or concatenated (flat lists of pixels), the
    band members re-indexed into the joined pixel order and padded to one
    length."""
    same = len({r["samples"].shape for r in results}) == 1 and results[0]["samples"].ndim > 1
    out = {}
    for k in results[0]:
        if k in ("band_idx", "band_rgba"):
            continue
        out[k] = (np.stack if same else np.concatenate)([r[k] for r in results])
    idx, rows, off = [], [], 0
    L = max((r["band_rgba"].shape[1] for r in results), default=0)
    for r in results:
        idx.append(r["band_idx"] + off)
        b = r["band_rgba"]
        rows.append(np.concatenate([b, np.full((b.shape[0], L - b.shape[1], 4), np.nan)], 1))
        off += r["samples"].size
    out["band_idx"] = np.concatenate(idx)
    out["band_rgba"] = np.concatenate(rows) if rows else np.zeros((0, L, 4))
    return out


def render_all(scene, band_eps=1e-3, pixels=None):
    """Per-eye oracle results joined by concat (a leading eye axis)."""
    return concat([render(scene, e, pixels=pixels, band_eps=band_eps) for e in eyes(scene)])
