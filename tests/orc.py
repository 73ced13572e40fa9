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
           term_alpha=None, nthreads=None, lit=None):
    """Oracle result for one eye of a scene (eye defaults to the first);
    lit overrides the scene's light (False: unlit)."""
    if eye is None:
        eye = eyes(scene)[0]
    lt = scene.light if lit is None else (lit or None)
    return oracle.render(volume(scene, data), transfers(tfs or scene.tfs),
                         camera(cam or scene.cam), scene.width, scene.height, eye,
                         scene.step, scene.term_alpha if term_alpha is None else term_alpha,
                         band_eps, scene.background, pixels, nthreads, light(lt))


def render_all(scene, band_eps=1e-3, pixels=None):
    """Stacked per-eye oracle results: dict of arrays with a leading eye axis."""
    outs = [render(scene, e, pixels=pixels, band_eps=band_eps) for e in eyes(scene)]
    return {k: np.stack([o[k] for o in outs]) for k in outs[0]}
