"""Crops of the oracle's input for single rays (test infrastructure, like the
rest of oracle/).

A volume too large to copy to the host whole is checked pixel by pixel: the
oracle renders each sampled pixel on the crop of voxels its ray can read,
with the crop's origin moved to the crop's first voxel, which gives that ray
the same samples as the whole volume.  The ray and its clip against the
extended box [-1, n] follow the camera model of the oracle (pixel centres,
off-axis stereo eyes, orthographic screen rectangle).
"""
import numpy as np


def ray_crop(cam, W, H, eye, px, py, dims, margin=3):
    """Index-space box [lo, hi) holding the part of pixel (px, py)'s ray that
    lies in the volume's extended box [-1, n] per axis, widened by `margin`
    voxels and clipped to the grid (unit spacing, origin 0); None if the ray
    misses."""
    f = np.array(cam.forward, float)
    f /= np.linalg.norm(f)
    rt = np.cross(f, np.array(cam.up, float))
    rt /= np.linalg.norm(rt)
    u = np.cross(rt, f)
    sx = (px + 0.5) * 2.0 / W - 1.0
    sy = 1.0 - (py + 0.5) * 2.0 / H
    c = np.array(cam.center, float)
    if cam.projection == "perspective":
        h = cam.convergence * np.tan(0.5 * cam.fov_y)
        w = h * W / H
        s = float(eye)
        o = c + s * 0.5 * cam.eye_separation * rt
        d = cam.convergence * f - s * 0.5 * cam.eye_separation * rt + sx * w * rt + sy * h * u
        t0 = 0.0
    else:
        h = 0.5 * cam.ortho_height
        w = h * W / H
        o = c + sx * w * rt + sy * h * u
        d = f
        t0 = -np.inf
    t1 = np.inf
    n = np.array(dims, float)
    for a in range(3):
        if d[a] != 0.0:
            ta, tb = (-1.0 - o[a]) / d[a], (n[a] - o[a]) / d[a]
            t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
        elif not -1.0 <= o[a] <= n[a]:
            return None
    if not t0 < t1:
        return None
    p0, p1 = o + t0 * d, o + t1 * d
    lo = np.maximum(np.floor(np.minimum(p0, p1)) - margin, 0).astype(int)
    hi = np.minimum(np.ceil(np.maximum(p0, p1)) + margin + 1, n).astype(int)
    return lo, hi
