"""Hand-built scenes with closed-form or invariant answers.

Used to pin the oracle (CPU) and, through the same constructions, the GPU
path.  Everything here is a voxel array plus render parameters; no rendering
arithmetic.
"""
import math

import numpy as np

from paper_1407_2089_amd.synth import TF, Cam, Scene


def ortho_down_z(nx, ny, width, height, ortho_height, forward_sign=1.0):
    """Orthographic camera looking along +z (or -z) centred over the x-y
    extent; with up = -y, image columns follow +x and rows follow +y."""
    c = ((nx - 1) / 2.0, (ny - 1) / 2.0, -5.0 if forward_sign > 0 else 1e3)
    up = (0.0, -1.0, 0.0)
    return Cam("ortho", c, (0.0, 0.0, forward_sign), up, ortho_height=ortho_height)


def slab_scene(dtype=np.uint8, bits=8, v=200, z_a=5, z_b=15, nz=24, nxy=16,
               lo=None, hi=1.0, curve=0.3, alpha_mul=0.8, rgb=(0.9, 0.6, 0.3),
               term_alpha=1.0):
    """Constant slab: voxel planes z_a..z_b (inclusive) hold v, every other
    plane is 0.  Ortho view along +z, step 1, so samples sit at half-integer z.
    The floor is placed above v / 2 so the two edge samples are transparent."""
    full = (1 << bits) - 1
    vol = np.zeros((1, nz, nxy, nxy), dtype)
    vol[0, z_a:z_b + 1] = v
    if lo is None:
        lo = 0.5 * (v / 2.0 / full + v / full)
    tf = TF(lo, hi, curve, alpha_mul, rgb)
    cam = ortho_down_z(nxy, nxy, 8, 8, 8.0)
    return Scene("slab", vol, bits, [tf], cam, 8, 8, False, 1.0, term_alpha)


def slab_closed_form(scene, v, z_a, z_b):
    """Expected interior-pixel result of slab_scene: A = 1 - (1 - a)^n with
    n = z_b - z_a interior samples, colour = capped TF colour times A; plus the
    sample count at which an early-termination threshold stops the ray."""
    tf = scene.tfs[0]
    full = (1 << scene.bits) - 1
    u = min(1.0, max(0.0, (v / full - tf.lo) / (tf.hi - tf.lo)))
    g = (1.0 - tf.curve) * u + tf.curve * u * u
    a = min(1.0, tf.alpha_mul * g)
    n = z_b - z_a
    A = 1.0 - (1.0 - a) ** n
    rgb = [min(1.0, g * c) * A for c in tf.rgb]
    n_before = z_a + 1  # transparent samples at z = -0.5 .. z_a - 0.5
    stop = None
    tau = scene.term_alpha
    if tau < 1.0 and 0.0 < a < 1.0:
        m = math.ceil(math.log(1.0 - tau) / math.log(1.0 - a))
        if m <= n:
            stop = n_before + m
            A_stop = 1.0 - (1.0 - a) ** m
            rgb = [min(1.0, g * c) * A_stop for c in tf.rgb]
            A = A_stop
    return np.array(rgb + [A]), a, stop


def linear_field(nx, ny, nz, coef=(3, 5, 7, 11), dtype=np.uint16):
    """V = alpha i + beta j + gamma k + delta (integers, within the dtype)."""
    a, b, g, d = coef
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (a * i + b * j + g * k + d).astype(dtype)[None]


def mirror_volume(seed, nx=33, ny=24, nz=20, channels=2):
    """Random volume symmetric about x = (nx - 1) / 2."""
    rng = np.random.default_rng(seed)
    half = rng.integers(0, 256, size=(channels, nz, ny, (nx + 1) // 2), dtype=np.int64)
    full = np.concatenate([half, half[..., : nx // 2][..., ::-1]], axis=-1)
    return full.astype(np.uint8)


def mirror_camera(nx, ny, nz, sep=3.0):
    """Perspective stereo camera whose centre, forward and up lie in the
    mirror plane x = (nx - 1) / 2."""
    cx = (nx - 1) / 2.0
    c = (cx, ny * 1.8, nz * 1.4)
    target = np.array([cx, (ny - 1) / 2.0, (nz - 1) / 2.0])
    fwd = target - np.array(c)
    fwd /= np.linalg.norm(fwd)
    dist = float(np.linalg.norm(target - np.array(c)))
    return Cam("perspective", c, tuple(fwd), (0.0, 0.0, 1.0), math.radians(40.0), 1.0,
               sep, dist)


def random_volume(seed, shape_czyx, dtype=np.uint8, high=None):
    rng = np.random.default_rng(seed)
    if high is None:
        high = 256 if dtype == np.uint8 else 4096
    return rng.integers(0, high, size=shape_czyx).astype(dtype)
