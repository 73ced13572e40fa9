"""FP64 CPU oracle for the stereo multichannel ray caster.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library or its binding.
It shares no code with the GPU path.  The arithmetic lives in ``oracle.c``;
this module only marshals numpy arrays into it through ctypes.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build

__all__ = ["Volume", "Transfer", "Camera", "Light", "sample", "gradient", "shade",
           "render", "load"]

_lib = None


class _Volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("channels", C.c_int32), ("bytes_per_voxel", C.c_int32),
                ("bits", C.c_int32), ("spacing", C.c_double * 3),
                ("origin", C.c_double * 3), ("data", C.c_void_p)]


class _Transfer(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("curve", C.c_double),
                ("alpha_mul", C.c_double), ("rgb", C.c_double * 3),
                ("visible", C.c_int32)]


class _Camera(C.Structure):
    _fields_ = [("projection", C.c_int32), ("center", C.c_double * 3),
                ("forward", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y", C.c_double), ("ortho_height", C.c_double),
                ("eye_separation", C.c_double), ("convergence", C.c_double)]


class _View(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("eye", C.c_int32),
                ("step", C.c_double), ("term_alpha", C.c_double),
                ("band_eps", C.c_double), ("background", C.c_double * 4),
                ("lit", C.c_int32), ("light_dir", C.c_double * 3),
                ("ambient", C.c_double), ("diffuse", C.c_double)]


class Light:
    """Global directional light: ``direction`` points towards the light
    (world space); shade = ambient + diffuse * max(0, n . l)."""

    def __init__(self, direction=(0.0, 0.0, -1.0), ambient=0.3, diffuse=0.7):
        self.direction = tuple(float(x) for x in direction)
        self.ambient, self.diffuse = float(ambient), float(diffuse)


def load():
    """Load liboracle.so, building it first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        lib.orc_sample.argtypes = [C.POINTER(_Volume), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
        lib.orc_sample.restype = C.c_int
        lib.orc_sample_points.argtypes = [C.POINTER(_Volume), C.c_void_p, C.c_int64,
                                          C.c_void_p]
        lib.orc_sample_points.restype = C.c_int
        P = C.c_void_p
        lib.orc_gradient_points.argtypes = [C.POINTER(_Volume), C.c_void_p, C.c_int64,
                                            C.c_void_p]
        lib.orc_gradient_points.restype = C.c_int
        lib.orc_shade.argtypes = [C.POINTER(_Volume), C.POINTER(_View), C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        lib.orc_shade.restype = C.c_int
        lib.orc_render.argtypes = [C.POINTER(_Volume), C.POINTER(_Transfer),
                                   C.POINTER(_Camera), C.POINTER(_View), P, P,
                                   C.c_int64, P, P, P, P, P, P, P, P, P, C.c_int32,
                                   C.c_int]
        lib.orc_render.restype = C.c_int
        _lib = lib
    return _lib


class Volume:
    """One frame of a multichannel volume: ``data`` is [C][Z][Y][X] uint8/uint16."""

    def __init__(self, data, bits=None, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
        data = np.ascontiguousarray(data)
        if data.ndim == 3:
            data = data[None]
        if data.dtype not in (np.uint8, np.uint16):
            raise TypeError("voxels must be uint8 or uint16")
        self.data = data
        self.bits = int(bits if bits is not None else 8 * data.dtype.itemsize)
        self.spacing = tuple(float(s) for s in spacing)
        self.origin = tuple(float(o) for o in origin)

    def _c(self):
        c, nz, ny, nx = self.data.shape
        return _Volume(nx, ny, nz, c, self.data.dtype.itemsize, self.bits,
                       (C.c_double * 3)(*self.spacing), (C.c_double * 3)(*self.origin),
                       self.data.ctypes.data)


class Transfer:
    def __init__(self, lo=0.0, hi=1.0, curve=0.0, alpha_mul=1.0, rgb=(1.0, 1.0, 1.0),
                 visible=True):
        self.lo, self.hi, self.curve, self.alpha_mul = float(lo), float(hi), float(curve), float(alpha_mul)
        self.rgb = tuple(float(x) for x in rgb)
        self.visible = bool(visible)

    def _c(self):
        return _Transfer(self.lo, self.hi, self.curve, self.alpha_mul,
                         (C.c_double * 3)(*self.rgb), int(self.visible))


class Camera:
    def __init__(self, projection="perspective", center=(0, 0, 0), forward=(0, 0, 1),
                 up=(0, -1, 0), fov_y=0.785398, ortho_height=1.0, eye_separation=0.0,
                 convergence=1.0):
        self.projection = 1 if projection in ("perspective", 1) else 0
        self.center = tuple(float(x) for x in center)
        self.forward = tuple(float(x) for x in forward)
        self.up = tuple(float(x) for x in up)
        self.fov_y = float(fov_y)
        self.ortho_height = float(ortho_height)
        self.eye_separation = float(eye_separation)
        self.convergence = float(convergence)

    def _c(self):
        d3 = C.c_double * 3
        return _Camera(self.projection, d3(*self.center), d3(*self.forward), d3(*self.up),
                       self.fov_y, self.ortho_height, self.eye_separation, self.convergence)


def sample(vol: Volume, points):
    """Trilinear field (raw intensity units) of every channel at index-space
    points [n][3] (x, y, z).  Returns float64 [n][C]."""
    lib = load()
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    cv = vol._c()
    out = np.zeros((pts.shape[0], vol.data.shape[0]), dtype=np.float64)
    lib.orc_sample_points(C.byref(cv), pts.ctypes.data, pts.shape[0], out.ctypes.data)
    return out


def _view(width, height, eye, step, term_alpha, band_eps, background, light):
    lit = light is not None
    d = light.direction if lit else (0.0, 0.0, 0.0)
    return _View(int(width), int(height), int(eye), float(step), float(term_alpha),
                 float(band_eps), (C.c_double * 4)(*[float(b) for b in background]),
                 int(lit), (C.c_double * 3)(*d), light.ambient if lit else 0.0,
                 light.diffuse if lit else 0.0)


def gradient(vol: Volume, points):
    """Central-difference gradient (raw intensity per world unit) of every
    channel at index-space points [n][3].  Returns float64 [n][C][3]."""
    lib = load()
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    cv = vol._c()
    out = np.zeros((pts.shape[0], vol.data.shape[0], 3), dtype=np.float64)
    lib.orc_gradient_points(C.byref(cv), pts.ctypes.data, pts.shape[0], out.ctypes.data)
    return out


def shade(vol: Volume, light, point):
    """Per-channel shade and shade margin at one index-space point."""
    lib = load()
    p = np.ascontiguousarray(point, dtype=np.float64).reshape(3)
    nc = vol.data.shape[0]
    s, m = np.zeros(nc), np.zeros(nc)
    cv = vol._c()
    view = _view(1, 1, 0, 1.0, 1.0, 0.0, (0, 0, 0, 0), light)
    lib.orc_shade(C.byref(cv), C.byref(view), p.ctypes.data, s.ctypes.data, m.ctypes.data)
    return s, m


def render(vol: Volume, transfers, cam: Camera, width, height, eye=0, step=1.0,
           term_alpha=1.0, band_eps=1e-3, background=(0, 0, 0, 0), pixels=None,
           nthreads=None, light=None, stop_at=None, members=True):
    """Render one eye (-1 left, 0 mono, +1 right), lit by ``light`` (a
    Light, or None for no lighting).  ``pixels`` is an optional int64 array of
    linear pixel indices j * width + i.  ``stop_at`` (optional, one int per
    rendered pixel): k >= 0 forces that ray to stop after exactly k samples
    (R_k of the acceptance rule), -1 keeps the termination threshold.
    Returns a dict of float64 / int32 numpy arrays keyed rgba, samples,
    nominal, count_margin, band_lo, band_hi, band_k, lit_margin; with
    ``members`` also band_idx (flat indices, into the rendered pixels, of the
    pixels whose band is not empty) and band_rgba [len(band_idx)][L][4]:
    member j of a pixel is R_k for k = band_k[0] + j up to band_k[1] (NaN
    past its last member)."""
    lib = load()
    if len(transfers) != vol.data.shape[0]:
        raise ValueError("one transfer function per channel is required")
    tfs = (_Transfer * len(transfers))(*[t._c() for t in transfers])
    view = _view(width, height, eye, step, term_alpha, band_eps, background, light)
    if pixels is None:
        npix = int(width) * int(height)
        pix_ptr = None
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pixels.size
        pix_ptr = pixels.ctypes.data
    stop_ptr = None
    if stop_at is not None:
        stop_at = np.ascontiguousarray(stop_at, dtype=np.int32).reshape(-1)
        if stop_at.size != npix:
            raise ValueError("stop_at needs one entry per rendered pixel")
        stop_ptr = stop_at.ctypes.data
    res = {
        "rgba": np.zeros((npix, 4), np.float64),
        "samples": np.zeros(npix, np.int32),
        "nominal": np.zeros(npix, np.int32),
        "count_margin": np.zeros(npix, np.float64),
        "band_lo": np.zeros((npix, 4), np.float64),
        "band_hi": np.zeros((npix, 4), np.float64),
        "band_k": np.zeros((npix, 2), np.int32),
        "lit_margin": np.zeros(npix, np.float64),
    }
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    cv, cc = vol._c(), cam._c()
    rc = lib.orc_render(C.byref(cv), tfs, C.byref(cc), C.byref(view), pix_ptr, stop_ptr, npix,
                        res["rgba"].ctypes.data, res["samples"].ctypes.data,
                        res["nominal"].ctypes.data, res["count_margin"].ctypes.data,
                        res["band_lo"].ctypes.data, res["band_hi"].ctypes.data,
                        res["band_k"].ctypes.data, res["lit_margin"].ctypes.data,
                        None, 0, int(nthreads))
    if rc != 0:
        raise ValueError("orc_render rejected its arguments")
    if members and stop_at is None:
        # Every member of each non-empty band: the band pixels marched once
        # more, recording R_k at each stop count k of the band (one run of
        # consecutive counts: opacity never decreases).
        bk = res["band_k"]
        idx = np.flatnonzero(bk[:, 0] >= 0)
        span = (bk[idx, 1] - bk[idx, 0] + 1) if idx.size else np.zeros(0, np.int64)
        L = int(span.max()) if idx.size else 0
        band = np.full((idx.size, L, 4), np.nan)
        if idx.size:
            all_pix = (np.arange(npix, dtype=np.int64) if pixels is None else pixels)
            sub = np.ascontiguousarray(all_pix[idx], dtype=np.int64)
            m = sub.size
            scratch = {k: np.zeros(v.shape[1:] and (m,) + v.shape[1:] or (m,), v.dtype)
                       for k, v in res.items()}
            rc = lib.orc_render(C.byref(cv), tfs, C.byref(cc), C.byref(view), sub.ctypes.data,
                                None, m, scratch["rgba"].ctypes.data,
                                scratch["samples"].ctypes.data, scratch["nominal"].ctypes.data,
                                scratch["count_margin"].ctypes.data,
                                scratch["band_lo"].ctypes.data, scratch["band_hi"].ctypes.data,
                                scratch["band_k"].ctypes.data, scratch["lit_margin"].ctypes.data,
                                band.ctypes.data, L, int(nthreads))
            if rc != 0:
                raise ValueError("orc_render rejected its arguments")
            # entries past a pixel's last member stay NaN
            for q in range(m):
                band[q, span[q]:] = np.nan
        res["band_idx"] = idx
        res["band_rgba"] = band
    if pixels is None:
        for key in res:
            if key not in ("band_idx", "band_rgba"):
                res[key] = res[key].reshape((int(height), int(width)) + res[key].shape[1:])
    return res
