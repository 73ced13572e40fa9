"""Seeded synthetic inputs: volumes, transfer functions and cameras.

These stand in for the paper's confocal sequences (Methods: adult mouse SVZ
explants, one channel of stem cells and one of ependyma / vasculature, 512 x
512 x 25 stacks every 20 minutes, low-SNR fluorescence).  The recordings are
not available, so each workload is drawn from a seed with the same shapes,
channel roles and intensity character: Gaussian blobs, ellipsoidal cells,
spline-shaped vessels and shot noise.

This module holds no rendering arithmetic.  It produces the voxel arrays and
the parameter records that both the GPU path and the CPU oracle consume.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------- parameters


@dataclass
class TF:
    """Transfer-function sliders for one channel (floor, ceiling, curve,
    alpha multiplier, colour, visibility)."""
    lo: float = 0.0
    hi: float = 1.0
    curve: float = 0.0
    alpha_mul: float = 1.0
    rgb: tuple = (1.0, 1.0, 1.0)
    visible: bool = True


@dataclass
class Cam:
    projection: str = "perspective"  # or "ortho"
    center: tuple = (0.0, 0.0, 0.0)
    forward: tuple = (0.0, 0.0, 1.0)
    up: tuple = (0.0, -1.0, 0.0)
    fov_y: float = math.radians(45.0)
    ortho_height: float = 1.0
    eye_separation: float = 0.0
    convergence: float = 1.0


@dataclass
class Light:
    """Global directional light: direction points towards the light (world
    space); a channel's colour is scaled by ambient + diffuse * max(0, n . l)."""
    direction: tuple = (0.0, 0.0, -1.0)
    ambient: float = 0.3
    diffuse: float = 0.7


@dataclass
class Scene:
    """One frame of one workload: voxels [C][Z][Y][X] plus everything a render
    request needs."""
    name: str
    volume: np.ndarray
    bits: int
    tfs: list
    cam: Cam
    width: int
    height: int
    stereo: bool
    step: float
    term_alpha: float
    background: tuple = (0.0, 0.0, 0.0, 0.0)
    spacing: tuple = (1.0, 1.0, 1.0)
    origin: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)
    light: Light = None     # None: unlit


# ------------------------------------------------------------------ cameras


def orbit_camera(dims, azimuth_deg, elevation_deg, fov_deg, dist_scale=1.0,
                 stereo=True, spacing=(1.0, 1.0, 1.0)):
    """Perspective camera looking at the volume centre from (azimuth,
    elevation); distance chosen so the bounding sphere fills the vertical
    field of view (times dist_scale).  Separation is distance / 30 and the
    zero-parallax plane passes through the volume centre."""
    nx, ny, nz = dims
    ext = np.array([(nx - 1) * spacing[0], (ny - 1) * spacing[1], (nz - 1) * spacing[2]])
    centre = ext / 2.0
    radius = 0.5 * float(np.linalg.norm([nx * spacing[0], ny * spacing[1], nz * spacing[2]]))
    dist = radius / math.sin(math.radians(fov_deg) / 2.0) * dist_scale
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    offset = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    eye = centre + dist * offset
    forward = -offset
    up = np.array([0.0, 0.0, 1.0])
    if abs(float(np.dot(up, forward))) > 0.99:
        up = np.array([0.0, 1.0, 0.0])
    return Cam("perspective", tuple(eye), tuple(forward), tuple(up), math.radians(fov_deg),
               1.0, dist / 30.0 if stereo else 0.0, dist)


def random_view_camera(rng, dims, stereo=True):
    """View direction uniform on the sphere, fov U[30, 60] degrees, distance
    R / sin(fov / 2) * U[1, 1.5]."""
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    az = math.degrees(math.atan2(v[1], v[0]))
    el = math.degrees(math.asin(max(-1.0, min(1.0, v[2]))))
    fov = rng.uniform(30.0, 60.0)
    return orbit_camera(dims, az, el, fov, rng.uniform(1.0, 1.5), stereo)


# ------------------------------------------------------------ shape stamps


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _window(shape_zyx, centre_xyz, half):
    nz, ny, nx = shape_zyx
    lo = [max(0, int(math.floor(centre_xyz[a] - half))) for a in range(3)]
    hi = [min((nx, ny, nz)[a], int(math.ceil(centre_xyz[a] + half)) + 1) for a in range(3)]
    if any(hi[a] <= lo[a] for a in range(3)):
        return None
    z, y, x = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                          np.arange(lo[0], hi[0]), indexing="ij")
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    return sl, x.astype(np.float32), y.astype(np.float32), z.astype(np.float32)


def stamp_ellipsoid(buf, centre, radii, rot, peak):
    """Max-combine an ellipsoid with a one-voxel soft edge into buf [Z][Y][X]."""
    w = _window(buf.shape, centre, max(radii) + 1.5)
    if w is None:
        return
    sl, x, y, z = w
    d = np.stack([x - centre[0], y - centre[1], z - centre[2]], axis=-1)
    q = d @ rot  # local coordinates (rot columns are the axes)
    rho = np.sqrt(((q / np.asarray(radii)) ** 2).sum(-1))
    s = (rho - 1.0) * min(radii)
    val = peak * np.clip(0.5 - s, 0.0, 1.0)
    np.maximum(buf[sl], val.astype(buf.dtype), out=buf[sl])


def catmull_rom(points, per_unit=2.0):
    """Dense samples of the Catmull-Rom cubic spline through the control
    points (end points repeated)."""
    p = np.asarray(points, dtype=np.float64)
    p = np.vstack([p[:1], p, p[-1:]])
    out = []
    for s in range(1, len(p) - 2):
        p0, p1, p2, p3 = p[s - 1], p[s], p[s + 1], p[s + 2]
        n = max(2, int(np.linalg.norm(p2 - p1) * per_unit))
        t = np.linspace(0.0, 1.0, n, endpoint=False)[:, None]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t * t
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t * t * t))
    out.append(p[-2][None])
    return np.vstack(out)


def stamp_tube(buf, points, radius, peak):
    """Max-combine a tube of the given radius (soft one-voxel edge) around a
    dense polyline into buf."""
    for c in points:
        w = _window(buf.shape, c, radius + 1.5)
        if w is None:
            continue
        sl, x, y, z = w
        dist = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        val = peak * np.clip(radius + 0.5 - dist, 0.0, 1.0)
        np.maximum(buf[sl], val.astype(buf.dtype), out=buf[sl])


# ---------------------------------------------------------------- volumes


def blobs_u8(dims, n_blobs, sigma, peak, noise_max, seed):
    """Gaussian blobs (centres U[8, n - 8]) plus integer-uniform noise, uint8."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    val = np.zeros((nz, ny, nx), np.float64)
    for _ in range(n_blobs):
        c = [rng.uniform(8, n - 8) for n in (nx, ny, nz)]
        r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
        val += peak * np.exp(-r2 / (2.0 * sigma * sigma))
    val += rng.integers(0, noise_max + 1, size=val.shape)
    return np.clip(np.rint(val), 0, 255).astype(np.uint8)[None]


def cells_and_vessels(dims, channels, bits, seed, n_cells=40, n_tubes=10,
                      background=100.0):
    """Confocal-like multichannel frame, [C][Z][Y][X].  Channel 0: ellipsoidal
    cells (radii U[4, 8]); channel 1: cubic-spline vessels (radius 3);
    channels 2 and 3: small round nuclei and puncta.  Counts scale with the
    volume.  Shot noise: Poisson(background + signal), clipped to full scale."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    full = (1 << bits) - 1
    scale = full / 4095.0
    out_dtype = np.uint8 if bits <= 8 else np.uint16
    vol = np.zeros((channels, nz, ny, nx), out_dtype)
    for c in range(channels):
        sig = np.zeros((nz, ny, nx), np.float32)
        if c == 0:
            for _ in range(n_cells):
                centre = [rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)]
                radii = rng.uniform(4.0, 8.0, size=3)
                stamp_ellipsoid(sig, centre, radii, _rotation(rng), rng.uniform(1200, 3000) * scale)
        elif c == 1:
            for _ in range(n_tubes):
                k = int(rng.integers(4, 7))
                ctrl = np.column_stack([rng.uniform(0, nx, k), rng.uniform(0, ny, k),
                                        rng.uniform(0, nz, k)])
                stamp_tube(sig, catmull_rom(ctrl), 3.0, rng.uniform(1500, 3500) * scale)
        else:
            n = max(1, n_cells * (4 if c == 2 else 20) // 4)
            rad = 2.0 if c == 2 else 1.0
            for _ in range(n):
                centre = [rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)]
                stamp_ellipsoid(sig, centre, (rad, rad, rad), np.eye(3),
                                rng.uniform(1200, 3000) * scale)
        noisy = rng.poisson(background * scale + sig.astype(np.float64))
        vol[c] = np.minimum(noisy, full).astype(out_dtype)
    return vol


# ------------------------------------------------ large volumes on the GPU


def _stamp_ellipsoids_t(torch, sig, centres, radii, rots, peaks):
    """Max-combine ellipsoids (one-voxel soft edge) into sig [Z][Y][X] (torch)."""
    nz, ny, nx = sig.shape
    dev = sig.device
    for c, r, R, pk in zip(centres, radii, rots, peaks):
        h = float(max(r)) + 1.5
        lo = [max(0, int(math.floor(c[a] - h))) for a in range(3)]
        hi = [min((nx, ny, nz)[a], int(math.ceil(c[a] + h)) + 1) for a in range(3)]
        if any(hi[a] <= lo[a] for a in range(3)):
            continue
        z = torch.arange(lo[2], hi[2], device=dev, dtype=torch.float32).view(-1, 1, 1) - c[2]
        y = torch.arange(lo[1], hi[1], device=dev, dtype=torch.float32).view(1, -1, 1) - c[1]
        x = torch.arange(lo[0], hi[0], device=dev, dtype=torch.float32).view(1, 1, -1) - c[0]
        q = [x * float(R[0, k]) + y * float(R[1, k]) + z * float(R[2, k]) for k in range(3)]
        rho = torch.sqrt((q[0] / r[0]) ** 2 + (q[1] / r[1]) ** 2 + (q[2] / r[2]) ** 2)
        val = pk * torch.clamp(0.5 - (rho - 1.0) * float(min(r)), 0.0, 1.0)
        view = sig[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        torch.maximum(view, val, out=view)


def _stamp_tube_t(torch, sig, pts, radius, peak, chunk=24):
    """Max-combine a tube around a dense polyline, chunk by chunk (torch)."""
    nz, ny, nx = sig.shape
    dev = sig.device
    P = torch.as_tensor(pts, dtype=torch.float32, device=dev)
    for s0 in range(0, len(pts), chunk):
        seg = P[s0:s0 + chunk]
        mn = seg.min(0).values - radius - 1.5
        mx = seg.max(0).values + radius + 1.5
        lo = [max(0, int(math.floor(float(mn[a])))) for a in range(3)]
        hi = [min((nx, ny, nz)[a], int(math.ceil(float(mx[a]))) + 1) for a in range(3)]
        if any(hi[a] <= lo[a] for a in range(3)):
            continue
        z = torch.arange(lo[2], hi[2], device=dev, dtype=torch.float32)
        y = torch.arange(lo[1], hi[1], device=dev, dtype=torch.float32)
        x = torch.arange(lo[0], hi[0], device=dev, dtype=torch.float32)
        d2 = None
        for pnt in seg:
            e = ((z - pnt[2]) ** 2).view(-1, 1, 1) + ((y - pnt[1]) ** 2).view(1, -1, 1) + \
                ((x - pnt[0]) ** 2).view(1, 1, -1)
            d2 = e if d2 is None else torch.minimum(d2, e)
        val = peak * torch.clamp(radius + 0.5 - torch.sqrt(d2), 0.0, 1.0)
        view = sig[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        torch.maximum(view, val, out=view)


class DeviceSeries:
    """Seeded confocal-like time series generated on the GPU, one frame at a
    time: objects are drawn once (numpy generator), cells move by a random
    walk from frame to frame, and each frame gets fresh shot noise from a
    device generator seeded per (seed, frame).  Channel roles: 0 cells,
    1 vessels (static), 2 nuclei, 3 puncta.  Returns frames as torch tensors
    [C][Z][Y][X] (uint8, or int16 holding uint16 bits)."""

    def __init__(self, dims, channels, bits, seed, frames=1, device="cuda", density=1.0,
                 walk_sigma=1.0, background=100.0):
        import torch
        self.torch = torch
        self.dims, self.channels, self.bits, self.seed = tuple(dims), channels, bits, seed
        self.frames, self.device, self.walk = frames, device, walk_sigma
        self.background = background
        rng = np.random.default_rng(seed)
        nx, ny, nz = dims
        full = (1 << bits) - 1
        self.scale = full / 4095.0
        vol_frac = nx * ny * nz / float(512 * 512 * 64)
        n_cells = max(1, int(round(40 * vol_frac * density)))
        n_tubes = max(1, int(round(10 * math.sqrt(vol_frac) * density)))
        self.cells = [(np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)]),
                       rng.uniform(4.0, 8.0, size=3), _rotation(rng),
                       rng.uniform(1200, 3000) * self.scale) for _ in range(n_cells)]
        self.tubes = []
        for _ in range(n_tubes):
            k = int(rng.integers(4, 7))
            ctrl = np.column_stack([rng.uniform(0, nx, k), rng.uniform(0, ny, k),
                                    rng.uniform(0, nz, k)])
            self.tubes.append((catmull_rom(ctrl, per_unit=1.0), rng.uniform(1500, 3500) * self.scale))
        self.small = []
        # channels 2-5: nuclei (radius 2), puncta (1), large bodies (3), small
        # puncta (1.5); drawn in this order so that fewer channels draw the
        # same objects
        for c, (per, rad) in zip((2, 3, 4, 5), ((4, 2.0), (20, 1.0), (1, 3.0), (10, 1.5))):
            n = max(1, n_cells * per // 4)
            self.small.append([(np.array([rng.uniform(0, nx), rng.uniform(0, ny),
                                          rng.uniform(0, nz)]), rad,
                                rng.uniform(1200, 3000) * self.scale) for _ in range(n)])
        self.walk_rng = np.random.default_rng(seed + 7919)
        self.walk_steps = [self.walk_rng.normal(0.0, walk_sigma, size=(len(self.cells), 3))
                           for _ in range(frames)]
        self._static = None

    def _static_channels(self):
        torch = self.torch
        if self._static is None:
            nx, ny, nz = self.dims
            st = {}
            if self.channels > 1:
                sig = torch.zeros((nz, ny, nx), dtype=torch.float32, device=self.device)
                for pts, pk in self.tubes:
                    _stamp_tube_t(torch, sig, pts, 3.0, float(pk))
                st[1] = sig
            for c in range(2, self.channels):
                sig = torch.zeros((nz, ny, nx), dtype=torch.float32, device=self.device)
                objs = self.small[c - 2]
                _stamp_ellipsoids_t(torch, sig, [o[0] for o in objs],
                                    [(o[1],) * 3 for o in objs], [np.eye(3)] * len(objs),
                                    [float(o[2]) for o in objs])
                st[c] = sig
            self._static = st
        return self._static

    def frame(self, t):
        torch = self.torch
        nx, ny, nz = self.dims
        full = (1 << self.bits) - 1
        offs = np.zeros((len(self.cells), 3))
        for k in range(1, t + 1):
            offs += self.walk_steps[k]
        sig0 = torch.zeros((nz, ny, nx), dtype=torch.float32, device=self.device)
        _stamp_ellipsoids_t(torch, sig0, [c[0] + o for c, o in zip(self.cells, offs)],
                            [c[1] for c in self.cells], [c[2] for c in self.cells],
                            [float(c[3]) for c in self.cells])
        st = self._static_channels()
        g = torch.Generator(device=self.device)
        g.manual_seed(int(self.seed) * 1000003 + int(t))
        out_dtype = torch.uint8 if self.bits <= 8 else torch.int16
        out = torch.empty((self.channels, nz, ny, nx), dtype=out_dtype, device=self.device)
        for c in range(self.channels):
            sig = sig0 if c == 0 else st[c]
            lam = sig + self.background * self.scale
            noisy = torch.poisson(lam, generator=g).clamp_(max=full)
            if out_dtype == torch.uint8:
                out[c] = noisy.to(torch.uint8)
            else:
                out[c] = noisy.to(torch.int32).to(torch.int16)
            del noisy, lam
        return out


# --------------------------------------------------------------- workloads


def tiny_scene(seed=1):
    """1-channel 64x64x32 uint8: three Gaussian blobs (sigma 3, peak 200)
    plus uniform noise 0..20; one 256x256 orthographic mono view along +z,
    step 0.5, linear-ramp alpha, no early termination."""
    vol = blobs_u8((64, 64, 32), 3, 3.0, 200.0, 20, seed)
    cam = Cam("ortho", (31.5, 31.5, -10.0), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0),
              ortho_height=64.0)
    return Scene("tiny 1ch u8 64x64x32, 256x256 ortho mono", vol, 8, [TF()], cam,
                 256, 256, False, 0.5, 1.0)


def realistic_scene(seed=2, width=1920, height=1080, dims=(512, 512, 64), volume=True):
    """2-channel 12-bit uint16 512x512x64: 40 ellipsoidal cells (green) and 10
    spline vessels (red) with Poisson noise; perspective stereo 1920x1080 per
    eye from azimuth 30, elevation 50 degrees, fov 45; step 1, early
    termination at alpha 0.99.  volume=False leaves the voxels out (None):
    the render parameters alone."""
    vol = cells_and_vessels(dims, 2, 12, seed, n_cells=40, n_tubes=10) if volume else None
    cam = orbit_camera(dims, 30.0, 50.0, 45.0)
    lo, hi = 300.0 / 4095.0, 3000.0 / 4095.0
    tfs = [TF(lo, hi, 0.0, 1.0, (0.0, 1.0, 0.0)), TF(lo, hi, 0.0, 1.0, (1.0, 0.0, 0.0))]
    return Scene(f"realistic 2ch u16-12 {dims[0]}x{dims[1]}x{dims[2]}, "
                 f"{width}x{height} perspective stereo", vol, 12, tfs, cam,
                 width, height, True, 1.0, 0.99)


SCENES = {"tiny": tiny_scene, "realistic": realistic_scene}


def montage(dims, channels, seed, tile=(1024, 1024), distinct=3, device="cuda", log=None):
    """Seeded stand-in for a stitched confocal montage, [C][Z][Y][X] uint8 on
    the GPU: a grid of tile-sized fields cut from `distinct` generated 8-bit
    frames (DeviceSeries, full depth), tile (gx, gy) taking frame
    (gx + 2 gy) mod distinct, mirrored in x on odd columns and in y on odd
    rows, the last row and column cropped to the montage's edge.  `log`, if
    given, is called with a line per generated frame."""
    import torch
    nx, ny, nz = dims
    tx, ty = tile
    tiles = []
    for k in range(distinct):
        tiles.append(DeviceSeries((tx, ty, nz), channels, 8, seed + 101 * k,
                                  device=device).frame(0))
        if log is not None:
            log(f"montage tile frame {k + 1} of {distinct} generated")
    out = torch.empty((channels, nz, ny, nx), dtype=torch.uint8, device=device)
    for gy in range((ny + ty - 1) // ty):
        for gx in range((nx + tx - 1) // tx):
            t = tiles[(gx + 2 * gy) % distinct]
            if gx % 2:
                t = t.flip(3)
            if gy % 2:
                t = t.flip(2)
            w, h = min(tx, nx - gx * tx), min(ty, ny - gy * ty)
            out[:, :, gy * ty:gy * ty + h, gx * tx:gx * tx + w] = t[:, :, :h, :w]
    return out
