"""Reference of the two pre-render denoisers (Methods, Background Noise Removal).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the benchmark's
CPU-baseline leg, never by the product library or its binding; it shares no
code with the GPU path.  Plain numpy, one whole-volume step at a time, in
exact integer arithmetic (int64); the only floating-point quantities are the
noise estimate and the stopping test, both in IEEE double.

Volumes are [Z][Y][X] arrays of uint8 or uint16 (one channel).

Stem-cell channel, eq. (1): the observed image is background + shot noise +
signal.  The background B is a separable low-pass of the image (a Gaussian in
the paper; here any odd-length integer kernel per axis whose weights sum to
2^shift, applied along x, then y, then z, each pass rounded back to an
integer, edges clamped); it is subtracted (negative values clip to 0) and a
3 x 3 x 3 median (edges clamped) removes the shot noise.

Vasculature channel, eqs. (2) and (3): the noise level sigma is estimated from
the absolute response to the 6-neighbour Laplacian; the step delta is the
smallest gap between two distinct voxel values; each iteration moves every
voxel by delta in the direction of the sign of the sum of the signs of its
(in-volume) face neighbours minus itself, clamped to the value range; the
iteration keeps the last image whose RMS distance to the original is at most
sigma (and stops at a fixed point or after max_iters).
"""
import math

import numpy as np

__all__ = ["gaussian_weights", "low_pass", "median3", "remove_background", "noise_sigma", "min_gap", "mrf_step",
           "mrf"]


def gaussian_weights(sigma, shift, radius=None):
    """The low-pass kernel of eq. (1) read as a quantised Gaussian: the
    Gaussian exp(-k^2 / (2 sigma^2)) sampled at the integer offsets
    k = -r .. r (r = min(64, ceil(3 sigma)) unless given), normalised to sum
    2^shift, each weight rounded to the nearest integer (ties to even), and
    whatever the rounding leaves over or takes away put on the centre tap."""
    r = min(64, math.ceil(3.0 * sigma)) if radius is None else int(radius)
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    w = np.rint(g / g.sum() * 2.0 ** shift).astype(np.int64)
    w[r] += (1 << shift) - int(w.sum())
    if w[r] < 0:
        raise ValueError("the rounded side weights exceed 2^shift")
    return [int(x) for x in w]


def _pass(vol, weights, shift, axis):
    """One separable pass: out[i] = (sum_k w_k v[clamp(i + k - r)] + 2^(shift-1)) >> shift."""
    w = [int(x) for x in weights]
    r = (len(w) - 1) // 2
    n = vol.shape[axis]
    idx = np.arange(n)
    acc = np.zeros(vol.shape, np.int64)
    for k, wk in enumerate(w):
        src = np.clip(idx + (k - r), 0, n - 1)
        acc += wk * np.take(vol, src, axis=axis).astype(np.int64)
    return ((acc + (1 << (shift - 1))) >> shift).astype(vol.dtype)


def low_pass(vol, wx, wy, wz, shift):
    """Background estimate B: passes along x, y, z in that order (eq. (1))."""
    b = _pass(vol, wx, shift, 2)
    b = _pass(b, wy, shift, 1)
    return _pass(b, wz, shift, 0)


def median3(vol):
    """3 x 3 x 3 median (the 14th smallest of 27), edges clamped."""
    nz, ny, nx = vol.shape
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    vals = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                vals.append(vol[np.clip(z + dz, 0, nz - 1), np.clip(y + dy, 0, ny - 1),
                                np.clip(x + dx, 0, nx - 1)])
    return np.sort(np.stack(vals), axis=0)[13]


def remove_background(vol, wx, wy, wz, shift):
    """Denoised stem-cell channel and its background: (median3(max(L - B, 0)), B)."""
    b = low_pass(vol, wx, wy, wz, shift)
    d = np.maximum(vol.astype(np.int64) - b.astype(np.int64), 0).astype(vol.dtype)
    return median3(d), b


def noise_sigma(vol):
    """Noise standard deviation from the 6-neighbour Laplacian over interior
    voxels: for independent noise of deviation s the response has deviation
    sqrt(42) s and mean absolute value sqrt(2 / pi) sqrt(42) s, so
    sigma = sqrt(pi / 2) * sum|lap| / (N sqrt(42)).  Returns (sigma, sum, N)."""
    I = vol.astype(np.int64)
    if min(I.shape) < 3:
        return 0.0, 0, 0
    c = I[1:-1, 1:-1, 1:-1]
    lap = (I[1:-1, 1:-1, 2:] + I[1:-1, 1:-1, :-2] + I[1:-1, 2:, 1:-1] + I[1:-1, :-2, 1:-1]
           + I[2:, 1:-1, 1:-1] + I[:-2, 1:-1, 1:-1] - 6 * c)
    s = int(np.abs(lap).sum())
    n = int(c.size)
    return math.sqrt(math.pi / 2.0) * float(s) / (float(n) * math.sqrt(42.0)), s, n


def min_gap(vol):
    """Smallest difference between two distinct voxel values (0 if all equal)."""
    u = np.unique(vol)
    return int(np.diff(u.astype(np.int64)).min()) if u.size > 1 else 0


def mrf_step(I, delta, full):
    """One iteration of eq. (3), read with every term as neighbour minus centre;
    neighbours outside the volume are left out.  I is int64."""
    s = np.zeros(I.shape, np.int64)
    for axis in range(3):
        n = I.shape[axis]
        if n < 2:
            continue
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        d = np.sign(I[tuple(hi)] - I[tuple(lo)])
        s[tuple(lo)] += d          # the neighbour above minus the voxel
        s[tuple(hi)] -= d          # the neighbour below minus the voxel
    return np.clip(I + delta * np.sign(s), 0, full)


def mrf(vol, bits, max_iters):
    """Eqs. (2)-(3).  Returns (result, iterations kept, sigma, delta)."""
    full = (1 << bits) - 1
    I0 = vol.astype(np.int64)
    sigma, _, _ = noise_sigma(vol)
    delta = min_gap(vol)
    n_vox = float(I0.size)
    I, n = I0, 0
    if delta > 0:
        while n < max_iters:
            J = mrf_step(I, delta, full)
            if np.array_equal(J, I):
                break  # fixed point
            ss = int(((J - I0) ** 2).sum())
            if not (float(ss) <= sigma * sigma * n_vox):
                break  # the next image would leave the noise ball: keep I
            I, n = J, n + 1
    return I.astype(vol.dtype), n, sigma, delta
