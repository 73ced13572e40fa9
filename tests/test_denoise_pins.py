"""Pins for the denoising oracle (Methods, Background Noise Removal): closed
forms, brute force on tiny inputs and invariants, chosen so that a wrong axis,
a dropped rounding term, a wrong window or the printed sign pattern of eq. (3)
fails at least one of them."""
import itertools
import statistics

import numpy as np
import pytest

from oracle import denoise as dn

BIN = [1, 2, 1]          # binomial low-pass, sum 4 = 2^2


def test_low_pass_of_a_constant_is_the_constant():
    v = np.full((5, 6, 7), 1234, np.uint16)
    w = [3, 10, 38, 10, 3]  # sums to 64
    assert np.array_equal(dn.low_pass(v, w, w, w, 6), v)


def test_low_pass_keeps_a_linear_ramp_away_from_the_edges():
    # Symmetric weights reproduce a linear function exactly (the odd moments
    # cancel), so every voxel at least r from the x edges keeps its value.
    nx, r = 30, 3
    v = np.zeros((4, 5, nx), np.uint16)
    v[:] = (17 * np.arange(nx) + 100)[None, None, :]
    w = [1, 6, 15, 20, 15, 6, 1]  # binomial of order 6, sum 64
    b = dn.low_pass(v, w, w, w, 6)
    assert np.array_equal(b[..., r:nx - r], v[..., r:nx - r])
    # clamped edges: the left edge sees its own value r times too often
    assert b[0, 0, 0] > v[0, 0, 0]


def test_low_pass_impulse_response_is_the_outer_product():
    # A spike of 64 A through [1, 2, 1] / 4 per axis: every pass divides
    # exactly, so B = A w_x w_y w_z (an outer product, orientation included).
    v = np.zeros((7, 9, 11), np.uint16)
    v[3, 4, 5] = 64 * 5
    wx, wy, wz = [1, 2, 1], [1, 2, 1], [1, 2, 1]
    b = dn.low_pass(v, wx, wy, wz, 2)
    exp = np.zeros_like(b, dtype=np.int64)
    for dz, dy, dx in itertools.product(range(3), repeat=3):
        exp[2 + dz, 3 + dy, 4 + dx] = 5 * wz[dz] * wy[dy] * wx[dx]
    assert np.array_equal(b.astype(np.int64), exp)


def test_low_pass_applies_each_axis_kernel_to_its_axis():
    # A spike through an asymmetric-in-size set of kernels: x wide, y none,
    # z narrow; the footprint shows which kernel went along which axis.
    v = np.zeros((9, 9, 9), np.uint16)
    v[4, 4, 4] = 4096
    b = dn.low_pass(v, [1, 4, 6, 4, 1], [16], [4, 8, 4], 4)
    nz = np.argwhere(b > 0)
    assert set(nz[:, 2]) == {2, 3, 4, 5, 6}      # x: 5 taps
    assert set(nz[:, 1]) == {4}                  # y: identity
    assert set(nz[:, 0]) == {3, 4, 5}            # z: 3 taps


def test_low_pass_weights_are_applied_as_a_correlation():
    # out[i] = sum_k w_k v[i + k - r]: the weights [0, 0, 4] / 4 read the next
    # voxel (the last one is clamped onto itself), along each axis in turn.
    v = np.arange(2 * 3 * 4, dtype=np.uint8).reshape(2, 3, 4)
    b = dn.low_pass(v, [0, 0, 4], [4], [4], 2)
    assert np.array_equal(b[..., :3], v[..., 1:]) and np.array_equal(b[..., 3], v[..., 3])
    b = dn.low_pass(v, [4], [0, 0, 4], [4], 2)
    assert np.array_equal(b[:, :2], v[:, 1:]) and np.array_equal(b[:, 2], v[:, 2])
    b = dn.low_pass(v, [4], [4], [4, 0, 0], 2)
    assert np.array_equal(b[1], v[0]) and np.array_equal(b[0], v[0])


def test_pass_rounds_half_up_once_per_pass():
    # x pass over [0, 0, 1, 0, 0] with [1, 2, 1] / 4: (1 + 2) >> 2 = 0 beside
    # the one and (2 + 2) >> 2 = 1 on it; [0, 0, 3, 0, 0] gives (3 + 2) >> 2 = 1
    # beside and (6 + 2) >> 2 = 2 on it.  A single row and plane are clamped
    # onto themselves (4 v + 2) >> 2 = v in the y and z passes.
    v = np.zeros((1, 1, 5), np.uint8)
    v[0, 0, 2] = 1
    assert dn.low_pass(v, BIN, BIN, BIN, 2).tolist() == [[[0, 0, 1, 0, 0]]]
    v[0, 0, 2] = 3
    assert dn.low_pass(v, BIN, BIN, BIN, 2).tolist() == [[[0, 1, 2, 1, 0]]]


def test_median_brute_force_on_tiny_volumes():
    rng = np.random.default_rng(7)
    for shape in [(1, 1, 1), (2, 3, 4), (3, 1, 5), (4, 4, 2)]:
        v = rng.integers(0, 1000, size=shape).astype(np.uint16)
        m = dn.median3(v)
        nz, ny, nx = shape
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            win = [int(v[min(max(z + a, 0), nz - 1), min(max(y + b, 0), ny - 1),
                         min(max(x + c, 0), nx - 1)])
                   for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
            assert m[z, y, x] == statistics.median(win)


def test_median_removes_an_isolated_spike_and_keeps_a_ramp():
    v = np.full((6, 6, 6), 50, np.uint8)
    v[2, 3, 4] = 250
    assert np.array_equal(dn.median3(v), np.full_like(v, 50))
    r = np.zeros((3, 4, 9), np.uint16)
    r[:] = (11 * np.arange(9))[None, None, :]
    assert np.array_equal(dn.median3(r), r)


def test_background_removal_of_a_spike_on_a_flat_field():
    # c + 64 A at one voxel: B = c + A (w x w x w) exactly, so L - B is
    # 56 A at the spike and negative (clipped to 0) around it; the median
    # then removes the lone non-zero voxel.
    c, A = 300, 10
    v = np.full((7, 7, 7), c, np.uint16)
    v[3, 3, 3] += 64 * A
    out, b = dn.remove_background(v, BIN, BIN, BIN, 2)
    assert b[3, 3, 3] == c + 8 * A and b[3, 3, 4] == c + 4 * A and b[0, 0, 0] == c
    assert np.array_equal(out, np.zeros_like(v))
    # a block of 3 x 3 x 3 bright voxels survives the median at its centre
    v = np.full((9, 9, 9), c, np.uint16)
    v[3:6, 3:6, 3:6] += 640
    out, _ = dn.remove_background(v, BIN, BIN, BIN, 2)
    assert out[4, 4, 4] > 0 and out[0, 0, 0] == 0


def test_min_gap():
    assert dn.min_gap(np.array([[[3, 7, 12, 7]]], np.uint16)) == 4
    assert dn.min_gap(np.array([[[9, 9]]], np.uint8)) == 0
    assert dn.min_gap(np.array([[[0, 65535, 65534]]], np.uint16)) == 1


def test_mrf_step_moves_a_spike_and_its_neighbours_by_delta():
    I = np.full((5, 5, 5), 100, np.int64)
    I[2, 2, 2] = 140
    J = dn.mrf_step(I, 3, 255)
    exp = I.copy()
    exp[2, 2, 2] -= 3        # six higher-than-neighbour terms: sum -6
    for dz, dy, dx in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        exp[2 + dz, 2 + dy, 2 + dx] += 3   # one higher neighbour: sum +1
    assert np.array_equal(J, exp)


def test_mrf_step_reading_of_the_signs_on_a_ramp():
    # Every term is neighbour minus centre: on an increasing ramp along x an
    # interior voxel sees -1 and +1 (sum 0, unchanged), the first voxel only
    # +1 (rises), the last only -1 (falls).  The printed alternation would
    # give -2 inside and lower the whole ramp.
    I = np.zeros((2, 3, 6), np.int64)
    I[:] = (10 * np.arange(6))[None, None, :]
    J = dn.mrf_step(I, 2, 1000)
    assert np.array_equal(J[..., 1:-1], I[..., 1:-1])
    assert (J[..., 0] == 2).all() and (J[..., -1] == 48).all()


def test_mrf_step_clamps_to_the_value_range():
    # After some steps values need not be delta apart: 254 below a 255
    # neighbour would rise past full scale, 1 above a 0 would fall below 0.
    I = np.array([[[254, 255]]], np.int64)
    assert dn.mrf_step(I, 2, 255).tolist() == [[[255, 253]]]
    I = np.array([[[1, 0]]], np.int64)
    assert dn.mrf_step(I, 2, 255).tolist() == [[[0, 2]]]
    I = np.array([[[255, 0, 255]]], np.int64)
    assert dn.mrf_step(I, 5, 255).tolist() == [[[250, 5, 250]]]


def test_noise_sigma_estimates_independent_noise():
    rng = np.random.default_rng(3)
    s = 20.0
    v = np.clip(np.rint(1000 + rng.normal(0, s, size=(48, 48, 48))), 0, 65535).astype(np.uint16)
    sigma, S, N = dn.noise_sigma(v)
    assert N == 46 ** 3
    assert abs(sigma / s - 1) < 0.02
    # a linear ramp has zero Laplacian inside: no noise
    r = np.zeros((5, 6, 7), np.uint16)
    r[:] = (3 * np.arange(7))[None, None, :] + (5 * np.arange(6))[None, :, None]
    assert dn.noise_sigma(r)[0] == 0.0


def test_mrf_stops_inside_the_noise_ball():
    rng = np.random.default_rng(5)
    base = np.zeros((24, 24, 24), np.float64)
    base[6:18, 6:18, 6:18] = 800
    v = np.clip(np.rint(200 + base + rng.normal(0, 15, base.shape)), 0, 4095).astype(np.uint16)
    out, n, sigma, delta = dn.mrf(v, 12, 200)
    assert delta == 1 and n > 0
    d = out.astype(np.int64) - v.astype(np.int64)
    assert float((d ** 2).sum()) <= sigma * sigma * v.size          # eq. (2) holds
    nxt = dn.mrf_step(out.astype(np.int64), delta, 4095)
    over = float(((nxt - v.astype(np.int64)) ** 2).sum()) > sigma * sigma * v.size
    assert over or n == 200                                          # and one more would not
    # denoising lowers the noise: the interior of the cube is smoother
    assert np.std(out[9:15, 9:15, 9:15].astype(float)) < np.std(v[9:15, 9:15, 9:15].astype(float))


def test_mrf_leaves_a_ramp_and_a_constant_alone():
    r = np.zeros((5, 6, 7), np.uint16)
    r[:] = (3 * np.arange(7))[None, None, :]
    out, n, sigma, _ = dn.mrf(r, 16, 50)
    assert sigma == 0.0 and n == 0 and np.array_equal(out, r)
    c = np.full((4, 4, 4), 9, np.uint8)
    out, n, _, delta = dn.mrf(c, 8, 50)
    assert delta == 0 and n == 0 and np.array_equal(out, c)


# ------------------------------------------------- quantised Gaussian weights

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                    "gaussian_sigma1_r3_shift8.txt")


def _golden_gaussian():
    with open(GOLDEN) as fh:
        rows = [l for l in fh if l.strip() and not l.startswith("#")]
    return [int(x) for x in rows[0].split()]


def test_gaussian_weights_hand_computed_case():
    # sigma 1, radius 3, shift 8: worked out by hand (fixture header)
    assert dn.gaussian_weights(1.0, 8, 3) == _golden_gaussian()


def _trunc_normal_var(sigma, a):
    """Variance of a normal N(0, sigma^2) truncated to [-a, a] (closed form)."""
    import math
    z = a / sigma
    phi = math.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return sigma * sigma * (1.0 - 2.0 * z * phi / math.erf(z / math.sqrt(2.0)))


@pytest.mark.parametrize("sigma,shift", [(1.5, 14), (2.0, 14), (3.0, 16), (4.0, 16),
                                         (10.0, 16), (16.0, 16), (20.0, 16)])
def test_gaussian_weights_properties(sigma, shift):
    import math
    w = np.array(dn.gaussian_weights(sigma, shift), np.int64)
    r = (len(w) - 1) // 2
    assert r == min(64, math.ceil(3 * sigma)) and len(w) == 2 * r + 1
    assert w.sum() == 1 << shift                     # exact sum
    assert np.array_equal(w, w[::-1])                # symmetric
    assert (w >= 0).all()
    assert (np.diff(w[:r]) >= 0).all()               # side weights rise towards the centre
    # the centre carries the rounding remainder of the 2r side weights (each
    # off by at most 1/2), so it is the exact value within r
    c = 2.0 ** shift / (1.0 + 2.0 * np.exp(-np.arange(1, r + 1) ** 2 / (2 * sigma ** 2)).sum())
    assert abs(w[r] - c) <= r + 0.5
    # each side weight follows the continuous normal density scaled to 2^shift
    # (the discrete normalisation differs from the continuous one by well
    # under 1e-3 relative for sigma >= 1.5, less the truncated tails)
    k = np.arange(-r, r + 1)
    dens = np.exp(-k * k / (2.0 * sigma * sigma)) / (sigma * math.sqrt(2.0 * math.pi))
    tail = math.erfc((r + 0.5) / (sigma * math.sqrt(2.0)))
    approx = dens / (1.0 - tail) * 2.0 ** shift
    side = np.arange(len(w)) != r
    assert np.abs(w[side] - approx[side]).max() <= 1.0 + 2e-3 * approx.max()
    # second moment: the normal truncated at r + 1/2 (midpoint rule)
    var = float((w * k * k).sum()) / 2.0 ** shift
    assert abs(var - _trunc_normal_var(sigma, r + 0.5)) <= 0.02 * sigma * sigma + 0.1


def test_gaussian_weights_remainder_goes_to_the_centre():
    # sigma 0.6, radius 2 (by hand): g = exp(-k^2 / 0.72) = 1, 0.24935,
    # 0.00387, sum 1.50644.  Shift 4: 16 g / sum = 10.621, 2.648, 0.041 ->
    # 11, 3, 0, sum 17: the centre gives one back, 10.  Shift 3: 5.311,
    # 1.324, 0.021 -> 5, 1, 0, sum 7: the centre takes one more, 6.
    assert dn.gaussian_weights(0.6, 4, 2) == [0, 3, 10, 3, 0]
    assert dn.gaussian_weights(0.6, 3, 2) == [0, 1, 6, 1, 0]
    # a flat wide kernel at a tiny shift cannot be normalised
    with pytest.raises(ValueError):
        dn.gaussian_weights(100.0, 3, 5)
