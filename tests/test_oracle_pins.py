"""Pins for the FP64 oracle: closed forms, invariants and brute force.

Each test fixes a result by something other than the oracle's own code, so
that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import orc
import scenes
from paper_1407_2089_amd.synth import TF, Cam, Light, Scene


# ------------------------------------------------------------------ P1 empty

@pytest.mark.parametrize("invisible", [False, True])
def test_p1_empty_volume_returns_background(invisible):
    vol = np.zeros((2, 12, 10, 14), np.uint16)
    if invisible:
        vol[:] = 3000
    tfs = [TF(0.0, 1.0, visible=not invisible), TF(0.1, 0.9, 0.5, visible=not invisible)]
    cam = scenes.mirror_camera(14, 10, 12)
    bg = (0.2, 0.3, 0.4, 0.5)
    sc = Scene("p1", vol, 12, tfs, cam, 21, 13, True, 0.7, 0.95, bg)
    for eye in (-1, 1):
        r = orc.render(sc, eye)
        exp = np.array([bg[3] * bg[0], bg[3] * bg[1], bg[3] * bg[2], bg[3]])
        assert np.array_equal(r["rgba"], np.broadcast_to(exp, r["rgba"].shape))
    assert (r["nominal"] > 0).any()  # rays did cross the box


# ------------------------------------------------------------------ P2 slab

@pytest.mark.parametrize("dtype,bits,v", [(np.uint8, 8, 200), (np.uint16, 12, 2500),
                                          (np.uint16, 16, 40000)])
def test_p2_constant_slab_closed_form(dtype, bits, v):
    sc = scenes.slab_scene(dtype, bits, v, z_a=5, z_b=15)
    exp, a, _ = scenes.slab_closed_form(sc, v, 5, 15)
    assert 0.0 < a < 1.0
    r = orc.render(sc)
    np.testing.assert_allclose(r["rgba"].reshape(-1, 4), np.broadcast_to(exp, (64, 4)),
                               rtol=0, atol=1e-12)
    # every sample in the extended box is taken: z from -1 to nz, step 1
    assert (r["samples"] == sc.volume.shape[1] + 1).all()


@pytest.mark.parametrize("tau", [0.5, 0.9, 0.99])
def test_p2_slab_early_termination(tau):
    sc = scenes.slab_scene(alpha_mul=1.0, curve=0.0, term_alpha=tau, z_a=3, z_b=20, nz=26)
    exp, a, stop = scenes.slab_closed_form(sc, 200, 3, 20)
    assert stop is not None
    r = orc.render(sc, band_eps=1e-9)
    assert (r["samples"] == stop).all()
    np.testing.assert_allclose(r["rgba"].reshape(-1, 4), np.broadcast_to(exp, (64, 4)),
                               rtol=0, atol=1e-12)
    # termination never costs more than 1 - tau of any component
    full = orc.render(sc, term_alpha=1.0)
    assert np.abs(full["rgba"] - r["rgba"]).max() <= 1.0 - tau + 1e-12


def test_p2_termination_band_brackets_neighbours():
    # alpha per sample chosen so that A_k lands within eps of tau at one k
    sc = scenes.slab_scene(alpha_mul=1.0, curve=0.0, term_alpha=0.99, z_a=3, z_b=40, nz=44)
    exp, a, stop = scenes.slab_closed_form(sc, 200, 3, 40)
    m = stop - 4  # interior samples at the stop
    A = [1 - (1 - a) ** k for k in range(m - 3, m + 4)]
    eps = max(abs(x - 0.99) for x in A[2:5]) + 1e-9
    r = orc.render(sc, band_eps=eps)
    lo, hi = r["band_k"][..., 0], r["band_k"][..., 1]
    inside = [k + 4 for k, x in zip(range(m - 3, m + 4), A) if abs(x - 0.99) <= eps]
    members = inside + [k + 1 for k in inside]  # and one sample past each of them
    assert (lo == min(members)).all() and (hi == max(members)).all()
    # the band's colour range covers exactly those stops
    g = (200 / 255 - sc.tfs[0].lo) / (1 - sc.tfs[0].lo)
    Ak = [1 - (1 - a) ** (k - 4) for k in members]
    exp_lo = min(Ak) * g * np.array(sc.tfs[0].rgb)
    exp_hi = max(Ak) * g * np.array(sc.tfs[0].rgb)
    np.testing.assert_allclose(r["band_lo"][..., :3].reshape(-1, 3), np.broadcast_to(exp_lo, (64, 3)),
                               atol=1e-12)
    np.testing.assert_allclose(r["band_hi"][..., :3].reshape(-1, 3), np.broadcast_to(exp_hi, (64, 3)),
                               atol=1e-12)


def test_p2_band_members_are_the_forced_stops_closed_form():
    # Each member R_k of the termination band is the ray stopped after exactly
    # k samples: on the slab, transparent samples until z_a and then
    # A_k = 1 - (1 - a)^(k - z_a - 1), colour g rgb A_k, for every k of the
    # band's range, in order.
    sc = scenes.slab_scene(alpha_mul=1.0, curve=0.0, term_alpha=0.99, z_a=3, z_b=40, nz=44)
    _, a, stop = scenes.slab_closed_form(sc, 200, 3, 40)
    r = orc.render(sc, band_eps=4e-3)
    assert r["band_idx"].size == 64  # every interior ray crosses the band
    g = (200 / 255 - sc.tfs[0].lo) / (1 - sc.tfs[0].lo)
    k0, k1 = r["band_k"].reshape(-1, 2)[0]
    assert k0 <= stop <= k1 and k1 - k0 >= 1
    for j, k in enumerate(range(k0, k1 + 1)):
        A = 1 - (1 - a) ** (k - 4)
        exp = [A * g * c for c in sc.tfs[0].rgb] + [A]
        np.testing.assert_allclose(r["band_rgba"][:, j], np.broadcast_to(exp, (64, 4)),
                                   rtol=0, atol=1e-12)
    assert np.isnan(r["band_rgba"][:, k1 - k0 + 1:]).all()
    # a forced stop past the last sample gives the full ray
    full = orc.render(sc, term_alpha=1.0)
    late = orc.render(sc, stop_at=np.full(64, 10_000), term_alpha=0.99)
    np.testing.assert_array_equal(late["rgba"], full["rgba"])
    # and a forced stop at 0 gives the background
    none = orc.render(sc, stop_at=np.zeros(64), term_alpha=0.99)
    assert not none["rgba"].any()


def test_p2_background_behind_partial_opacity_closed_form():
    # Slab of opacity 0 < A < 1 over a coloured background:
    # rgb = A g c + (1 - A) bg_a bg_rgb, alpha = A + (1 - A) bg_a.
    sc = scenes.slab_scene(dtype=np.uint16, bits=12, v=2500, z_a=5, z_b=8)
    exp, a, _ = scenes.slab_closed_form(sc, 2500, 5, 8)
    A = exp[3]
    assert 0.2 < A < 0.8
    for bg in ((0.2, 0.5, 0.9, 0.6), (1.0, 0.0, 0.3, 1.0), (0.7, 0.7, 0.1, 0.25)):
        sc.background = bg
        r = orc.render(sc)["rgba"].reshape(-1, 4)
        want = [exp[q] + (1 - A) * bg[3] * bg[q] for q in range(3)] + [A + (1 - A) * bg[3]]
        np.testing.assert_allclose(r, np.broadcast_to(want, r.shape), rtol=0, atol=1e-12)


def test_acceptance_rule_is_per_band_member():
    # A pixel in the band passes when it is within tol of one member, not
    # merely inside the componentwise box around all members.
    import gpu
    sc = scenes.slab_scene(alpha_mul=1.0, curve=0.0, term_alpha=0.99, z_a=3, z_b=40, nz=44,
                           rgb=(0.9, 0.1, 0.5))
    ref = orc.render(sc, band_eps=1e-3)
    members = ref["band_rgba"][0]
    members = members[~np.isnan(members[:, 0])]
    assert len(members) >= 2
    tol = 1e-3
    for m in members:  # every member passes, with its own sample count
        gpu.compare(np.broadcast_to(m, (8, 8, 4)), None, ref, tol)
    # a point inside the box [min - tol, max + tol] but far from every member:
    # red from the first member, alpha from the last
    odd = members[0].copy()
    odd[3] = members[-1][3]
    assert np.abs(members - odd).max(-1).min() > tol
    with pytest.raises(AssertionError):
        gpu.compare(np.broadcast_to(odd, (8, 8, 4)), None, ref, tol)


def test_p2_two_channel_slab_merge_closed_form():
    # Both channels fill the same planes.  The sample's alpha is the larger
    # channel alpha (capped at 1); its colour is the per-component sum of the
    # channel colours, capped at 1.
    v0, v1 = 200, 120
    vol = np.zeros((2, 20, 16, 16), np.uint8)
    vol[0, 4:8] = v0
    vol[1, 4:8] = v1
    lo0 = 0.5 * (v0 / 2 / 255 + v0 / 255)
    lo1 = 0.5 * (v0 / 2 / 255 + v1 / 255)  # above both channels' edge values
    tfs = [TF(lo0, 0.7, 0.2, 0.6, (0.8, 0.7, 0.1)), TF(lo1, 0.5, -0.3, 1.2, (0.5, 0.2, 0.3))]
    sc = Scene("p2m", vol, 8, tfs, scenes.ortho_down_z(16, 16, 8, 8, 8.0), 8, 8, False,
               1.0, 1.0)
    g = []
    for t, v in zip(tfs, (v0, v1)):
        u = min(1.0, max(0.0, (v / 255 - t.lo) / (t.hi - t.lo)))
        g.append((1 - t.curve) * u + t.curve * u * u)
    a = min(1.0, max(tfs[0].alpha_mul * g[0], tfs[1].alpha_mul * g[1]))
    assert abs(tfs[0].alpha_mul * g[0] - tfs[1].alpha_mul * g[1]) > 0.05
    rgb = [min(1.0, g[0] * tfs[0].rgb[q] + g[1] * tfs[1].rgb[q]) for q in range(3)]
    assert rgb[0] == 1.0 and rgb[1] < 1.0  # the cap is exercised on red only
    A = 1 - (1 - a) ** 3  # three interior samples: z = 4.5, 5.5, 6.5
    r = orc.render(sc)["rgba"].reshape(-1, 4)
    np.testing.assert_allclose(r, np.broadcast_to([c * A for c in rgb] + [A], r.shape),
                               rtol=0, atol=1e-12)


# ------------------------------------------------------------ P3 trilinear

def test_p3_linear_field_is_reproduced_exactly():
    nx, ny, nz = 9, 7, 6
    coef = (3, 5, 7, 11)
    vol = oracle.Volume(scenes.linear_field(nx, ny, nz, coef), 16)
    rng = np.random.default_rng(0)
    pts = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1], size=(500, 3))
    got = oracle.sample(vol, pts)[:, 0]
    exp = coef[0] * pts[:, 0] + coef[1] * pts[:, 1] + coef[2] * pts[:, 2] + coef[3]
    np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-12)


def test_p3_voxel_centres_zero_outside_and_faces():
    rng = np.random.default_rng(1)
    data = rng.integers(0, 4096, size=(3, 5, 6, 7)).astype(np.uint16)
    vol = oracle.Volume(data, 12)
    k, j, i = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()], -1).astype(np.float64)
    got = oracle.sample(vol, pts)
    exp = data.reshape(3, -1).T.astype(np.float64)
    assert np.array_equal(got, exp)
    # all eight taps outside the grid -> 0
    out = oracle.sample(vol, [[-1.5, 2, 2], [7.2, 1, 1], [3, -1.01, 2], [3, 2, 5.5]])
    assert np.all(out == 0)
    # on the faces of the extended box [-1, n] the field is exactly 0 ...
    face = oracle.sample(vol, [[-1.0, 2.3, 1.7], [7.0, 2.3, 1.7], [3.1, -1.0, 2.2],
                               [3.1, 6.0, 2.2], [3.1, 2.2, -1.0], [3.1, 2.2, 5.0]])
    assert np.all(face == 0)
    # ... and halfway from the face to the first voxel it is half that voxel
    half = oracle.sample(vol, [[-0.5, 2.0, 1.0]])[0]
    assert np.array_equal(half, 0.5 * data[:, 1, 2, 0])
    # continuity across the last voxel: approaching x = n from inside
    near = oracle.sample(vol, [[7.0 - 1e-9, 2.0, 1.0]])[0]
    assert np.all(np.abs(near) < 1e-5)


# ------------------------------------------------------------ P4 stereo mirror

def test_p4_mirror_symmetric_volume_gives_mirrored_eyes():
    nx, ny, nz = 33, 24, 20
    vol = scenes.mirror_volume(4, nx, ny, nz)
    cam = scenes.mirror_camera(nx, ny, nz, sep=3.0)
    tfs = [TF(0.1, 0.9, 0.2, 0.6, (0.2, 0.9, 0.1)), TF(0.3, 0.8, -0.4, 1.3, (0.9, 0.1, 0.5))]
    sc = Scene("p4", vol, 8, tfs, cam, 40, 30, True, 0.8, 0.97)
    left = orc.render(sc, -1)
    right = orc.render(sc, 1)
    assert left["rgba"][..., 3].max() > 0.2
    np.testing.assert_allclose(left["rgba"], right["rgba"][:, ::-1], rtol=0, atol=1e-12)
    assert not np.allclose(left["rgba"], right["rgba"], atol=1e-3)  # parallax is visible


def test_p4_zero_separation_stereo_equals_mono():
    nx, ny, nz = 20, 17, 11
    vol = scenes.random_volume(5, (1, nz, ny, nx))
    cam = scenes.mirror_camera(nx, ny, nz, sep=0.0)
    sc = Scene("p4b", vol, 8, [TF(0.2, 0.9)], cam, 24, 18, True, 0.5, 0.98)
    mono = orc.render(sc, 0)["rgba"]
    for eye in (-1, 1):
        assert np.array_equal(orc.render(sc, eye)["rgba"], mono)


# ------------------------------------------------------------- P5 order

def test_p5_front_to_back_order_of_two_slabs():
    nz = 20
    vol = np.zeros((2, nz, 8, 8), np.uint8)
    vol[0, 4:6] = 200   # red slab, nearer when looking along +z
    vol[1, 12:14] = 150  # green slab
    lo = 0.5 * (100 / 255 + 200 / 255)  # only the slab-interior sample of ch0 is opaque-ish
    tf0 = TF(lo, 1.0, 0.0, 1.0, (1.0, 0.0, 0.0))
    lo1 = 0.5 * (75 / 255 + 150 / 255)
    tf1 = TF(lo1, 1.0, 0.0, 1.0, (0.0, 1.0, 0.0))
    g1 = (200 / 255 - lo) / (1.0 - lo)
    g2 = (150 / 255 - lo1) / (1.0 - lo1)
    a1, a2 = g1, g2
    for sign in (1.0, -1.0):
        cam = scenes.ortho_down_z(8, 8, 4, 4, 4.0, forward_sign=sign)
        sc = Scene("p5", vol, 8, [tf0, tf1], cam, 4, 4, False, 1.0, 1.0)
        r = orc.render(sc)["rgba"].reshape(-1, 4)
        if sign > 0:
            exp = [a1 * g1, (1 - a1) * a2 * g2, 0.0, a1 + (1 - a1) * a2]
        else:
            exp = [(1 - a2) * a1 * g1, a2 * g2, 0.0, a2 + (1 - a2) * a1]
        np.testing.assert_allclose(r, np.broadcast_to(exp, r.shape), rtol=0, atol=1e-12)


# ------------------------------------------------------------ P6 opaque

def test_p6_opaque_first_sample():
    vol = np.full((1, 6, 8, 8), 255, np.uint8)
    sc = Scene("p6", vol, 8, [TF(0.0, 0.5, 0.0, 1.0, (0.3, 0.6, 0.9))],
               scenes.ortho_down_z(8, 8, 4, 4, 4.0), 4, 4, False, 1.0, 1.0)
    r = orc.render(sc)
    assert (r["samples"] == 1).all()
    np.testing.assert_array_equal(r["rgba"].reshape(-1, 4),
                                  np.broadcast_to([0.3, 0.6, 0.9, 1.0], (16, 4)))


# ------------------------------------------------------------ P7 channels

def test_p7_channel_permutation_invariance():
    nx, ny, nz = 18, 15, 12
    vol = scenes.random_volume(7, (4, nz, ny, nx), np.uint16, 4096)
    tfs = [TF(0.1, 0.8, 0.3, 0.7, (1, 0, 0)), TF(0.2, 0.9, -0.5, 1.5, (0, 1, 0)),
           TF(0.05, 0.6, 0.0, 0.3, (0, 0, 1)), TF(0.3, 0.7, 1.0, 2.0, (1, 1, 0))]
    cam = scenes.mirror_camera(nx, ny, nz, 2.0)
    sc = Scene("p7", vol, 12, tfs, cam, 16, 12, True, 0.9, 0.95)
    base = orc.render(sc, 1)["rgba"]
    perm = [2, 0, 3, 1]
    got = orc.render(sc, 1, data=np.ascontiguousarray(vol[perm]),
                     tfs=[tfs[p] for p in perm])["rgba"]
    np.testing.assert_allclose(got, base, rtol=0, atol=1e-12)


# ------------------------------------------------------------ P8 bound

def test_p8_termination_changes_result_by_at_most_one_minus_tau():
    nx, ny, nz = 24, 20, 16
    vol = scenes.random_volume(8, (2, nz, ny, nx), np.uint8)
    tfs = [TF(0.1, 0.7, 0.0, 0.8, (0.5, 1, 0.2)), TF(0.2, 0.9, 0.5, 1.2, (1, 0.3, 0.6))]
    sc = Scene("p8", vol, 8, tfs, scenes.mirror_camera(nx, ny, nz, 2.0), 20, 16, True,
               0.6, 0.99)
    a = orc.render(sc, -1)
    b = orc.render(sc, -1, term_alpha=1.0)
    d = np.abs(a["rgba"] - b["rgba"]).max()
    assert 0.0 < d <= 0.01 + 1e-12
    assert (a["samples"] <= b["samples"]).all() and (a["samples"] < b["samples"]).any()


# ------------------------------------------------------------ P9 rotation

def test_p9_rotation_about_z_is_invariant():
    n, nz = 16, 10
    rng = np.random.default_rng(9)
    V = rng.integers(0, 256, size=(1, nz, n, n)).astype(np.uint8)
    # V'(i, j, k) = V(j, n - 1 - i, k); arrays are indexed [k][j][i]
    Vp = np.empty_like(V)
    for j in range(n):
        for i in range(n):
            Vp[0, :, j, i] = V[0, :, n - 1 - i, j]
    cam = Cam("perspective", (3.0, -30.0, 25.0), (0.3, 1.0, -0.6), (0.0, 0.0, 1.0),
              math.radians(35), 1.0, 2.5, 40.0)

    def inv(p):  # Q^-1 (a, b) = (n - 1 - b, a)
        return (n - 1 - p[1], p[0], p[2])

    def inv_lin(v):  # linear part (a, b) -> (-b, a)
        return (-v[1], v[0], v[2])

    camp = Cam("perspective", inv(cam.center), inv_lin(cam.forward), inv_lin(cam.up),
               cam.fov_y, 1.0, cam.eye_separation, cam.convergence)
    tf = [TF(0.1, 0.9, 0.2, 1.0, (0.4, 0.7, 1.0))]
    sc = Scene("p9", V, 8, tf, cam, 32, 24, True, 0.5, 0.99)
    scp = Scene("p9r", Vp, 8, tf, camp, 32, 24, True, 0.5, 0.99)
    for eye in (-1, 1):
        a = orc.render(sc, eye)
        b = orc.render(scp, eye)
        assert a["rgba"][..., 3].max() > 0.3
        np.testing.assert_allclose(a["rgba"], b["rgba"], rtol=0, atol=1e-12)


# ------------------------------------------------------------ P10 brute force

def test_p10_two_cube_brute_force():
    V = np.array([[[10, 20], [30, 40]], [[50, 60], [70, 80]]], np.uint8)[None]  # [k][j][i]
    tf = TF(0.0, 1.0, 0.0, 1.0, (1.0, 1.0, 1.0))
    cam = Cam("ortho", (0.5, 0.5, -3.0), (0, 0, 1), (0, -1, 0), ortho_height=2.0)
    sc = Scene("p10", V, 8, [tf], cam, 1, 1, False, 1.0, 1.0)
    r = orc.render(sc)
    # ray x = y = 0.5 crosses z from -1 to 2; samples at z = -0.5, 0.5, 1.5
    plane0 = (10 + 20 + 30 + 40) / 4.0
    plane1 = (50 + 60 + 70 + 80) / 4.0
    vals = [0.5 * plane0, 0.5 * (plane0 + plane1), 0.5 * plane1]
    C = A = 0.0
    for x in vals:
        a = x / 255.0
        C += (1 - A) * a * a
        A += (1 - A) * a
    assert r["samples"][0, 0] == 3
    np.testing.assert_allclose(r["rgba"][0, 0], [C, C, C, A], rtol=0, atol=1e-15)


# ------------------------------------------------------- P11 orientation

def test_p11_axis_aligned_projection_closed_form():
    nx, ny, nz = 12, 9, 7
    rng = np.random.default_rng(11)
    col = rng.integers(0, 256, size=(ny, nx))
    V = np.broadcast_to(col, (nz, ny, nx)).astype(np.uint8)[None].copy()
    cam = Cam("ortho", ((nx - 1) / 2, (ny - 1) / 2, -4.0), (0, 0, 1), (0, -1, 0),
              ortho_height=float(ny))
    sc = Scene("p11", V, 8, [TF()], cam, nx, ny, False, 1.0, 1.0)
    r = orc.render(sc)
    f = col / 255.0
    h = f / 2.0
    q = (1 - f) ** (nz - 1)
    A = 1 - (1 - h) ** 2 * q
    C = h * h + (1 - h) * (1 - q) * f + (1 - h) * q * h * h  # geometric series
    exp = np.stack([C, C, C, A], -1)
    np.testing.assert_allclose(r["rgba"], exp, rtol=0, atol=1e-12)
    # sample count: extended box length nz + 1 at step 1, half-step phase; a
    # column of 255 is opaque (alpha 1) and stops at its first full sample
    assert (r["nominal"] == nz + 1).all()
    assert (r["samples"][col < 255] == nz + 1).all()
    assert (r["samples"][col == 255] == 2).all() and (col == 255).any()


def test_p11_sample_count_closed_form_tiny_workload():
    from paper_1407_2089_amd.synth import tiny_scene
    sc = tiny_scene()
    r = orc.render(sc)
    n = math.ceil((32 + 1) / 0.5 - 0.5)
    assert n == 66 and (r["nominal"] == n).all() and (r["samples"] == n).all()


# ------------------------------------------------------- P12 projection

def test_p12_perspective_stereo_projects_points_correctly():
    n = 40
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = np.array([26.0, 14.0, 22.0])
    V = 250.0 * np.exp(-((i - X[0]) ** 2 + (j - X[1]) ** 2 + (k - X[2]) ** 2) / (2 * 1.2 ** 2))
    V = np.rint(V).astype(np.uint8)[None]
    centre = np.array([19.5, 19.5, 19.5])
    eye_pos = centre + np.array([-10.0, -95.0, 30.0])
    fwd = centre - eye_pos
    dist = float(np.linalg.norm(fwd))
    fwd /= dist
    W, H, sep, conv, fov = 160, 120, 8.0, dist * 0.8, math.radians(30)
    cam = Cam("perspective", tuple(eye_pos), tuple(fwd), (0, 0, 1), fov, 1.0, sep, conv)
    sc = Scene("p12", V, 8, [TF(0.05, 0.6)], cam, W, H, True, 0.25, 1.0)
    f = fwd
    r = np.cross(f, [0, 0, 1]); r /= np.linalg.norm(r)
    u = np.cross(r, f)
    d = X - eye_pos
    xr, yu, zf = d @ r, d @ u, d @ f
    h = conv * math.tan(fov / 2); w = h * W / H
    for eye in (-1, 1):
        img = orc.render(sc, eye)["rgba"][..., 3]
        jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ci = (img * ii).sum() / img.sum()
        cj = (img * jj).sum() / img.sum()
        s_off = eye * sep / 2
        sx = (s_off + (xr - s_off) * conv / zf) / w
        sy = (yu * conv / zf) / h
        ei = (sx + 1) * W / 2 - 0.5
        ej = (1 - sy) * H / 2 - 0.5
        assert abs(ci - ei) < 0.3 and abs(cj - ej) < 0.3, (eye, ci, ei, cj, ej)


# ------------------------------------------------------- P13 world scale

def test_p13_uniform_world_scale_invariance():
    # Scaling voxel spacing, origin, camera and step by one factor s leaves the
    # image unchanged (pins the spacing and origin handling).
    nx, ny, nz = 20, 16, 12
    V = scenes.random_volume(13, (2, nz, ny, nx), np.uint8)
    tfs = [TF(0.1, 0.9, 0.3, 0.8, (0.9, 0.2, 0.4)), TF(0.2, 0.7, -0.2, 1.1, (0.1, 0.8, 0.5))]
    base_cam = scenes.mirror_camera(nx, ny, nz, sep=2.0)
    o = (1.5, -2.0, 0.5)
    a = orc.render(Scene("s1", V, 8, tfs, base_cam, 24, 18, True, 0.7, 0.97, origin=o), -1)
    s = 2.5
    # the map X -> s X sends voxel positions o + i to s o + i s and the camera
    # to s c; directions, fov and the order of samples are unchanged
    cam = Cam("perspective", tuple(s * np.array(base_cam.center)), base_cam.forward,
              base_cam.up, base_cam.fov_y, 1.0, s * base_cam.eye_separation,
              s * base_cam.convergence)
    b = orc.render(Scene("s2", V, 8, tfs, cam, 24, 18, True, 0.7 * s, 0.97,
                         spacing=(s, s, s), origin=tuple(s * np.array(o))), -1)
    assert a["rgba"][..., 3].max() > 0.2
    np.testing.assert_allclose(a["rgba"], b["rgba"], rtol=0, atol=1e-11)
    assert np.array_equal(a["samples"], b["samples"])


def test_p13_anisotropic_sample_count_closed_form():
    # Ortho ray along z with z spacing 2.5 and step 1: the extended box spans
    # (nz + 1) * 2.5 world units, so ceil((nz + 1) * 2.5 - 1/2) samples.
    nz = 9
    V = np.full((1, nz, 6, 6), 10, np.uint8)
    cam = Cam("ortho", (2.5, 2.5, -3.0), (0, 0, 1), (0, -1, 0), ortho_height=2.0)
    r = orc.render(Scene("az", V, 8, [TF(0.5, 1.0)], cam, 3, 3, False, 1.0, 1.0,
                         spacing=(1.0, 1.0, 2.5)))
    assert (r["nominal"] == math.ceil((nz + 1) * 2.5 - 0.5)).all()


# ------------------------------------------------------------- P14 lighting

def test_p14_gradient_of_a_linear_field_closed_form():
    # Central differences reproduce a linear field's slope exactly, per axis
    # divided by that axis's spacing (pins axis order, spacing and sign).
    nx, ny, nz = 12, 9, 7
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coef = [(20, 3, 7, 10), (1, 30, 2, 50)]
    V = np.stack([a * i + b * j + c * k + d for a, b, c, d in coef]).astype(np.uint16)
    sp = (2.0, 1.0, 0.5)
    vol = oracle.Volume(V, 12, spacing=sp, origin=(4.0, -1.0, 2.0))
    rng = np.random.default_rng(3)
    pts = rng.uniform((1, 1, 1), (nx - 2, ny - 2, nz - 2), size=(50, 3))
    g = oracle.gradient(vol, pts)
    for c, (a, b, cc, _) in enumerate(coef):
        np.testing.assert_allclose(g[:, c], np.broadcast_to([a / sp[0], b / sp[1], cc / sp[2]],
                                                            (50, 3)), rtol=1e-12, atol=1e-12)


def test_p14_gradient_of_a_quadratic_field_closed_form():
    # For v = i^2 the trilinear field between voxels is the chord of i^2, and
    # its central difference over one voxel is exactly 2 p at any interior p
    # (a one-sided or half-voxel difference, or the nearest voxel's gradient,
    # gives 2 p +- 1 or 2 round(p) instead).
    nx = 40
    V = np.zeros((1, 4, 4, nx), np.uint16)
    V[0] = (np.arange(nx) ** 2)[None, None, :]
    vol = oracle.Volume(V, 16)
    xs = np.linspace(1.0, nx - 2.0, 97)
    pts = np.stack([xs, np.full_like(xs, 1.5), np.full_like(xs, 1.25)], axis=1)
    g = oracle.gradient(vol, pts)
    np.testing.assert_allclose(g[:, 0, 0], 2.0 * xs, rtol=1e-12)
    assert np.all(g[:, 0, 1:] == 0.0)


def test_p14_shade_special_cases():
    # Linear field with gradient g: the normal is -g / |g|.  A light along the
    # normal gives ambient + diffuse, against it or across it the ambient
    # only, at 45 degrees ambient + diffuse / sqrt 2; a flat field has no
    # surface and gives ambient + diffuse.  Light vectors are not unit length.
    nx, ny, nz = 8, 8, 8
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    V = (30 * i + 10 * j + 5 * k + 20).astype(np.uint16)[None]
    vol = oracle.Volume(V, 12)
    g = np.array([30.0, 10.0, 5.0])
    n = -g / np.linalg.norm(g)
    m = np.cross(n, [0.0, 0.0, 1.0])
    m /= np.linalg.norm(m)
    ka, kd = 0.2, 0.7
    p = (3.4, 4.1, 3.7)
    cases = [(3 * n, ka + kd), (-2 * n, ka), (5 * m, ka), (n + m, ka + kd / math.sqrt(2))]
    for l, expect in cases:
        s, marg = oracle.shade(vol, oracle.Light(tuple(l), ka, kd), p)
        assert abs(s[0] - expect) < 1e-12, (l, s, expect)
        assert 0.0 < marg[0] < 1e-4
    flat = oracle.Volume(np.full((1, 6, 6, 6), 900, np.uint16), 12)
    s, marg = oracle.shade(flat, oracle.Light((1.0, 2.0, 3.0), ka, kd), (2.5, 2.5, 2.5))
    assert s[0] == ka + kd and marg[0] == 0.0


def test_p14_lit_thin_slab_closed_form():
    # One voxel layer v = 20 i + 10 (uint8), spacing (2, 1, 0.5), seen along
    # +z by an orthographic camera whose rays cross interior columns.  Each
    # ray takes two samples, at z = -1/2 and +1/2 (index space), both with
    # value V / 2 (V = 20 x + 10): raw gradients (5, 0, V / 2) and
    # (5, 0, -V / 2) per world unit.  With the light l = (0.2, 0, -1) the
    # first sample faces the light and the second faces away (ambient only).
    nx, ny = 8, 5
    V = np.zeros((1, 1, ny, nx), np.uint8)
    V[0, 0] = (20 * np.arange(nx) + 10)[None, :]
    m, rgb = 0.9, (1.0, 0.5, 0.25)
    ka, kd = 0.25, 0.6
    ldir = np.array([0.2, 0.0, -1.0])
    cam = Cam("ortho", (7.0, 2.0, -3.0), (0, 0, 1), (0, -1, 0), ortho_height=1.0)
    sc = Scene("lit slab", V, 8, [TF(0.0, 1.0, 0.0, m, rgb)], cam, 6, 2, False, 0.5, 1.0,
               spacing=(2.0, 1.0, 0.5))
    sc.light = Light(tuple(ldir), ka, kd)
    r = orc.render(sc)
    assert (r["samples"] == 2).all()
    lhat = ldir / np.linalg.norm(ldir)
    for jj in range(2):
        for ii in range(6):
            x_world = 7.0 + (2 * (ii + 0.5) / 6 - 1) * 1.5
            Vx = 20 * (x_world / 2.0) + 10
            u = 0.5 * Vx / 255.0
            a = m * u
            shades = []
            for gz in (0.5 * Vx, -0.5 * Vx):
                gv = np.array([5.0, 0.0, gz])
                shades.append(ka + kd * max(0.0, float(-gv @ lhat) / np.linalg.norm(gv)))
            assert shades[0] > ka and shades[1] == ka
            col = a * u * shades[0] + (1 - a) * a * u * shades[1]
            exp = [col * rgb[0], col * rgb[1], col * rgb[2], a + (1 - a) * a]
            np.testing.assert_allclose(r["rgba"][jj, ii], exp, rtol=0, atol=1e-12)
    assert r["lit_margin"].max() < 1e-5


def test_p14_lighting_scales_colour_only():
    # Lighting never changes opacity or sample counts; ambient 1 with no
    # diffuse term is the unlit image, and a pure ambient term k scales the
    # colour by k (colour sums kept below the cap, black background).
    nx, ny, nz = 18, 14, 10
    V = scenes.random_volume(17, (2, nz, ny, nx), np.uint16, 4096)
    tfs = [TF(0.1, 0.8, 0.2, 1.2, (0.5, 0.0, 0.2)), TF(0.2, 0.9, -0.3, 0.7, (0.0, 0.5, 0.3))]
    cam = scenes.mirror_camera(nx, ny, nz, sep=1.5)
    sc = Scene("lit", V, 12, tfs, cam, 20, 16, True, 0.8, 0.97, spacing=(1.0, 1.5, 0.8))
    for eye in (-1, 1):
        base = orc.render(sc, eye, lit=False)
        sc.light = Light((0.3, -0.5, 0.8), 0.35, 0.65)
        lit = orc.render(sc, eye)
        assert np.array_equal(lit["rgba"][..., 3], base["rgba"][..., 3])
        assert np.array_equal(lit["samples"], base["samples"])
        assert not np.allclose(lit["rgba"][..., :3], base["rgba"][..., :3], atol=1e-3)
        sc.light = Light((0.3, -0.5, 0.8), 1.0, 0.0)
        same = orc.render(sc, eye)
        assert np.array_equal(same["rgba"], base["rgba"])
        sc.light = Light((0.3, -0.5, 0.8), 0.4, 0.0)
        half = orc.render(sc, eye)
        np.testing.assert_allclose(half["rgba"][..., :3], 0.4 * base["rgba"][..., :3],
                                   rtol=0, atol=1e-12)
        assert np.array_equal(half["lit_margin"], np.zeros_like(half["lit_margin"]))
        sc.light = None
