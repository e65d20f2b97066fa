"""Pins of the ray-marching oracle (CPU).

Each pin checks the oracle against something other than itself: the number of
samples a ray spends in one voxel (counted by hand), the closed form of
compositing identical samples, an independent back-to-front formulation of the
"over" operator, exact table-entry boundaries, and symmetries of the view.
"""

import math

import numpy as np
import pytest

from oracle.render import F, render, transfer_index, trilinear
from workloads.camera import axis_view, orbit_view, ramp_lut


def _view(origin, d, right=(0, 0, 0), up=(0, 0, 0), width=1, height=1, steps=16):
    return {"origin": list(origin), "right": list(right), "up": list(up), "dir": list(d),
            "width": width, "height": height, "steps": steps}


def _lut(r=0.25, g=0.5, b=1.0, a=0.125):
    lut = np.zeros((256, 4), dtype=np.float32)
    lut[:] = (r, g, b, a)
    return lut


def test_empty_volume_is_transparent():
    img = render(np.zeros((0, 3)), np.zeros(0), _view((0, 0, 0), (F, 0, 0)), _lut())
    assert img.shape == (1, 1, 4) and np.all(img == 0)


def test_one_voxel_seen_by_four_samples():
    """Samples every quarter spacing from x = -2 along +x: the nearest-voxel rule
    puts x in [-1/2, 1/2) on the voxel at 0, i.e. samples k = 6, 7, 8, 9."""
    view = _view((-2 * F, 0, 0), (F // 4, 0, 0), steps=16)
    a = 0.125
    img = render(np.array([[0, 0, 0]]), np.array([0.5]), view, _lut(a=a))
    A = 1 - (1 - a) ** 4
    np.testing.assert_allclose(img[0, 0], [0.25 * A, 0.5 * A, 1.0 * A, A], rtol=1e-14)
    # steps of 3/8: the voxel covers [-1/2, 1/2), half-open
    step = 3 * F // 8
    cases = [(-2 * F, 3),            # offsets 1.5, 1.875, 2.25 past the start
             (-2 * F - F // 8, 2),   # the third sample lands exactly on +1/2: next voxel
             (-5 * F // 4, 3)]       # the first lands exactly on -1/2: this voxel
    for start, count in cases:
        img = render(np.array([[0, 0, 0]]), np.array([0.5]), _view((start, 0, 0), (step, 0, 0)),
                     _lut(a=a))
        assert img[0, 0, 3] == pytest.approx(1 - (1 - a) ** count, rel=1e-14), (start, count)


def test_front_to_back_equals_back_to_front():
    """A ray through a column of voxels with random values and a random table:
    front-to-back accumulation equals the back-to-front 'over' recursion."""
    rng = np.random.default_rng(3)
    n = 12
    coords = np.stack([np.arange(n), np.zeros(n, int), np.zeros(n, int)], axis=1)
    vals = rng.uniform(0, 1, n).astype(np.float32)
    lut = rng.uniform(0, 1, (256, 4)).astype(np.float32)
    lut[:, 3] *= 0.3
    view = _view((-F // 2, 0, 0), (F, 0, 0), steps=n)  # one sample per voxel
    img = render(coords, vals, view, lut)
    e = transfer_index(vals, 1.0, 0.0)
    C = np.zeros(3)
    A = 0.0
    for k in reversed(range(n)):
        c, a = lut[e[k], :3].astype(np.float64), float(lut[e[k], 3])
        C = a * c + (1 - a) * C
        A = a + (1 - a) * A
    np.testing.assert_allclose(img[0, 0], np.r_[C, A], rtol=1e-12, atol=1e-15)


def test_transfer_entries_at_exact_boundaries():
    v = np.array([0.0, 1 / 256, 2 / 256 - 2 ** -20, 0.5, 255 / 256, 1.0, 7.0, -0.1, np.nan,
                  np.inf, -np.inf], dtype=np.float32)
    assert list(transfer_index(v, 1.0, 0.0)) == [0, 1, 1, 128, 255, 255, 255, 0, 0, 255, 0]
    # scale and offset: t = (v - offset) * scale
    assert list(transfer_index(np.float32([3.0, 3.5, 4.0]), 0.5, 3.0)) == [0, 64, 128]


def test_uniform_slab_gives_uniform_image():
    """Every ray of an axis view crosses a full slab the same number of times."""
    g = np.mgrid[0:6, 0:5, 0:4].reshape(3, -1).T
    vals = np.full(len(g), 0.7, dtype=np.float32)
    view = axis_view((0, 0, 0), (5, 4, 3), axis=0, step=0.5)
    img = render(g, vals, view, _lut(a=0.05))
    assert img.shape == (4, 5, 4)
    a = float(np.float32(0.05))  # the table holds FP32
    A = 1 - (1 - a) ** 12  # 6 voxels x 2 samples each
    np.testing.assert_allclose(img[..., 3], A, rtol=1e-14)


def test_rotated_views_of_a_sphere_agree():
    """A voxelised ball seen along +x and along +y (views that are exact axis
    permutations of each other) gives the same image."""
    r = 6
    g = np.mgrid[-r:r + 1, -r:r + 1, -r:r + 1].reshape(3, -1).T
    ball = g[np.sum(g * g, axis=1) <= r * r]
    vals = (np.sqrt(np.sum(ball * ball, axis=1)) / r).astype(np.float32)
    lut = ramp_lut(0.2)
    vx = orbit_view((0, 0, 0), 10, 180, 0, 17, 17, pixel=1.0, step=0.5)
    vy = orbit_view((0, 0, 0), 10, 270, 0, 17, 17, pixel=1.0, step=0.5)
    ix = render(ball, vals, vx, lut)
    iy = render(ball, vals, vy, lut)
    assert ix[..., 3].max() > 0.5
    np.testing.assert_array_equal(ix, iy)
    # and the image of a ball is symmetric under flips of both image axes
    np.testing.assert_allclose(ix, ix[::-1, ::-1], rtol=0, atol=1e-15)


def test_orbit_view_geometry():
    v = orbit_view((10, 20, 30), 50, 0, 0, 3, 2, pixel=2.0, step=0.25, steps=None)
    assert v["dir"] == [-F // 4, 0, 0]  # looking from +x towards the centre
    assert v["steps"] == 400
    assert v["right"][0] == 0 and v["up"] == [0, 0, 2 * F]
    # centre of the image plane lies `distance` before the centre
    o = np.array(v["origin"]) + (np.array(v["right"]) * 1 + np.array(v["up"]) * 0.5)
    np.testing.assert_allclose(o / F, [60, 20, 30], atol=1e-6)
    assert math.isclose(np.linalg.norm(v["right"]) / F, 2.0, rel_tol=1e-6)


# -- trilinear sampling -------------------------------------------------------------

def test_trilinear_at_voxel_centres_is_nearest():
    """Samples exactly at voxel centres weigh one corner only: the image is the
    nearest-voxel image, bit for bit."""
    r = 5
    g = np.mgrid[-r:r + 1, -r:r + 1, -r:r + 1].reshape(3, -1).T
    ball = g[np.sum(g * g, axis=1) <= r * r]
    vals = np.random.default_rng(4).uniform(0, 1, len(ball)).astype(np.float32)
    lut = np.random.default_rng(5).uniform(0, 1, (256, 4)).astype(np.float32)
    lut[:, 3] *= 0.2
    view = _view((-8 * F, -6 * F, -6 * F), (F, 0, 0), right=(0, F, 0), up=(0, 0, F), width=13,
                 height=13, steps=17)
    a = render(ball, vals, view, lut)
    b = render(ball, vals, dict(view, filter="trilinear"), lut)
    assert a[..., 3].max() > 0.5
    np.testing.assert_array_equal(a, b)


def test_trilinear_constant_field_is_exact():
    """The eight weights are integers summing to 2^24, so a field that is the
    same at all corners comes back exactly, at any fraction."""
    rng = np.random.default_rng(6)
    v = rng.uniform(-3, 3, 500).astype(np.float32)
    sites = np.tile(np.arange(8), (500, 1))
    frac = rng.integers(0, 256, (500, 3))
    for k in range(500):
        val, hit = trilinear(np.full(8, v[k], dtype=np.float32), sites[k:k + 1], frac[k:k + 1])
        assert hit[0] and val[0] == v[k]


def test_trilinear_matches_scipy_map_coordinates():
    """An independent trilinear interpolation (scipy.ndimage, order 1) of the
    dense array with zeros at empty voxels, at the 8-bit quantised positions."""
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(7)
    dense = rng.uniform(0.1, 1.0, (6, 6, 6)).astype(np.float32)
    dense[rng.uniform(size=dense.shape) < 0.3] = 0.0  # empty voxels
    coords = np.argwhere(dense != 0)
    values = dense[tuple(coords.T)]
    idx = -np.ones(dense.shape, dtype=np.int64)
    idx[tuple(coords.T)] = np.arange(len(coords))
    base = rng.integers(0, 5, (400, 3))
    frac = rng.integers(0, 256, (400, 3))
    sites = np.stack([idx[base[:, 0] + (c & 1), base[:, 1] + ((c >> 1) & 1), base[:, 2] + (c >> 2)]
                      for c in range(8)], axis=1)
    val, hit = trilinear(values, sites, frac)
    ref = map_coordinates(dense.astype(np.float64), (base + frac / 256.0).T, order=1)
    np.testing.assert_allclose(val, ref, rtol=1e-6, atol=1e-7)
    # a hit needs a site among the corners of non-zero weight
    w = np.stack([np.prod([np.where((c >> a) & 1, frac[:, a], 256 - frac[:, a]) for a in range(3)],
                          axis=0) for c in range(8)], axis=1)
    assert np.array_equal(hit, np.any((w > 0) & (sites >= 0), axis=1))


def test_trilinear_ramp_between_two_voxels():
    """Between voxels 0 and 1 on the x axis the value is v0 + (v1 - v0) a / 256,
    and half way to an empty voxel it is half the value."""
    v0, v1 = np.float32(0.25), np.float32(0.875)
    a = np.arange(256)
    frac = np.stack([a, np.zeros_like(a), np.zeros_like(a)], axis=1)
    sites = np.full((256, 8), -1)
    sites[:, 0], sites[:, 1] = 0, 1
    val, hit = trilinear(np.array([v0, v1]), sites, frac)
    exact = (float(v0) * (256 - a) + float(v1) * a) / 256.0
    assert hit.all() and np.array_equal(val, exact.astype(np.float32))
    sites[:, 1] = -1
    val, _ = trilinear(np.array([v0, v1]), sites, frac)
    assert val[128] == v0 / 2


def test_trilinear_samples_seeing_one_voxel():
    """Steps of 1/8 from x = -2 past one voxel at 0: with trilinear filtering the
    voxel carries weight for base voxel -1 at non-zero fractions (k = 9..15) and
    for base voxel 0 (k = 16..23): 15 samples, against 8 for the nearest voxel.
    With a table of constant opacity alpha the image is 1 - (1 - alpha)^15."""
    a = 0.125
    view = _view((-2 * F, 0, 0), (F // 8, 0, 0), steps=40)
    near = render(np.array([[0, 0, 0]]), np.array([0.5]), view, _lut(a=a))
    tri = render(np.array([[0, 0, 0]]), np.array([0.5]), dict(view, filter="trilinear"), _lut(a=a))
    assert near[0, 0, 3] == pytest.approx(1 - (1 - a) ** 8, rel=1e-14)
    assert tri[0, 0, 3] == pytest.approx(1 - (1 - a) ** 15, rel=1e-14)


# -- per-ray directions (pinhole views) ---------------------------------------------

def test_per_ray_directions_by_hand():
    """Three rays from one eye at x = -4, directions (1/2, -1/8 + i/8, 0) for
    pixel i, through a column of voxels (0, y, 0), y = -2..2, with distinct
    values and an opaque table: each pixel shows the first voxel its ray meets,
    which is (0, i - 1, 0) (sample k = 7 lands at x = -1/2, y = -7/8 + 7 i / 8)."""
    col = np.array([[0, y, 0] for y in range(-2, 3)])
    vals = np.array([0.0, 0.25, 0.5, 0.75, 0.99], dtype=np.float32)  # entries 0, 64, 128, 192, 253
    lut = np.zeros((256, 4), dtype=np.float32)
    lut[:, 0] = np.arange(256)
    lut[:, 3] = 1.0
    view = {"origin": [-4 * F, 0, 0], "right": [0, 0, 0], "up": [0, 0, 0],
            "dir": [F // 2, -F // 8, 0], "dir_right": [0, F // 8, 0], "dir_up": [0, 0, 0],
            "width": 3, "height": 1, "steps": 20}
    img = render(col, vals, view, lut)
    assert list(img[0, :, 0]) == [64.0, 128.0, 192.0]
    assert np.all(img[0, :, 3] == 1.0)


def test_zero_direction_spread_is_the_orthographic_view():
    r = 4
    g = np.mgrid[-r:r + 1, -r:r + 1, -r:r + 1].reshape(3, -1).T
    ball = g[np.sum(g * g, axis=1) <= r * r]
    vals = np.random.default_rng(8).uniform(0, 1, len(ball)).astype(np.float32)
    v = orbit_view((0, 0, 0), 10, 30, 20, 9, 7, pixel=1.1, step=0.4)
    a = render(ball, vals, v, ramp_lut(0.2))
    b = render(ball, vals, dict(v, dir_right=[0, 0, 0], dir_up=[0, 0, 0]), ramp_lut(0.2))
    np.testing.assert_array_equal(a, b)


def test_perspective_view_geometry():
    from workloads.camera import perspective_view
    v = perspective_view((10, 20, 30), 50, 0, 0, 5, 5, fov=40, step=0.5)
    assert v["right"] == [0, 0, 0] and v["up"] == [0, 0, 0]
    np.testing.assert_allclose(np.array(v["origin"]) / F, [60, 20, 30], atol=1e-6)
    centre = np.array(v["dir"]) + 2 * np.array(v["dir_right"]) + 2 * np.array(v["dir_up"])
    np.testing.assert_allclose(centre / F, [-0.5, 0, 0], atol=1e-5)  # the central ray
    # the edge rays open at the field of view
    top = np.array(v["dir"]) + 2 * np.array(v["dir_right"]) + 5 * np.array(v["dir_up"]) - np.array(v["dir_up"]) / 2
    assert math.degrees(math.atan2(top[2], -top[0])) == pytest.approx(20.0, abs=0.01)
