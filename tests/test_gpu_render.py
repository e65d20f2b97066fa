"""GPU ray marcher (HIP kernel through the C ABI) against the oracle's.

The oracle (oracle/render.py) is pinned in tests/test_oracle_render.py.  Sample
positions are fixed-point integers and the table entry is an FP32 decision taken
the same way on both sides, so the set of samples each ray composites is the
same; only the FP32 compositing differs from the oracle's FP64.  Per sample the
GPU rounds three times (the weight (1 - A) a, then C and A), so after K samples
every channel is within 4 K 2^-24 of the oracle's value.  Pixels whose ray meets
no site are exactly zero on both sides; that also checks that skipping empty
blocks never skips a sample that contributes.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from workloads.camera import FIX, axis_view, orbit_view, ramp_lut  # noqa: E402
from oracle.render import render as oracle_render, render_rays  # noqa: E402
from paper_1906_11925_amd import LB, HemelbError  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tol(view):
    return 4.0 * max(1, view["steps"]) * 2.0 ** -24


def _check(img, ref, view):
    img = img.cpu().numpy().astype(np.float64)
    assert img.shape == ref.shape
    assert np.array_equal(img[..., 3] == 0, ref[..., 3] == 0)
    assert np.abs(img - ref).max() <= _tol(view)


def _tree_small():
    return wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1)


def _centre(g):
    c = g.coords
    return (c.min(axis=0) + c.max(axis=0)) / 2.0, float(np.linalg.norm(c.max(axis=0) - c.min(axis=0)))


@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "tree_small"])
@pytest.mark.parametrize("angles", [(0, 0), (30, 20), (200, -35), (90, 89)])
def test_random_values_match_oracle(name, angles):
    _gpu()
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "tree_small": _tree_small}[name]()
    vals = np.random.default_rng(7).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    centre, size = _centre(g)
    pixel = size / 40.0
    view = orbit_view(centre, size, angles[0], angles[1], 48, 40, pixel=pixel, step=0.5)
    lut = ramp_lut(0.08)
    lb = LB.from_geometry(g)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut, scale=1.0, offset=0.0)
    ref = oracle_render(g.coords, vals, view, lut)
    assert ref[..., 3].max() > 0.05
    _check(img, ref, view)


def test_speed_of_a_simulated_flow():
    """The field a user renders: |u| after 300 steps of the pipe, with a transfer
    scale and offset."""
    _gpu()
    g = wl.pipe()
    lb = LB.from_geometry(g)
    lb.step(300)
    _, u, _ = lb.observables()
    speed = torch.linalg.vector_norm(u, dim=1).contiguous()
    s = speed.cpu().numpy()
    scale, offset = float(1.0 / s.max()), float(s.min())
    view = orbit_view((9.5, 9.5, 31.5), 60, 60, 30, 64, 64, pixel=1.1, step=0.25)
    lut = ramp_lut(0.1)
    img = lb.render(speed, view, lut, scale=scale, offset=offset)
    ref = oracle_render(g.coords, s, view, lut, scale=scale, offset=offset)
    _check(img, ref, view)


def test_transfer_entry_boundaries():
    """Values on exact table-entry boundaries, and beyond both ends."""
    _gpu()
    g = wl.closed_box(8, 1, 1)
    vals = np.array([0.0, 1 / 256, 0.5, 255 / 256, 1.0, 3.0, -1.0, 2 / 256 - 2 ** -20],
                    dtype=np.float32)
    lut = np.zeros((256, 4), dtype=np.float32)
    lut[:, 0] = np.arange(256) / 255.0
    lut[:, 3] = 1.0  # opaque: each ray shows exactly its first sample's entry
    view = {"origin": [0, 0, -2 * FIX], "right": [FIX, 0, 0], "up": [0, 0, 0],
            "dir": [0, 0, FIX], "width": 8, "height": 1, "steps": 4}
    lb = LB.from_geometry(g)
    order = np.lexsort((g.coords[:, 2], g.coords[:, 1], g.coords[:, 0]))
    v = np.empty(g.n_sites, dtype=np.float32)
    v[order] = vals
    img = lb.render(torch.from_numpy(v).cuda(), view, lut).cpu().numpy()
    ref = oracle_render(g.coords, v, view, lut)
    np.testing.assert_array_equal(img[0, :, 0], ref[0, :, 0].astype(np.float32))
    assert list(np.rint(img[0, :, 0] * 255).astype(int)) == [0, 1, 128, 255, 255, 255, 0, 1]


def test_edge_views():
    _gpu()
    g = wl.aneurysm(half=True)
    vals = np.random.default_rng(3).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    t = torch.from_numpy(vals).cuda()
    lut = ramp_lut(0.2)
    lb = LB.from_geometry(g)
    views = [
        # pointing away from the volume
        {"origin": [-50 * FIX, 0, 0], "right": [0, FIX, 0], "up": [0, 0, FIX],
         "dir": [-FIX, 0, 0], "width": 5, "height": 3, "steps": 100},
        # no samples
        dict(orbit_view((96, 80, 48), 150, 10, 10, 7, 5), steps=0),
        # a standing ray: every sample at one point inside the volume
        {"origin": [int(g.coords[100, 0]) * FIX, int(g.coords[100, 1]) * FIX,
                    int(g.coords[100, 2]) * FIX], "right": [FIX, 0, 0], "up": [0, FIX, 0],
         "dir": [0, 0, 0], "width": 3, "height": 2, "steps": 37},
        # one pixel; a ragged image wider than one workgroup of rays
        orbit_view((96, 80, 48), 150, 45, 45, 1, 1, pixel=2.0, step=0.7),
        orbit_view((96, 80, 48), 150, 300, -10, 37, 19, pixel=6.0, step=1.3),
        # the whole box straight along an axis
        axis_view(g.coords.min(axis=0), g.coords.max(axis=0), axis=1, pixel=3.0, step=0.5),
    ]
    for view in views:
        img = lb.render(t, view, lut, scale=1.5, offset=0.1)
        ref = oracle_render(g.coords, vals, view, lut, scale=1.5, offset=0.1)
        _check(img, ref, view)
    assert np.all(lb.render(t, views[0], lut).cpu().numpy() == 0)


def test_full_size_tree_sampled_rays():
    """The benchmark's view of the 5.6M-site tree, rendered whole on the GPU;
    the oracle recomputes 128 seeded pixels (32 of them among the lit ones)."""
    _gpu()
    g = wl.config_geometry("tree1024")
    vals = np.random.default_rng(11).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    lb = LB.from_geometry(g, storage="f16")
    view = orbit_view((512, 512, 512), 900, 35, 25, 512, 512, pixel=1024 / 512 * 1.4, step=1.0)
    lut = ramp_lut(0.05)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(5)
    pix = rng.integers(0, 512, (96, 2))
    lit = np.argwhere(img[..., 3] > 0)
    pix = np.concatenate([pix, lit[rng.choice(len(lit), 32, replace=False)][:, ::-1]])
    O, R, U = (np.asarray(view[k], dtype=np.int64) for k in ("origin", "right", "up"))
    origins = O[None, :] + pix[:, :1] * R[None, :] + pix[:, 1:] * U[None, :]
    ref = render_rays(g.coords, vals, origins, view["dir"], view["steps"], lut)
    got = img[pix[:, 1], pix[:, 0]]
    assert np.array_equal(got[:, 3] == 0, ref[:, 3] == 0)
    assert np.abs(got - ref).max() <= _tol(view)


def test_render_errors():
    _gpu()
    g = wl.pipe()
    t = torch.zeros(g.n_sites, dtype=torch.float32, device="cuda")
    lb = LB.from_geometry(g)
    lut = ramp_lut()
    for bad in (dict(width=0), dict(height=20000), dict(steps=-1)):
        view = dict(orbit_view((9, 9, 31), 40, 0, 0, 4, 4), **bad)
        with pytest.raises(HemelbError) as ei:
            lb.render(t, view, lut)
        assert ei.value.code == L.HEMELB_EINVAL
    with pytest.raises(HemelbError) as ei:
        lb.render(t, orbit_view((9, 9, 31), 40, 0, 0, 4, 4), lut, scale=float("nan"))
    assert ei.value.code == L.HEMELB_EINVAL
    from paper_1906_11925_amd import links
    _, nbr = links(g.labels, g.shape, g.periodic, 15)
    nocoords = LB(nbr, g.tau, iolets=list(g.iolets))
    with pytest.raises(HemelbError) as ei:
        nocoords.render(t, orbit_view((9, 9, 31), 40, 0, 0, 4, 4), lut)
    assert "coordinates" in str(ei.value)


# -- trilinear sampling ------------------------------------------------------------
# The filtered value is the same bits on both sides (integer weights, exact FP64
# products), so the sample set and every table entry match; only the FP32
# compositing differs, as for the nearest voxel.

@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "tree_small"])
@pytest.mark.parametrize("angles", [(0, 0), (30, 20), (200, -35), (90, 89)])
def test_trilinear_random_values_match_oracle(name, angles):
    _gpu()
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "tree_small": _tree_small}[name]()
    vals = np.random.default_rng(8).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    centre, size = _centre(g)
    view = dict(orbit_view(centre, size, angles[0], angles[1], 48, 40, pixel=size / 40.0,
                           step=0.37), filter="trilinear")
    lut = ramp_lut(0.08)
    lb = LB.from_geometry(g)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut, scale=1.3, offset=0.05)
    ref = oracle_render(g.coords, vals, view, lut, scale=1.3, offset=0.05)
    assert ref[..., 3].max() > 0.05
    _check(img, ref, view)
    # filtering differs from the nearest voxel off the voxel centres
    near = oracle_render(g.coords, vals, dict(view, filter="nearest"), lut, scale=1.3, offset=0.05)
    assert not np.array_equal(near, ref)


def test_trilinear_edge_views():
    _gpu()
    g = wl.aneurysm(half=True)
    vals = np.random.default_rng(9).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    t = torch.from_numpy(vals).cuda()
    lut = ramp_lut(0.2)
    lb = LB.from_geometry(g)
    lo, hi = g.coords.min(axis=0), g.coords.max(axis=0)
    low = g.coords[np.argmin(g.coords[:, 2])]  # a site of the lowest layer
    views = [
        # pointing away from the volume
        {"origin": [-50 * FIX, 0, 0], "right": [0, FIX, 0], "up": [0, 0, FIX],
         "dir": [-FIX, 0, 0], "width": 5, "height": 3, "steps": 100},
        # no samples
        dict(orbit_view((96, 80, 48), 150, 10, 10, 7, 5), steps=0),
        # a standing ray between voxel centres inside the volume
        {"origin": [int(g.coords[100, 0]) * FIX + FIX // 3, int(g.coords[100, 1]) * FIX + 5,
                    int(g.coords[100, 2]) * FIX + FIX // 2], "right": [FIX, 0, 0],
         "up": [0, FIX, 0], "dir": [0, 0, 0], "width": 3, "height": 2, "steps": 37},
        # rays 0.4 below the lowest layer of sites: base voxel one below the sites,
        # the corner above it carries weight 153/256
        {"origin": [(int(low[0]) - 20) * FIX, (int(low[1]) - 8) * FIX + FIX // 3,
                    (int(lo[2]) - 1) * FIX + 153 * 4096], "right": [0, FIX // 2, 0],
         "up": [0, 0, 0], "dir": [FIX // 4, 0, 0], "width": 32, "height": 1, "steps": 160},
        # one pixel; a ragged image wider than one workgroup of rays
        orbit_view((96, 80, 48), 150, 45, 45, 1, 1, pixel=2.0, step=0.7),
        orbit_view((96, 80, 48), 150, 300, -10, 37, 19, pixel=6.0, step=1.3),
        # the whole box straight along an axis, samples between voxel centres
        dict(axis_view(lo, hi, axis=1, pixel=3.0, step=0.45)),
    ]
    for k, view in enumerate(views):
        view = dict(view, filter="trilinear")
        img = lb.render(t, view, lut, scale=1.5, offset=0.1)
        ref = oracle_render(g.coords, vals, view, lut, scale=1.5, offset=0.1)
        if k == 3:
            assert ref[..., 3].max() > 0  # the low-face rays do see sites
        _check(img, ref, view)
    assert np.all(lb.render(t, dict(views[0], filter="trilinear"), lut).cpu().numpy() == 0)


def test_trilinear_full_size_tree_sampled_rays():
    """The 5.6M-site tree through the trilinear filter; the oracle recomputes
    128 seeded pixels (32 of them among the lit ones)."""
    _gpu()
    g = wl.config_geometry("tree1024")
    vals = np.random.default_rng(12).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    lb = LB.from_geometry(g, storage="f16")
    view = dict(orbit_view((512, 512, 512), 900, 35, 25, 512, 512, pixel=1024 / 512 * 1.4,
                           step=0.9), filter="trilinear")
    lut = ramp_lut(0.05)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(13)
    pix = rng.integers(0, 512, (96, 2))
    lit = np.argwhere(img[..., 3] > 0)
    pix = np.concatenate([pix, lit[rng.choice(len(lit), 32, replace=False)][:, ::-1]])
    O, R, U = (np.asarray(view[k], dtype=np.int64) for k in ("origin", "right", "up"))
    origins = O[None, :] + pix[:, :1] * R[None, :] + pix[:, 1:] * U[None, :]
    ref = render_rays(g.coords, vals, origins, view["dir"], view["steps"], lut,
                      filter="trilinear")
    got = img[pix[:, 1], pix[:, 0]]
    assert np.array_equal(got[:, 3] == 0, ref[:, 3] == 0)
    assert np.abs(got - ref).max() <= _tol(view)


def test_unknown_filter_is_rejected():
    _gpu()
    g = wl.pipe()
    lb = LB.from_geometry(g)
    t = torch.zeros(g.n_sites, dtype=torch.float32, device="cuda")
    with pytest.raises(HemelbError) as ei:
        lb.render(t, dict(orbit_view((9, 9, 31), 40, 0, 0, 4, 4), filter=2), ramp_lut())
    assert ei.value.code == L.HEMELB_EINVAL


# -- pinhole (perspective) views ------------------------------------------------------

@pytest.mark.parametrize("filt", ["nearest", "trilinear"])
@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "tree_small"])
@pytest.mark.parametrize("angles", [(25, 15), (250, -40)])
def test_perspective_views_match_oracle(name, angles, filt):
    _gpu()
    from workloads.camera import perspective_view
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "tree_small": _tree_small}[name]()
    vals = np.random.default_rng(14).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    centre, size = _centre(g)
    view = dict(perspective_view(centre, 1.2 * size, angles[0], angles[1], 44, 36, fov=45,
                                 step=0.41), filter=filt)
    lut = ramp_lut(0.08)
    lb = LB.from_geometry(g)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut, scale=1.2, offset=0.02)
    ref = oracle_render(g.coords, vals, view, lut, scale=1.2, offset=0.02)
    assert ref[..., 3].max() > 0.05
    _check(img, ref, view)


def test_perspective_full_size_tree_sampled_rays():
    """A pinhole view of the 5.6M-site tree; the oracle recomputes 128 seeded
    pixels (32 among the lit ones), each with its own direction."""
    _gpu()
    from workloads.camera import perspective_view
    g = wl.config_geometry("tree1024")
    vals = np.random.default_rng(15).uniform(0.0, 1.0, g.n_sites).astype(np.float32)
    lb = LB.from_geometry(g, storage="f16")
    view = perspective_view((512, 512, 512), 1400, 35, 25, 512, 512, fov=50, step=1.0)
    lut = ramp_lut(0.05)
    img = lb.render(torch.from_numpy(vals).cuda(), view, lut).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(16)
    pix = rng.integers(0, 512, (96, 2))
    lit = np.argwhere(img[..., 3] > 0)
    pix = np.concatenate([pix, lit[rng.choice(len(lit), 32, replace=False)][:, ::-1]])
    O, D, DR, DU = (np.asarray(view[k], dtype=np.int64) for k in ("origin", "dir", "dir_right", "dir_up"))
    origins = np.repeat(O[None, :], len(pix), axis=0)
    dirs = D[None, :] + pix[:, :1] * DR[None, :] + pix[:, 1:] * DU[None, :]
    ref = render_rays(g.coords, vals, origins, dirs, view["steps"], lut)
    got = img[pix[:, 1], pix[:, 0]]
    assert np.array_equal(got[:, 3] == 0, ref[:, 3] == 0)
    assert np.abs(got - ref).max() <= _tol(view)


def test_direction_spread_beyond_range_is_rejected():
    _gpu()
    g = wl.pipe()
    lb = LB.from_geometry(g)
    t = torch.zeros(g.n_sites, dtype=torch.float32, device="cuda")
    view = dict(orbit_view((9, 9, 31), 40, 0, 0, 4, 4), dir_right=[0, 1 << 47, 0])
    with pytest.raises(HemelbError) as ei:
        lb.render(t, view, ramp_lut())
    assert ei.value.code == L.HEMELB_EINVAL
