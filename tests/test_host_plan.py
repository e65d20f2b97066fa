"""Host planning of the device layout (CPU only, no device work): which
addressing the library picks, and the sizes it reports.

Block addressing cuts the lattice into 4x4x4 blocks and finds every link from
the sites' positions; the library checks each link against the caller's table
and uses the block form only where all of them agree.  These tests recompute
the block counts, ghost cells and byte figures independently in NumPy from the
site coordinates and compare.
"""

import math
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import workloads as wl
from paper_1906_11925_amd import lib as L
from paper_1906_11925_amd import links, plan
from paper_1906_11925_amd.lb import lattice_vectors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _args(g, q=15):
    coords, nbr = links(g.labels, g.shape, g.periodic, q)
    return coords, nbr, dict(lattice=q, coords=coords, iolets=list(g.iolets),
                             site_weight=g.site_weight())


def _expected_blocks(coords, nbr, q):
    """(fluid blocks, all blocks, ghost cells) from positions alone."""
    c = np.asarray(coords, dtype=np.int64)
    fb = {tuple(b) for b in (c >> 2)}
    lat = lattice_vectors(q)
    cells = set()
    for i in range(1, q):
        io = nbr[:, i] <= -2
        for p in c[io] - lat[i]:
            cells.add(tuple(p))
    gb = {tuple(np.asarray(p) >> 2) for p in cells}
    return len(fb), len(fb | gb), len(cells)


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "tree_small"])
def test_block_addressing_is_chosen_and_sized(name, q):
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "tree_small": lambda: wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3,
                                       seed=1)}[name]()
    coords, nbr, kw = _args(g, q)
    n = nbr.shape[0]
    auto = plan(nbr, g.tau, addressing="blocks", **kw)
    t16 = plan(nbr, g.tau, addressing="table16", **kw)
    t32 = plan(nbr, g.tau, addressing="table32", **kw)
    assert auto["addressing"] == L.ADDR_BLOCKS
    assert t16["addressing"] == L.ADDR_TABLE16 and t32["addressing"] == L.ADDR_TABLE32
    nfluid, nblocks, ncells = _expected_blocks(coords, nbr, q)
    links_io = int(np.sum(nbr[:, 1:] <= -2))
    assert auto["n_ghosts"] == t16["n_ghosts"] == links_io
    assert auto["pitch"] == math.ceil((n + ncells) / 64) * 64
    assert t16["pitch"] == math.ceil((n + links_io) / 64) * 64
    groups = math.ceil(n / 256)
    pops = 2 * q * 4
    # staged copies: per group an 8-byte entry, 28-byte rows for its own blocks and
    # 16-byte records (own blocks and their neighbours, each block at least once)
    assert auto["bytes_per_update"] >= pops + (8 * groups + 16 * nfluid) / n
    assert auto["bytes_per_update"] <= pops + (8 * groups + (28 + 16 + 27 * 16) * 2 * nblocks) / n
    assert t32["bytes_per_update"] == pops + 4 * (q - 1)
    assert auto["bytes_per_update"] < t16["bytes_per_update"] < t32["bytes_per_update"]
    assert auto["device_bytes"] < t16["device_bytes"] < t32["device_bytes"]


def test_default_addressing_is_blocks_where_they_apply():
    """Without a request: block addressing in every storage when the links are the
    ones the positions imply; the 16-bit table without coordinates."""
    g = wl.pipe()
    coords, nbr, kw = _args(g)
    for st in ("f32", "f16", "bf16"):
        assert plan(nbr, g.tau, storage=st, **kw)["addressing"] == L.ADDR_BLOCKS
    kw.pop("coords")
    assert plan(nbr, g.tau, **kw)["addressing"] == L.ADDR_TABLE16


def test_plan_matches_population_bytes():
    g = wl.pipe()
    _, nbr, kw = _args(g)
    for storage, elem in (("f32", 4), ("f16", 2), ("bf16", 2)):
        p = plan(nbr, g.tau, storage=storage, **kw)
        assert p["device_bytes"] > 2 * 15 * p["pitch"] * elem
        assert p["bytes_per_update"] > 2 * 15 * elem


def test_periodic_links_fall_back_to_the_table():
    g = wl.periodic_box(5, 7, 6)
    _, nbr, kw = _args(g)
    assert plan(nbr, g.tau, storage="f16", **kw)["addressing"] == L.ADDR_TABLE16
    with pytest.raises(L.HemelbError) as ei:
        plan(nbr, g.tau, addressing="blocks", **kw)
    assert ei.value.code == L.HEMELB_EINVAL
    assert "block addressing does not apply" in str(ei.value) and "positions imply" in str(ei.value)


def test_links_not_implied_by_positions_fall_back():
    """A wall placed between two neighbouring fluid sites (a reciprocal pair of
    fluid links turned into walls) is valid for the table but not positional."""
    g = wl.pipe()
    coords, nbr, kw = _args(g)
    bad = nbr.copy()
    s = 5000
    i = 1
    t = bad[s, i]
    assert t >= 0
    bad[s, i] = -1  # HEMELB_LINK_WALL
    bad[t, 2] = -1
    assert plan(bad, g.tau, storage="f16", **kw)["addressing"] == L.ADDR_TABLE16
    with pytest.raises(L.HemelbError) as ei:
        plan(bad, g.tau, addressing="blocks", **kw)
    assert f"site {s}, direction {i}" in str(ei.value) or f"site {t}, direction 2" in str(ei.value)


def test_one_position_with_two_iolet_ids_falls_back():
    g = wl.pipe()
    coords, nbr, kw = _args(g)
    bad = nbr.copy()
    s = int(np.nonzero(np.any(bad[:, 1:] <= -2, axis=1))[0][0])
    i = int(np.nonzero(bad[s] <= -2)[0][0])
    bad[s, i] = -3  # iolet 1 where the position lies past iolet 0
    assert plan(bad, g.tau, storage="f16", **kw)["addressing"] == L.ADDR_TABLE16


def test_no_coordinates_or_interpolated_walls_use_the_table():
    g = wl.pipe()
    coords, nbr, kw = _args(g)
    kw.pop("coords")
    assert plan(nbr, g.tau, storage="f16", **kw)["addressing"] == L.ADDR_TABLE16
    with pytest.raises(L.HemelbError) as ei:
        plan(nbr, g.tau, addressing="blocks", **kw)
    assert "coordinates" in str(ei.value)
    wq = np.full(nbr.shape, 0.3, dtype=np.float32)
    assert plan(nbr, g.tau, coords=coords, wall_q=wq, storage="f16", **kw)["addressing"] == \
        L.ADDR_TABLE16
    with pytest.raises(L.HemelbError) as ei:
        plan(nbr, g.tau, coords=coords, wall_q=wq, addressing="blocks", **kw)
    assert "interpolated" in str(ei.value)


def test_plan_rejects_what_create_rejects():
    g = wl.pipe()
    _, nbr, kw = _args(g)
    with pytest.raises(L.HemelbError) as ei:
        plan(nbr, 0.4, **kw)
    assert ei.value.code == L.HEMELB_EINVAL and "tau" in str(ei.value)
    with pytest.raises(ValueError):
        plan(nbr, g.tau, addressing="bricks", **kw)


def test_empty_lattice_plans():
    nbr = np.zeros((0, 15), dtype=np.int32)
    p = plan(nbr, 0.8, coords=np.zeros((0, 3), dtype=np.int32), addressing="blocks")
    assert p["n_sites"] == 0 and p["pitch"] == 64


def test_host_allocation_failure_is_an_error_code():
    """A host allocation that fails inside the planner comes back as
    HEMELB_ENOMEM (no C++ exception crosses the C ABI, no thread is left
    running): a child process caps its own address space just above what it
    holds, then plans a 4M-site periodic box whose tables need far more."""
    code = textwrap.dedent(f"""
        import resource, sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        import workloads as wl
        from paper_1906_11925_amd import links, plan, HemelbError
        from paper_1906_11925_amd import lib as L
        g = wl.periodic_box(160, 160, 160)
        coords, nbr = links(g.labels, g.shape, g.periodic, 15)
        used = int(open("/proc/self/statm").read().split()[0]) * resource.getpagesize()
        resource.setrlimit(resource.RLIMIT_AS, (used + (96 << 20), resource.RLIM_INFINITY))
        try:
            plan(nbr, g.tau, coords=coords)
        except HemelbError as e:
            print("code", e.code, str(e))
            sys.exit(0 if e.code == L.HEMELB_ENOMEM else 3)
        sys.exit(4)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "allocation" in r.stdout
