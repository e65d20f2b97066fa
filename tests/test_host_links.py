"""Host logic of the GPU path, checked on the CPU.

The library's C++ neighbour-table builder must classify every (site,
direction) pair exactly as the oracle's independent NumPy classification
does (pull streaming, Section 2: upstream point fluid / wall / past an
iolet), including periodic wrap-around; integer results, so bit-exact.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import lattice as olat
from oracle.links import Links
from paper_1906_11925_amd import links


GEOMS = {
    "pipe": wl.pipe,
    "couette": wl.couette,
    "channel": wl.channel,
    "closed": lambda: wl.closed_box(5, 4, 3),
    "periodic": lambda: wl.periodic_box(4, 3, 5),
    "periodic_thin": lambda: wl.periodic_box(1, 2, 3),
    "aneurysm_half": lambda: wl.aneurysm(half=True),
    "tree_small": lambda: wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1),
}


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", sorted(GEOMS))
def test_cpp_links_match_oracle(name, q):
    g = GEOMS[name]()
    coords, nbr = links(g.labels, g.shape, g.periodic, q)
    assert np.array_equal(coords, g.coords)
    ref = Links(g, olat.get(q)).codes()
    assert np.array_equal(nbr[:, 1:], ref[:, 1:])
    assert np.array_equal(nbr[:, 0], np.arange(g.n_sites))


def test_cpp_links_counts_only():
    g = wl.pipe()
    from paper_1906_11925_amd import lib as L
    import ctypes
    lib = L.load()
    lab = np.ascontiguousarray(g.labels)
    n = ctypes.c_int64(0)
    shp = np.array(g.shape, dtype=np.int32)
    per = np.zeros(3, dtype=np.int32)
    rc = lib.hemelb_lb_links(lab.ctypes.data_as(L.P(ctypes.c_uint8)), shp.ctypes.data_as(L.P(L.c_int32)),
                             per.ctypes.data_as(L.P(L.c_int32)), 15, ctypes.byref(n), None, None)
    assert rc == 0 and n.value == 13312
    rc = lib.hemelb_lb_links(lab.ctypes.data_as(L.P(ctypes.c_uint8)), shp.ctypes.data_as(L.P(L.c_int32)),
                             per.ctypes.data_as(L.P(L.c_int32)), 17, ctypes.byref(n), None, None)
    assert rc == L.HEMELB_EINVAL
