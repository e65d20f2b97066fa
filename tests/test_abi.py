"""The C-ABI library loads, exports every declared entry point, and rejects
invalid arguments on the host before any device work (CPU-only)."""

import ctypes
import os

import numpy as np
import pytest

import workloads as wl
from paper_1906_11925_amd import lib as L
from paper_1906_11925_amd import links

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = L.load()
    names = L.header_functions()
    assert "hemelb_lb_create" in names and "hemelb_lb_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L._SIGS), "binding signatures out of sync with the header"


def test_strerror():
    lib = L.load()
    assert lib.hemelb_lb_strerror(L.HEMELB_EINVAL) == b"invalid argument"
    assert lib.hemelb_lb_strerror(0) == b"success"


def _desc(nbr, q=15, tau=0.8, storage=0, flags=0, iolets=None, n_iolets=0, coords=None,
          alpha=None):
    d = L.DescT()
    d.lattice, d.storage, d.flags = q, storage, flags
    d.n_sites = nbr.shape[0]
    d.nbr = nbr.ctypes.data_as(L.P(L.c_int32))
    d.tau = tau
    d.n_iolets = n_iolets
    d.iolets = iolets
    if coords is not None:
        d.coords = coords.ctypes.data_as(L.P(L.c_int32))
    if alpha is not None:
        d.alpha = alpha.ctypes.data_as(L.P(L.c_float))
    return d


def _create(d):
    lib = L.load()
    h = ctypes.c_void_p()
    rc = lib.hemelb_lb_create(ctypes.byref(h), ctypes.byref(d))
    return rc, L.last_error()


@pytest.fixture(scope="module")
def box():
    g = wl.closed_box(4, 3, 5)
    coords, nbr = links(g.labels, g.shape, g.periodic, 15)
    return coords, nbr


def test_reject_bad_lattice(box):
    _, nbr = box
    rc, msg = _create(_desc(nbr, q=17))
    assert rc == L.HEMELB_EINVAL and "lattice" in msg


@pytest.mark.parametrize("tau", [0.5, 0.3, float("nan")])
def test_reject_bad_tau(box, tau):
    _, nbr = box
    rc, msg = _create(_desc(nbr, tau=tau))
    assert rc == L.HEMELB_EINVAL and "tau" in msg


def test_reject_bad_storage_and_flags(box):
    _, nbr = box
    assert _create(_desc(nbr, storage=7))[0] == L.HEMELB_EINVAL
    assert _create(_desc(nbr, flags=16))[0] == L.HEMELB_EINVAL
    rc, msg = _create(_desc(nbr, flags=L.FLAG_BLOCKS | L.FLAG_TABLE16))
    assert rc == L.HEMELB_EINVAL and "at most one" in msg


def test_reject_nonreciprocal_link(box):
    _, nbr = box
    bad = nbr.copy()
    s = 3
    i = next(i for i in range(1, 15) if bad[s, i] >= 0)
    bad[s, i] = (bad[s, i] + 1) % bad.shape[0]
    rc, msg = _create(_desc(bad))
    assert rc == L.HEMELB_EINVAL and "reciprocal" in msg and f"({s}, {i})" in msg


def test_reject_out_of_range_and_unknown_iolet(box):
    _, nbr = box
    bad = nbr.copy()
    bad[0, 1] = bad.shape[0] + 5
    assert _create(_desc(bad))[0] == L.HEMELB_EINVAL
    bad = nbr.copy()
    bad[0, 1] = -2  # iolet 0, but no iolets given
    rc, msg = _create(_desc(bad))
    assert rc == L.HEMELB_EINVAL and "iolet" in msg


def test_reject_bad_iolet_descriptor(box):
    _, nbr = box
    io = (L.IoletT * 1)()
    io[0].kind = 5
    rc, msg = _create(_desc(nbr, iolets=io, n_iolets=1))
    assert rc == L.HEMELB_EINVAL and "kind" in msg
    io[0].kind = L.IOLET_VELOCITY
    io[0].n_harm = 2  # harmonics without arrays
    rc, msg = _create(_desc(nbr, iolets=io, n_iolets=1))
    assert rc == L.HEMELB_EINVAL and "harmonics" in msg


def test_reject_bad_coords_and_alpha(box):
    coords, nbr = box
    c = coords.copy()
    c[2, 1] = -1
    assert _create(_desc(nbr, coords=c))[0] == L.HEMELB_EINVAL
    c = coords.copy()
    c[1] = c[0]
    rc, msg = _create(_desc(nbr, coords=c))
    assert rc == L.HEMELB_EINVAL and "duplicate" in msg
    a = np.full(nbr.shape[0], 0.5, dtype=np.float32)
    a[4] = 1.5
    rc, msg = _create(_desc(nbr, alpha=a))
    assert rc == L.HEMELB_EINVAL and "alpha" in msg


def test_null_handle_calls():
    lib = L.load()
    assert lib.hemelb_lb_step(None, 1) == L.HEMELB_EINVAL
    assert lib.hemelb_lb_destroy(None) == L.HEMELB_EINVAL
    out = (ctypes.c_double * 4)()
    assert lib.hemelb_lb_totals(None, out) == L.HEMELB_EINVAL


def test_render_rejects_null_arguments():
    lib = L.load()
    v = L.ViewT()
    assert lib.hemelb_lb_render(None, None, ctypes.byref(v), None) == L.HEMELB_EINVAL


def test_reject_too_many_sites():
    """N >= 2^30 is rejected on the host before anything is allocated."""
    nbr = np.zeros((1, 15), dtype=np.int32)
    d = _desc(nbr)
    d.n_sites = 1 << 30
    rc, msg = _create(d)
    assert rc == L.HEMELB_EINVAL and "2^30" in msg


def test_reject_bad_objective_and_order():
    lib = L.load()
    # objective calls on a NULL handle, adjoint calls out of order are host-side errors
    assert lib.hemelb_lb_set_objective(None, None) == L.HEMELB_EINVAL
    assert lib.hemelb_lb_adjoint_begin(None, 4) == L.HEMELB_EINVAL
    assert lib.hemelb_lb_adjoint_grads(None, None, None) == L.HEMELB_EINVAL


def test_one_hip_runtime_in_the_process():
    """Loading the library first (a host call before torch is imported) still
    leaves a single HIP runtime mapped: torch's, which the library binds to."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1906_11925_amd import links\n"
        "import workloads as wl\n"
        "g = wl.pipe(); links(g.labels, g.shape, g.periodic, 15)\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"
