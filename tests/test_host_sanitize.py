"""The host library's planner under sanitizers (CPU only, no device).

The site list and link builder (hemelb_lb_links) and the layout planner
(hemelb_lb_plan, which validates the table, Morton-orders the sites and builds
the 16-bit table and the block records on a pool of threads) are compiled from
the library's source for the host only, with AddressSanitizer +
UndefinedBehaviorSanitizer and, separately, ThreadSanitizer, and driven by a
small C++ program (tests/native/plan_driver.cpp) on the half aneurysm, a small
Murray tree and a periodic Couette cell.  The run must be clean (any report
aborts it with a non-zero status) and its plans must equal those of the
regular build.
"""

import dataclasses
import os
import struct
import subprocess

import numpy as np
import pytest

import workloads as wl
from paper_1906_11925_amd import build as B
from paper_1906_11925_amd import links, plan
from paper_1906_11925_amd import lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
NATIVE = os.path.join(HERE, "native")
SOURCES = [os.path.join(NATIVE, "plan_driver.cpp"), os.path.join(NATIVE, "launch_stubs.cpp")]

FLAGS = {L.FLAG_TABLE32: "table32", L.FLAG_TABLE16: "table16", L.FLAG_BLOCKS: "blocks"}
STORES = {0: "f32", 1: "f16"}


def _geometries():
    return {
        "aneurysm_half": wl.aneurysm(half=True),
        "tree_small": wl.tree(box=128, r0=8.0, root=(64.0, 64.0, 4.0), generations=4, seed=2),
        "couette": wl.couette(H=6, Lx=8, Lz=8),
    }


def _write_labels(path, g, q):
    X, Y, Z = g.shape
    with open(path, "wb") as f:
        f.write(struct.pack("<8i", X, Y, Z, *(1 if p else 0 for p in g.periodic), q,
                            len(g.iolets)))
        for io in g.iolets:
            kind = L.IOLET_PRESSURE if io.kind == "pressure" else L.IOLET_VELOCITY
            f.write(struct.pack("<i4d", kind, *(float(v) for v in io.direction), float(io.mean)))
        f.write(np.ascontiguousarray(g.labels, dtype=np.uint8).tobytes())


@pytest.fixture(scope="module", params=["address", "thread"])
def driver(request, tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / f"plan_driver_{request.param}")
    try:
        B.build_sanitized(request.param, SOURCES, out)
    except FileNotFoundError:
        pytest.skip("hipcc not available")
    return request.param, out


@pytest.mark.parametrize("q", [15, 19])
def test_planner_is_clean_under_sanitizers(driver, q, tmp_path):
    kind, exe = driver
    env = dict(os.environ)
    # any report ends the run with status 66; leak checks need ptrace, which a
    # container may not grant, so they stay off
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=66"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=66"
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=66"
    for name, g in _geometries().items():
        path = str(tmp_path / f"{name}.bin")
        _write_labels(path, g, q)
        res = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=600)
        assert res.returncode == 0, f"{kind} sanitizer, {name}: rc {res.returncode}\n{res.stderr[-4000:]}"
        assert "WARNING: ThreadSanitizer" not in res.stderr, res.stderr[-4000:]
        assert "runtime error" not in res.stderr, res.stderr[-4000:]
        lines = res.stdout.splitlines()
        coords, nbr = links(g.labels, g.shape, g.periodic, q)
        assert lines[0] == f"sites {nbr.shape[0]}"
        # the driver passes each iolet's mean and direction only (no harmonics)
        ios = [dataclasses.replace(io, cos=(), sin=()) for io in g.iolets]
        kw = dict(lattice=q, coords=coords, iolets=ios)
        got = [ln.split() for ln in lines[1:] if ln.startswith("plan")]
        assert len(got) == 6
        for tok in got:
            st, flag, rc = int(tok[2]), int(tok[4]), int(tok[6])
            want = None
            try:
                want = plan(nbr, 0.6, storage=STORES[st], addressing=FLAGS[flag], **kw)
            except L.HemelbError as e:
                assert rc == e.code, (name, tok)
                continue
            assert rc == 0, (name, tok)
            assert int(tok[8]) == want["addressing"]
            assert int(tok[10]) == want["n_ghosts"]
            assert int(tok[12]) == want["pitch"]
            assert abs(float(tok[14]) - want["bytes_per_update"]) < 1e-5
            assert int(tok[16]) == want["device_bytes"]
        broken = [ln for ln in lines if ln.startswith("broken")]
        if nbr.shape[0] > 1:
            assert broken == [f"broken rc {L.HEMELB_EINVAL}"], broken
