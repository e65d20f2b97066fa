"""Interpolated (BFL) walls on the GPU against the FP64 oracle.

The oracle's BFL walls are pinned by the exact off-grid Couette profile and
the pipe's true-radius Poiseuille flux (tests/test_oracle_physics.py).  The
library rounds every wall fraction to a multiple of 2^-15; the oracle is given
the same rounded fractions.
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from oracle.lbgk import LBGK  # noqa: E402
from oracle.links import IOLET_LINK, WALL_LINK  # noqa: E402
from paper_1906_11925_amd import LB, HemelbError  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

from lbtest import quantize, rel_max  # noqa: E402

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _q15(wq):
    k = np.clip(np.rint(wq * 32768.0), 1, 32767)
    return np.where(np.isnan(wq), np.nan, k / 32768.0)


def _fractions(g, q):
    return _q15(g.wall_fractions(LBGK(g, q).lat.c))


def _dev(lb):
    return lb.get_deviations().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "couette"])
def test_bfl_one_step_elementwise(name, q):
    _gpu()
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "couette": lambda: wl.couette(wall_gap=0.3)}[name]()
    wq = _fractions(g, q)
    o = LBGK(g, q, wall_q=wq)
    d = quantize(wl.random_deviations(q, o.n, 4, 1e-3), q, "f32")
    lb = LB.from_geometry(g, lattice=q, wall_q=wq)
    lb.set_deviations(torch.from_numpy(d), t=9)
    lb.step(1)
    gpu = _dev(lb)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    A, f = o.step(o.lat.w[:, None] + d, 9)
    op, ou, _, ow = o.observables(f)
    tol = 2.0 * q * q * 1e-3 * 2.0 ** -24
    assert np.abs(gpu - (A - o.lat.w[:, None])).max() < tol
    assert np.abs(u - ou.T).max() < tol and np.abs(w - ow).max() < tol
    assert np.abs(p - (op - 1 / 3)).max() < tol


def test_bfl_couette_offset_wall_on_gpu():
    _gpu()
    H, U, tau, gap = 8, 0.01, 1.0, 0.3
    g = wl.couette(H=H, Lx=2, Lz=2, U=U, tau=tau, wall_gap=gap)
    lb = LB.from_geometry(g, bfl=True)
    lb.step(1500)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    y = g.coords[:, 1]
    gq = round(gap * 32768) / 32768
    span = H - 0.5 + gq
    assert np.abs(u[:, 0] - U * (y + gq) / span).max() / U < 1e-5
    np.testing.assert_allclose(w[y == 0], (tau - 0.5) / 3 * U / span, rtol=1e-4)


def test_bfl_pipe_2000_steps_vs_oracle():
    _gpu()
    g = wl.pipe()
    wq = _fractions(g, 15)
    o = LBGK(g, 15, wall_q=wq)
    _, f = o.run(o.rest_state(), 0, 2000)
    op, ou, _, ow = o.observables(f)
    lb = LB.from_geometry(g, wall_q=wq)
    lb.step(2000)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    eu, ep, ew = rel_max(u, ou.T), rel_max(p, op - 1 / 3), rel_max(w, ow)
    print(f"pipe BFL f32: e_u={eu:.3e} e_p={ep:.3e} e_wss={ew:.3e}", flush=True)
    assert eu <= 1e-5 and ep <= 1e-5 and ew <= 1e-5


@pytest.mark.parametrize("q", [15, 19])
def test_wall_inlet_sites_ladd_and_bfl(q):
    """The paper's boundary set (section 3.B): Ladd velocity inlet, BFL walls, and
    at sites next to both the inlet and the wall, Ladd on the iolet links and BFL
    on the wall links of the same site.  The half aneurysm's inlet has such sites;
    they match the oracle element by element after one step, and the whole
    pulsatile flow matches it after 200 steps from rest."""
    _gpu()
    g = wl.aneurysm(half=True)
    wq = _fractions(g, q)
    o = LBGK(g, q, wall_q=wq)
    kind, iolet = o.links.kind, o.links.iolet
    vel = [k for k, io in enumerate(g.iolets) if io.kind == "velocity"]
    ladd = np.any((kind == IOLET_LINK) & np.isin(iolet, vel), axis=0)
    frac = np.nan_to_num(wq.T, nan=0.5)
    bfl = np.any((kind == WALL_LINK) & (frac != 0.5), axis=0)
    both = np.flatnonzero(ladd & bfl)
    print(f"D3Q{q}: {both.size} wall-inlet sites", flush=True)
    assert both.size > 50
    d = quantize(wl.random_deviations(q, o.n, 12, 1e-3), q, "f32")
    lb = LB.from_geometry(g, lattice=q, wall_q=wq)
    lb.set_deviations(torch.from_numpy(d), t=250)
    lb.step(1)
    gpu = _dev(lb)
    A, _ = o.step(o.lat.w[:, None] + d, 250)
    ref = A - o.lat.w[:, None]
    assert np.abs(gpu[:, both] - ref[:, both]).max() < 2.0 * q * q * 1e-3 * 2.0 ** -24
    lb.close()
    _, f = o.run(o.rest_state(), 0, 200)
    op, ou, _, ow = o.observables(f)
    lb = LB.from_geometry(g, lattice=q, wall_q=wq)
    lb.step(200)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    eu, ep, ew = rel_max(u, ou.T), rel_max(p, op - 1 / 3), rel_max(w, ow)
    print(f"D3Q{q} BFL + Ladd, 200 steps: e_u={eu:.3e} e_p={ep:.3e} e_wss={ew:.3e}", flush=True)
    assert eu <= 1e-5 and ep <= 1e-5 and ew <= 1e-5


def test_bfl_half_fraction_is_bit_identical_to_halfway():
    _gpu()
    g = wl.aneurysm(half=True)
    wq = np.where(np.isnan(g.wall_fractions(LBGK(g, 15).lat.c)), np.nan, 0.5)
    d = torch.from_numpy(quantize(wl.random_deviations(15, g.n_sites, 8, 1e-3), 15, "f16"))
    a = LB.from_geometry(g, storage="f16")
    b = LB.from_geometry(g, storage="f16", wall_q=wq)
    for lb in (a, b):
        lb.set_deviations(d)
        lb.step(10)
    assert torch.equal(a.get_state()[0], b.get_state()[0])


def test_adjoint_rejects_interpolated_walls():
    _gpu()
    g = wl.pipe(X=8, Y=8, Z=12, r2=9.0, inlet_velocity=(0.02, (), (), 1.0))
    lb = LB.from_geometry(g, bfl=True)
    lb.set_objective(1, 0.0, None, 0.0, (0, 2))
    lb.step(2)
    with pytest.raises(HemelbError) as ei:
        lb.adjoint_begin(2)
    assert ei.value.code == L.HEMELB_EINVAL
