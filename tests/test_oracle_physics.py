"""Physics pins of the FP64 oracle (CPU).

What fixes the oracle here is the physics and exact invariants, not a second
copy of its formulas:

* plane Couette flow between a resting bounce-back wall and a Ladd moving
  wall: the steady profile is linear and halfway bounce-back reproduces it
  exactly, so velocity, shear stress sigma_xy = rho nu U / H and the wall
  shear stress at the resting wall are known in closed form;
* plane channel with pressure iolets: halfway bounce-back gives the exact
  parabola at the "magic" relaxation Lambda = (tau - 1/2)^2 = 3/16
  (Ginzburg and d'Humieres, 2003) and a visibly different one elsewhere;
* straight pipe: Hagen-Poiseuille flux within a few percent (staircase wall);
  mirror symmetry to round-off;
* rest equilibrium invariance, mass (and momentum) conservation, and the
  exact mass bookkeeping across iolets;
* agreement of the sparse neighbour-list step with the dense shifted-array
  step (an independent formulation of the same streaming).
"""

import math

import numpy as np
import pytest

import workloads as wl
from workloads.geometry import Iolet
from oracle.lbgk import LBGK
from oracle.dense import DenseLBGK
from oracle.links import IOLET_LINK


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.5])
def test_couette_closed_form(tau):
    H, U = 8, 0.01
    g = wl.couette(H=H, Lx=2, Lz=2, U=U, tau=tau)
    o = LBGK(g, 15)
    nu = (tau - 0.5) / 3.0
    nsteps = int(30.0 / (nu * (math.pi / H) ** 2))
    A, f = o.run(o.rest_state(), 0, nsteps)
    p, u, sig, wss = o.observables(f)
    y = g.coords[:, 1]
    exact = U * (y + 0.5) / H
    assert np.abs(u[0] - exact).max() / U < 1e-10
    assert np.abs(u[1]).max() < 1e-14 and np.abs(u[2]).max() < 1e-14
    tau_xy = nu * U / H
    np.testing.assert_allclose(sig[0, 1], tau_xy, rtol=1e-9)
    np.testing.assert_allclose(sig[1, 0], tau_xy, rtol=1e-9)
    np.testing.assert_allclose(wss[y == 0], tau_xy, rtol=1e-9)
    # no bounce-back wall next to the moving-wall sites, so no wall normal there
    assert np.all(wss[y == H - 1] == 0.0)
    np.testing.assert_allclose(3 * p, 1.0, atol=1e-12)


def _channel_shape_error(tau, nsteps):
    H, L = 8, 48
    g = wl.channel(H=H, L=L, Lx=2, tau=tau)
    o = LBGK(g, 15)
    _, f = o.run(o.rest_state(), 0, nsteps)
    _, u, _, _ = o.observables(f)
    c = g.coords
    sel = (c[:, 2] == L // 2) & (c[:, 0] == 0)
    yp = c[sel, 1] - (H - 1) / 2.0
    r = u[2, sel] / (1.0 - (2.0 * yp / H) ** 2)
    return np.abs(r / r.mean() - 1.0).max()


def test_channel_parabola_at_magic_tau():
    assert _channel_shape_error(0.5 + math.sqrt(3.0) / 4.0, 6000) < 1e-6


def test_channel_parabola_slip_off_magic_tau():
    # the halfway wall position is tau-dependent away from Lambda = 3/16
    assert _channel_shape_error(0.6, 3000) > 1e-2


def test_pipe_poiseuille_and_symmetry():
    g = wl.pipe()
    assert g.n_sites == 13312
    o = LBGK(g, 15)
    _, f = o.run(o.rest_state(), 0, 2000)
    p, u, _, wss = o.observables(f)
    c = g.coords
    rho = 3 * p
    nu = (0.8 - 0.5) / 3.0
    zs = np.arange(16, 48)
    pm = np.array([p[c[:, 2] == z].mean() for z in zs])
    G = -np.polyfit(zs, pm, 1)[0]
    reff = math.sqrt(208 / math.pi)
    Q = np.array([(rho * u[2])[c[:, 2] == z].sum() for z in zs])
    assert Q.std() / Q.mean() < 1e-3
    q_hp = math.pi * G * reff ** 4 / (8 * nu)
    assert abs(Q.mean() / q_hp - 1) < 0.05
    sel = c[:, 2] == 32
    r2 = (c[sel, 0] - 9.5) ** 2 + (c[sel, 1] - 9.5) ** 2
    prof = G * (reff ** 2 - r2) / (4 * nu * rho[sel].mean())
    assert np.linalg.norm(u[2, sel] - prof) / np.linalg.norm(prof) < 0.08
    idx = {tuple(x): i for i, x in enumerate(c.tolist())}
    mx = np.array([idx[(19 - x, y, z)] for x, y, z in c.tolist()])
    sw = np.array([idx[(y, x, z)] for x, y, z in c.tolist()])
    assert np.abs(u[0] + u[0][mx]).max() < 1e-14
    assert np.abs(u[2] - u[2][mx]).max() < 1e-14
    assert np.abs(u[0] - u[1][sw]).max() < 1e-14
    assert np.abs(wss - wss[mx]).max() < 1e-16


@pytest.mark.parametrize("q", [15, 19])
def test_rest_state_invariant(q):
    """The rest equilibrium with iolets at rho = 1 / U = 0 is a fixed point.  The
    oracle stores plain f, whose lattice-weight sum is 1 only to round-off, so
    the pin is at round-off level here (shifted storage makes it exact)."""
    pipe = wl.pipe(rho_in=1.0, rho_out=1.0)
    g = wl.aneurysm(half=True)
    still = wl.geometry.Geometry(g.name, g.shape, g.labels, iolets=[
        Iolet("velocity", direction=(0.0, 1.0, 0.0), mean=0.0), Iolet("pressure", mean=1.0)],
        tau=0.6, profile=g.profile)
    for geom in (pipe, still, wl.couette(U=0.0)):
        o = LBGK(geom, q)
        A0 = o.rest_state()
        A, _ = o.run(A0, 0, 5)
        assert np.abs(A - A0).max() < 1e-15


@pytest.mark.parametrize("q", [15, 19])
def test_mass_conservation_closed_and_periodic(q):
    o = LBGK(wl.closed_box(6, 5, 7), q, tau=0.55)
    A = o.rest_state() + wl.random_deviations(q, o.n, 3, 1e-2 / q)
    m0, _ = o.totals(A)
    A, _ = o.run(A, 0, 300)
    m1, _ = o.totals(A)
    assert abs(m1 - m0) / m0 < 1e-13
    o = LBGK(wl.periodic_box(6, 5, 7), q, tau=0.55)
    A = o.rest_state() + wl.random_deviations(q, o.n, 4, 1e-2 / q)
    m0, p0 = o.totals(A)
    A, _ = o.run(A, 0, 300)
    m1, p1 = o.totals(A)
    assert abs(m1 - m0) / m0 < 1e-13
    assert np.abs(p1 - p0).max() < 1e-13


@pytest.mark.parametrize("name", ["pipe", "aneurysm_half"])
def test_mass_bookkeeping_across_iolets(name):
    """M(A_{t+1}) - M(A_t) equals the sum over iolet links (s, i) of the
    incoming value f_i(s) minus the outgoing population A_t[opp(i), s]."""
    g = wl.config_geometry(name)
    o = LBGK(g, 15)
    A = o.rest_state() + wl.random_deviations(15, o.n, 5, 1e-3)
    for t in range(3):
        An, f = o.step(A, t)
        lhs = math.fsum(An.ravel()) - math.fsum(A.ravel())
        terms = []
        for i in range(1, o.q):
            sel = o.links.kind[i] == IOLET_LINK
            terms += f[i, sel].tolist() + (-A[o.lat.opp[i], sel]).tolist()
        rhs = math.fsum(terms)
        # each stored value carries one rounding of the collision
        assert abs(lhs - rhs) < 1e-16 * o.n * o.q
        A = An


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", ["pipe", "couette", "channel", "closed", "periodic", "aneurysm_half"])
def test_sparse_matches_dense(q, name):
    g = {"pipe": wl.pipe, "couette": wl.couette, "channel": wl.channel,
         "closed": wl.closed_box, "periodic": wl.periodic_box,
         "aneurysm_half": lambda: wl.aneurysm(half=True)}[name]()
    o, d = LBGK(g, q), DenseLBGK(g, q)
    A = o.rest_state() + wl.random_deviations(q, o.n, 11, 1e-3)
    F = d.to_dense(A)
    for t in range(3):
        A, _ = o.step(A, t)
        F, _ = d.step(F, t)
    assert np.abs(d.to_sites(F) - A).max() < 1e-14


def test_tree_small_links_consistent():
    """Every fluid link of a small seeded tree is reciprocal, and inlet/outlet
    links exist."""
    g = wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1)
    o = LBGK(g, 15)
    L = o.links
    for i in range(1, o.q):
        fl = np.nonzero(L.kind[i] == 0)[0]
        assert np.array_equal(L.src[o.lat.opp[i], L.src[i, fl]], fl)
    kinds = set(np.unique(L.iolet[L.kind == IOLET_LINK]).tolist())
    assert kinds == {0, 1}


def test_sampled_step_equals_full_step():
    """The oracle's sampled form (links and step at chosen sites only, reading the
    full state) reproduces the full step at those sites exactly."""
    g = wl.aneurysm(half=True)
    full = LBGK(g, 15)
    sites = np.sort(np.random.default_rng(0).choice(full.n, 700, replace=False))
    alpha = np.random.default_rng(1).uniform(0, 0.01, full.n)
    full_a = LBGK(g, 15, alpha=alpha)
    samp = LBGK(g, 15, alpha=alpha, sites=sites)
    A = full.rest_state() + wl.random_deviations(15, full.n, 3, 1e-3)
    An, f = full_a.step(A, 5)
    As, fs = samp.step(A, 5)
    assert np.array_equal(As, An[:, sites]) and np.array_equal(fs, f[:, sites])


def test_pulsatile_inlet_mass_over_a_period():
    """Pulsatile Ladd inlet U(t) = U0 (1 + 0.5 sin(2 pi t / P)): the mass that
    enters during one period equals P * U0 * sum of W_s over the inlet plane
    (area-weighted parabolic profile), up to the rim sites whose links are
    partly walls (a few percent here).  The sinusoid integrates to zero over
    the period, so only the mean inlet speed survives."""
    P, U0 = 100, 0.02
    g = wl.pipe(X=12, Y=12, Z=16, r2=25.0, tau=0.8,
                inlet_velocity=(U0, (0.0,), (0.5 * U0,), float(P)))
    o = LBGK(g, 15)
    A = o.rest_state()
    A, _ = o.run(A, 0, P)
    inlet = [(i, np.nonzero((o.links.kind[i] == IOLET_LINK) & (o.links.iolet[i] == 0))[0])
             for i in range(1, o.q)]
    injected = 0.0
    for t in range(P, 2 * P):
        An, f = o.step(A, t)
        for i, sel in inlet:
            injected += np.sum(f[i, sel] - A[o.lat.opp[i], sel])
        A = An
    W = g.site_weight()
    plane = g.coords[:, 2] == 0
    expected = P * U0 * np.sum(W[plane])
    assert abs(injected / expected - 1.0) < 0.05


@pytest.mark.parametrize("gap", [0.2, 0.5, 0.8])
@pytest.mark.parametrize("tau", [0.6, 1.5])
def test_bfl_couette_offset_wall_exact(gap, tau):
    """Interpolated (BFL) walls place the wall where the geometry puts it: plane
    Couette with the resting wall at y = -gap is linear in y with zero at -gap,
    and sigma_xy = nu U / (H - 1/2 + gap), to round-off."""
    H, U = 8, 0.01
    g = wl.couette(H=H, Lx=2, Lz=2, U=U, tau=tau, wall_gap=gap)
    o = LBGK(g, 15, wall_q=g.wall_fractions(LBGK(g, 15).lat.c))
    nu = (tau - 0.5) / 3
    _, f = o.run(o.rest_state(), 0, int(40 / (nu * (math.pi / H) ** 2)))
    _, u, sig, wss = o.observables(f)
    y = g.coords[:, 1]
    span = H - 0.5 + gap
    assert np.abs(u[0] - U * (y + gap) / span).max() / U < 1e-10
    np.testing.assert_allclose(sig[0, 1], nu * U / span, rtol=1e-9)
    np.testing.assert_allclose(wss[y == 0], nu * U / span, rtol=1e-9)


def test_bfl_pipe_flux_uses_true_radius():
    """With BFL walls at the circle (radius 8) the pipe's flux matches
    Hagen-Poiseuille with the true radius far better than halfway bounce-back's
    staircase does (0.1% against 2%)."""
    g = wl.pipe()
    out = {}
    for name, wq in (("bb", None), ("bfl", g.wall_fractions(LBGK(g, 15).lat.c))):
        o = LBGK(g, 15, wall_q=wq)
        _, f = o.run(o.rest_state(), 0, 2000)
        p, u, _, _ = o.observables(f)
        c = g.coords
        zs = np.arange(16, 48)
        G = -np.polyfit(zs, [p[c[:, 2] == z].mean() for z in zs], 1)[0]
        Q = np.mean([((3 * p) * u[2])[c[:, 2] == z].sum() for z in zs])
        out[name] = Q / (math.pi * G * 8.0 ** 4 / (8 * 0.1))
    assert abs(out["bfl"] - 1) < 0.002
    assert abs(out["bb"] - 1) > 0.01


def test_bfl_half_is_halfway_bounce_back():
    g = wl.aneurysm(half=True)
    o = LBGK(g, 15)
    wq = np.where(np.isnan(g.wall_fractions(o.lat.c)), np.nan, 0.5)
    ob = LBGK(g, 15, wall_q=wq)
    A = o.rest_state() + wl.random_deviations(15, o.n, 2, 1e-3)
    assert np.array_equal(o.step(A, 3)[0], ob.step(A, 3)[0])
