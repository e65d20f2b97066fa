"""Closed-form pins of two oracle parts that the flow pins do not fix (CPU).

The Brinkman-damped collision (the adjoint workload's per-site damping field)
and the pressure iolet's incoming value (the link-wise equilibrium at the
iolet density with the site's own, one step lagged, velocity) are each checked
here against consequences that the mathematics fixes independently of how the
oracle writes them:

* the damped collision changes a site's momentum by exactly -(alpha/tau) m,
  keeps its mass, and relaxes its second moment towards rho/3 I + rho u_b u_b
  with u_b = (1 - alpha) u (moment identities of the quadratic equilibrium);
* in a periodic box streaming only moves populations around, so the total
  momentum decays exactly as (1 - alpha/tau)^n while the mass stays put;
* a uniform stream f^eq(rho_0, u_0) through a duct whose two pressure iolets
  hold rho_0 is a fixed point of the step, which pins both the imposed density
  and the velocity reading;
* a closed pipe whose iolets both hold rho_k has rho_k w_i as a fixed point, and
  the rest state at rho = 1 relaxes to it.

Each pin also rejects a planted mistake: a mutant oracle (a subclass made here,
on the CPU) that applies the damping to the density, to the linear term only,
reads u = 0 at the pressure iolet, or ignores the iolet density must fail it.
"""

import math

import numpy as np
import pytest

import workloads as wl
from workloads.geometry import Iolet
from oracle.lbgk import LBGK


# ---------------------------------------------------------------------------
# mutants: plausible mistakes in the two parts, planted in subclasses
# ---------------------------------------------------------------------------
class DampedDensity(LBGK):
    """Mistake: the damping factor multiplies the equilibrium's density."""

    def collide(self, f):
        rho, _, u = self.moments(f)
        a = 1.0 - self.alpha
        return f - self.omega * (f - self.feq(rho * a, u))


class DampedLinearOnly(LBGK):
    """Mistake: only the linear term of the equilibrium sees the damped velocity."""

    def collide(self, f):
        rho, _, u = self.moments(f)
        ub = u * (1.0 - self.alpha)[None, :]
        cu, cub = self.lat.cf @ u, self.lat.cf @ ub
        usq = np.sum(u * u, axis=0)
        feq = self.lat.w[:, None] * rho[None, :] * (1.0 + 3.0 * cub + 4.5 * cu * cu - 1.5 * usq)
        return f - self.omega * (f - feq)


class StillReservoir(LBGK):
    """Mistake: the pressure iolet injects the equilibrium at rest (u = 0)
    instead of at the site's own velocity."""

    def stream(self, A, t):
        self._still = True
        try:
            return super().stream(A, t)
        finally:
            self._still = False

    def moments(self, f):
        rho, m, u = super().moments(f)
        if getattr(self, "_still", False):
            return rho, 0.0 * m, 0.0 * u
        return rho, m, u


def unit_density_iolets(o):
    """Mistake: the pressure iolets inject at density 1 whatever they impose."""
    o.iolets = [Iolet("pressure", mean=1.0) if io.kind == "pressure" else io for io in o.iolets]
    return o


# ---------------------------------------------------------------------------
# Brinkman damping
# ---------------------------------------------------------------------------
def _second_moment(lat, f):
    return np.einsum("ia,ib,in->abn", lat.cf, lat.cf, f)


def _one_site_errors(cls, q, tau, seed):
    """Per-site errors of one damped collision against its moment identities:
    mass, momentum -(alpha/tau) m_s, and second moment
    (1 - w) Pi + w (rho/3 I + (1 - alpha)^2 m m^T / rho)."""
    g = wl.periodic_box(5, 4, 6)
    n = g.n_sites
    alpha = np.random.default_rng(seed).uniform(0.0, 0.5, n)
    o = cls(g, q, tau=tau, alpha=alpha)
    f = o.rest_state() + wl.random_deviations(q, n, seed + 1, 2e-3)
    A = o.collide(f)
    rho, m, _ = o.moments(f)
    rho2, m2, _ = o.moments(A)
    w = 1.0 / tau
    e_mass = np.abs(rho2 - rho).max()
    e_mom = np.abs(m2 - (1.0 - w * alpha)[None, :] * m).max() / np.abs(m).max()
    pi0, pi1 = _second_moment(o.lat, f), _second_moment(o.lat, A)
    peq = (rho / 3.0)[None, None, :] * np.eye(3)[:, :, None] \
        + ((1.0 - alpha) ** 2 / rho)[None, None, :] * m[:, None, :] * m[None, :, :]
    e_pi = np.abs(pi1 - ((1.0 - w) * pi0 + w * peq)).max()
    return e_mass, e_mom, e_pi


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("tau", [0.55, 0.8, 1.7])
def test_brinkman_collision_moments_per_site(q, tau):
    """One damped collision from a random state: each site keeps its mass
    exactly, its momentum becomes (1 - alpha_s/tau) m_s, and its second moment
    relaxes towards the equilibrium's rho/3 I + rho u_b u_b with
    u_b = (1 - alpha_s) u.  Catches the damping applied to the density or to
    the whole equilibrium (mass changes), to the momentum twice or with the
    wrong sign (momentum), or to the linear term only (second moment)."""
    e_mass, e_mom, e_pi = _one_site_errors(LBGK, q, tau, seed=3)
    assert e_mass < 1e-15
    assert e_mom < 1e-12
    assert e_pi < 1e-15


@pytest.mark.parametrize("cls, fails", [(DampedDensity, "mass"), (DampedLinearOnly, "pi")])
def test_brinkman_pins_reject_planted_mistakes(cls, fails):
    e_mass, e_mom, e_pi = _one_site_errors(cls, 15, 0.8, seed=3)
    err = {"mass": e_mass, "pi": e_pi}[fails]
    assert err > 1e-7, (cls.__name__, e_mass, e_mom, e_pi)


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("alpha", [0.01, 0.3])
def test_brinkman_periodic_box_momentum_decay(q, alpha):
    """Periodic box with a uniform damping field.  Streaming in a periodic box
    only permutes populations, so the totals change by the collision alone:
    the mass stays constant and the total momentum is m_0 (1 - alpha/tau)^n
    after n steps, from a uniform stream f^eq(rho_0, u_0) (which stays uniform)
    and from a random state alike."""
    tau, steps = 0.7, 50
    g = wl.periodic_box(6, 5, 7, tau=tau)
    o = LBGK(g, q, alpha=np.full(g.n_sites, alpha))
    n = o.n
    u0 = np.array([0.02, -0.01, 0.03])
    uniform = o.feq(np.full(n, 1.003), np.repeat(u0[:, None], n, axis=1))
    rand = o.rest_state() + wl.random_deviations(q, n, 9, 1e-3)
    for A in (uniform, rand):
        mass0, mom0 = o.totals(A)
        for k in range(1, steps + 1):
            A, _ = o.step(A, k - 1)
            if k % 10 == 0:
                mass, mom = o.totals(A)
                assert abs(mass - mass0) / mass0 < 1e-14
                expect = mom0 * (1.0 - alpha / tau) ** k
                assert np.abs(mom - expect).max() <= 1e-12 * np.abs(mom0).max()


def test_brinkman_full_damping_is_rest_equilibrium():
    """alpha = 1 removes the velocity from the equilibrium: at tau = 1 one step
    from any state lands on f^eq(rho, 0) = rho w_i at every site."""
    g = wl.periodic_box(4, 4, 4, tau=1.0)
    o = LBGK(g, 15, alpha=np.ones(g.n_sites))
    A = o.rest_state() + wl.random_deviations(15, o.n, 2, 1e-3)
    A1, f = o.step(A, 0)
    rho = f.sum(axis=0)
    assert np.abs(A1 - o.lat.w[:, None] * rho[None, :]).max() < 1e-16


# ---------------------------------------------------------------------------
# pressure iolets
# ---------------------------------------------------------------------------
def _duct_drift(cls, q, u0z, rho0=1.002, steps=20, mutate=None):
    g = wl.duct(3, 4, 10, rho_in=rho0, rho_out=rho0, tau=0.7)
    o = cls(g, q)
    if mutate:
        o = mutate(o)
    n = o.n
    u0 = np.array([0.0, 0.0, u0z])
    A0 = o.feq(np.full(n, rho0), np.repeat(u0[:, None], n, axis=1))
    A, _ = o.run(A0, 0, steps)
    return np.abs(A - A0).max()


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("u0z", [0.03, -0.05])
def test_pressure_iolet_uniform_stream_is_a_fixed_point(q, u0z):
    """A duct periodic across, with pressure iolets at both ends holding rho_0,
    filled with the uniform stream f^eq(rho_0, u_0 z) (flowing either way):
    every site pulls f^eq(rho_0, u_0) from its neighbours, and the iolet links
    get f^eq(rho_k, u_s) with u_s = u_0 read from the site's own populations,
    so the state is a fixed point to round-off.  Catches an iolet that injects
    the rest equilibrium (u = 0), the velocity with the wrong sign, or the
    wrong density."""
    assert _duct_drift(LBGK, q, u0z) < 1e-15


def test_pressure_iolet_pin_rejects_planted_mistakes():
    assert _duct_drift(StillReservoir, 15, 0.03) > 1e-4
    assert _duct_drift(LBGK, 15, 0.03, mutate=unit_density_iolets) > 1e-5


@pytest.mark.parametrize("q", [15, 19])
def test_pressure_iolet_imposes_its_density(q):
    """A pipe closed by walls along its side whose two pressure iolets both
    hold rho_k = 1.001: rho_k w_i (at rest) is a fixed point, and the rest
    state at rho = 1 fills up to it (density error below 1e-12 and no flow
    left after 1600 steps).  Catches an iolet that ignores the imposed
    density (the pipe would stay at rho = 1)."""
    rk = 1.001
    g = wl.pipe(X=8, Y=8, Z=12, r2=9.0, rho_in=rk, rho_out=rk, tau=0.8)
    o = LBGK(g, q)
    At = rk * o.rest_state()
    A1, _ = o.run(At, 0, 10)
    assert np.abs(A1 - At).max() < 1e-15
    A, _ = o.run(o.rest_state(), 0, 1600)
    rho, _, u = o.moments(A)
    assert np.abs(rho - rk).max() < 1e-12
    assert np.abs(u).max() < 1e-12
    m = unit_density_iolets(LBGK(g, q))
    A, _ = m.run(m.rest_state(), 0, 200)
    assert np.abs(A.sum(axis=0) - rk).max() > 9e-4


def test_pressure_iolet_lags_by_one_step():
    """The velocity the iolet reads is the site's stored (post-collision) one
    of the previous step, not the velocity after streaming: with a state
    whose stored velocity at the inlet sites differs from its neighbours',
    the injected populations follow the stored one.  Checked on one link
    against f^eq(rho_k, u_s) evaluated from the moments of A[:, s] by hand."""
    g = wl.duct(2, 2, 4, rho_in=1.002, rho_out=1.0, tau=0.7)
    o = LBGK(g, 15)
    A = o.rest_state() + wl.random_deviations(15, o.n, 5, 2e-3)
    f = o.stream(A, 0)
    lat = o.lat
    c = g.coords
    s = int(np.nonzero(c[:, 2] == 0)[0][0])
    i = int(np.nonzero((lat.c[:, 2] == 1) & (lat.c[:, 0] == 1) & (lat.c[:, 1] == 1))[0][0])
    rho_s = math.fsum(A[:, s])
    m_s = [math.fsum(A[k, s] * lat.c[k, a] for k in range(15)) for a in range(3)]
    u_s = [x / rho_s for x in m_s]
    cu = sum(lat.c[i, a] * u_s[a] for a in range(3))
    uu = sum(x * x for x in u_s)
    expect = float(lat.w_exact[i]) * 1.002 * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    assert abs(f[i, s] - expect) < 1e-17
