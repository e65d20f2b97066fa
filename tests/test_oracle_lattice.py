"""Pins of the oracle's lattice constants and local operators against what the
mathematics fixes (not against a retyping of the oracle's formulas).

The lattice must reproduce isotropic moments up to fourth order (the
property that makes the D3Q19 lattice of Section 2 recover Navier-Stokes);
the equilibrium must reproduce the hydrodynamic moments rho, rho u and
rho/3 I + rho u u; the LBGK collision must conserve mass and momentum.
"""

from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import lattice
from oracle.lbgk import LBGK
import workloads as wl


@pytest.mark.parametrize("q", [15, 19])
def test_moment_identities_exact(q):
    lat = lattice.get(q)
    c = lat.c.tolist()
    w = lat.w_exact
    assert sum(w) == 1
    for a in range(3):
        assert sum(wi * ci[a] for wi, ci in zip(w, c)) == 0
    for a, b in itertools.product(range(3), repeat=2):
        got = sum(wi * ci[a] * ci[b] for wi, ci in zip(w, c))
        assert got == (Fraction(1, 3) if a == b else 0)
    for a, b, g in itertools.product(range(3), repeat=3):
        assert sum(wi * ci[a] * ci[b] * ci[g] for wi, ci in zip(w, c)) == 0
    d = lambda i, j: 1 if i == j else 0  # noqa: E731
    for a, b, g, e in itertools.product(range(3), repeat=4):
        got = sum(wi * ci[a] * ci[b] * ci[g] * ci[e] for wi, ci in zip(w, c))
        want = Fraction(d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g), 9)
        assert got == want


@pytest.mark.parametrize("q", [15, 19])
def test_ordering_convention(q):
    lat = lattice.get(q)
    assert lat.q == q
    assert tuple(lat.c[0]) == (0, 0, 0)
    for k in range(1, q, 2):
        assert lat.opp[k] == k + 1 and lat.opp[k + 1] == k
        assert np.all(lat.c[k] == -lat.c[k + 1])
    assert len({tuple(v) for v in lat.c.tolist()}) == q
    norms = {15: {1, 3}, 19: {1, 2}}[q]
    assert {int(v @ v) for v in lat.c[1:]} == norms


@pytest.mark.parametrize("q", [15, 19])
def test_equilibrium_moments(q):
    o = LBGK(wl.closed_box(3, 3, 3), q)
    rng = np.random.default_rng(0)
    n = o.n
    rho = 1 + rng.uniform(-0.05, 0.05, n)
    u = rng.uniform(-0.08, 0.08, (3, n))
    fe = o.feq(rho, u)
    c = o.lat.cf
    np.testing.assert_allclose(fe.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(c.T @ fe, rho * u, rtol=1e-13, atol=1e-16)
    pi = np.einsum("ia,ib,in->abn", c, c, fe)
    want = rho / 3 * np.eye(3)[:, :, None] + rho * np.einsum("an,bn->abn", u, u)
    np.testing.assert_allclose(pi, want, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7])
def test_collision_conserves_and_tau1_is_equilibrium(q, tau):
    o = LBGK(wl.closed_box(3, 4, 2), q, tau=tau)
    f = o.rest_state() + wl.random_deviations(q, o.n, 7, 2e-3)
    A = o.collide(f)
    np.testing.assert_allclose(A.sum(0), f.sum(0), rtol=1e-14)
    np.testing.assert_allclose(o.lat.cf.T @ A, o.lat.cf.T @ f, atol=1e-16)
    if tau == 1.0:
        rho, _, u = o.moments(f)
        np.testing.assert_allclose(A, o.feq(rho, u), atol=1e-17)


def test_galilean_fixed_point():
    """A uniform equilibrium f^eq(1, u0) on a fully periodic box is a fixed point."""
    g = wl.periodic_box(4, 3, 5)
    o = LBGK(g, 15, tau=0.7)
    u0 = np.array([0.03, -0.02, 0.01])
    A = o.feq(np.ones(o.n), np.repeat(u0[:, None], o.n, axis=1))
    B, _ = o.run(A, 0, 20)
    np.testing.assert_allclose(B, A, atol=1e-16)
