"""Pins of the oracle's discrete adjoint (CPU).

What fixes the adjoint is the forward map itself, differentiated by a means
that shares none of the adjoint's algebra: central finite differences of the
FP64 forward step.

* dot-product tests per step: <L v, w> (L v by central differences of one step)
  equals <v, L^T w> (one reverse step), for the populations, the Brinkman
  field and the inlet's Fourier coefficients, with every link kind present
  (fluid, wall, Ladd velocity inlet, pressure outlet);
* full gradient of the flux + wall-shear objective over a window of steps
  against central differences of J, for all inlet coefficients, single alpha
  sites and a random alpha direction.
"""

import dataclasses

import numpy as np
import pytest

import workloads as wl
from oracle.lbgk import LBGK
from oracle.adjoint import Adjoint, Objective


def tiny_vessel(tau=0.7):
    return wl.pipe(X=8, Y=8, Z=12, r2=9.0, tau=tau,
                   inlet_velocity=(0.02, (0.0, 0.003), (0.01, 0.002), 40.0))


def _setup(alpha_seed=4, tau=0.7):
    g = tiny_vessel(tau)
    n = g.n_sites
    alpha = np.random.default_rng(alpha_seed).uniform(0.0, 0.01, n)
    o = LBGK(g, 15, alpha=alpha)
    c = g.coords
    _, has = o.wall_normals()
    dome = has & (c[:, 2] >= 4) & (c[:, 2] <= 7)
    return g, o, dome


def _with_theta(o, k, theta):
    io = o.iolets[k]
    H = len(io.cos)
    o.iolets[k] = dataclasses.replace(io, mean=float(theta[0]), cos=tuple(theta[1:1 + H]),
                                      sin=tuple(theta[1 + H:]))


def _theta(io):
    return np.array([io.mean, *io.cos, *io.sin], dtype=np.float64)


def test_one_step_dot_product():
    g, o, dome = _setup()
    rng = np.random.default_rng(1)
    A = o.rest_state() + wl.random_deviations(15, o.n, 2, 2e-3)
    t = 7
    obj = Objective(outlet=1, q_target=0.0, dome=dome, lam=0.0, window=(0, 0))
    adj = Adjoint(o, obj)
    v = rng.standard_normal(A.shape)
    w = rng.standard_normal(A.shape)
    eps = 1e-6
    Lv = (o.step(A + eps * v, t)[0] - o.step(A - eps * v, t)[0]) / (2 * eps)
    theta = {0: np.zeros(5)}
    f = o.stream(A, t)
    fhat, ah = adj.collide_T(f, w)
    LTw = adj.stream_T(fhat, A, t, theta)
    lhs, rhs = np.sum(Lv * w), np.sum(v * LTw)
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)
    # Brinkman field
    da = rng.standard_normal(o.n)
    a0 = o.alpha.copy()
    o.alpha = a0 + eps * da
    Ap = o.step(A, t)[0]
    o.alpha = a0 - eps * da
    Am = o.step(A, t)[0]
    o.alpha = a0
    lhs = np.sum((Ap - Am) / (2 * eps) * w)
    assert abs(lhs - np.sum(ah * da)) <= 1e-8 * abs(lhs)
    # inlet coefficients
    th0 = _theta(o.iolets[0])
    for k in range(5):
        e = np.zeros(5)
        e[k] = 1.0
        _with_theta(o, 0, th0 + eps * e)
        Ap = o.step(A, t)[0]
        _with_theta(o, 0, th0 - eps * e)
        Am = o.step(A, t)[0]
        _with_theta(o, 0, th0)
        lhs = np.sum((Ap - Am) / (2 * eps) * w)
        assert abs(lhs - theta[0][k]) <= 1e-7 * max(abs(lhs), 1e-12), k


@pytest.fixture(scope="module")
def problem():
    g, o, dome = _setup()
    T, W = 40, (25, 40)
    nominal = Adjoint(o, Objective(1, 0.0, dome, 0.0, W))
    _, _, qs = nominal.forward(o.rest_state(), T)
    q_target = 0.9 * qs.mean()
    flux_term = np.sum((qs - q_target) ** 2)
    wsum = 0.0
    A = o.rest_state()
    for t in range(T):
        f = o.stream(A, t)
        if W[0] <= t < W[1]:
            wsum += nominal.wss(f)[nominal.dome_idx].mean()
        A = o.collide(f)
    lam = flux_term / (wsum / (W[1] - W[0]))
    obj = Objective(1, q_target, dome, lam, W)
    return o, obj, T


def _J(o, obj, T):
    return Adjoint(o, obj).forward(o.rest_state(), T)[0]


def test_full_gradient_vs_finite_differences(problem):
    o, obj, T = problem
    adj = Adjoint(o, obj)
    J, tape, _ = adj.forward(o.rest_state(), T)
    theta, ahat, _ = adj.backward(tape, T)
    # both objective terms are active and of similar size
    assert J > 0
    th0 = _theta(o.iolets[0])
    for k in range(5):
        eps = 1e-7
        e = np.zeros(5)
        e[k] = eps
        _with_theta(o, 0, th0 + e)
        Jp = _J(o, obj, T)
        _with_theta(o, 0, th0 - e)
        Jm = _J(o, obj, T)
        _with_theta(o, 0, th0)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - theta[0][k]) <= 1e-6 * abs(fd) + 1e-12 * abs(J), (k, fd, theta[0][k])
    rng = np.random.default_rng(9)
    a0 = o.alpha.copy()
    sites = rng.choice(o.n, 6, replace=False)
    for s in sites:
        # one site moves J by ~1e-4 * eps: eps must stay well above J's round-off
        eps = 1e-4
        o.alpha = a0.copy()
        o.alpha[s] += eps
        Jp = _J(o, obj, T)
        o.alpha[s] -= 2 * eps
        Jm = _J(o, obj, T)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - ahat[s]) <= 1e-6 * abs(fd) + 1e-12 * abs(J), (s, fd, ahat[s])
    d = rng.standard_normal(o.n)
    eps = 1e-7
    o.alpha = a0 + eps * d
    Jp = _J(o, obj, T)
    o.alpha = a0 - eps * d
    Jm = _J(o, obj, T)
    o.alpha = a0
    fd = (Jp - Jm) / (2 * eps)
    assert abs(fd - np.dot(ahat, d)) <= 1e-6 * abs(fd)
