"""Writes adjoint_aneurysm_half.json: stored values for the GPU adjoint test on the
half-size aneurysm with a live inlet gradient, computed from the FP64 oracle alone.

Problem (the adjoint workload's geometry and objective, truncated): the half-size
aneurysm (199,360 sites, D3Q15, tau 0.6) from rest, its pulsatile Ladd inlet
U(t) = a0 + a1 cos(2 pi t / 4000) + b1 sin(2 pi t / 4000) at (a0, a1, b1) =
(0.02, 0, 0.01), a Brinkman field alpha ~ U[0, 0.01] (seed 4, rounded to FP32),
T = 600 steps, objective window = the last 200 steps.  In 600 steps the inlet's
signal, travelling at the lattice sound speed 1/sqrt(3), reaches the dome (about
125 sites downstream) and the outlet (about 250), so both terms of J depend on the
inlet coefficients.  The objective's constants are frozen as the adjoint workload
fixes them: Q* = 0.9 x the window-mean outlet flux of the nominal run, and the
weight of the dome shear term such that both terms are equal at the nominal point.

Stored: T, window, Q*, the shear weight, J at the nominal point, and the central
finite differences (J(theta + eps e_k) - J(theta - eps e_k)) / (2 eps) for every
inlet coefficient k, each J evaluated by the oracle's forward step and objective.

Run from the repository root: python tests/golden/make_adjoint_aneurysm_half.py
(about 20 minutes on 4 cores; each J is one 600-step FP64 run).
"""

import dataclasses
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle.adjoint import Adjoint, Objective  # noqa: E402
from oracle.lbgk import LBGK  # noqa: E402

OUT = os.path.join(HERE, "adjoint_aneurysm_half.json")
T = 600
WINDOW = (400, 600)
EPS = 1e-6


def setup():
    g = wl.aneurysm(half=True)
    n = g.n_sites
    alpha = np.random.default_rng(4).uniform(0.0, 0.01, n).astype(np.float32).astype(np.float64)
    c = g.coords.astype(np.float64)
    C, R = g.info["centre"], g.info["radius"]
    sphere = ((c[:, 0] - C[0]) ** 2 + (c[:, 1] - C[1]) ** 2 + (c[:, 2] - C[2]) ** 2) < (R + 2) ** 2
    return g, alpha, sphere


def objective_terms(theta, q_target, lam):
    """(J, flux term, window fluxes) of one forward run with inlet coefficients theta."""
    g, alpha, sphere = setup()
    io = g.iolets[0]
    g.iolets[0] = dataclasses.replace(io, mean=float(theta[0]), cos=(float(theta[1]),),
                                      sin=(float(theta[2]),))
    o = LBGK(g, 15, alpha=alpha)
    _, has = o.wall_normals()
    adj = Adjoint(o, Objective(1, q_target, has & sphere, lam, WINDOW))
    A = o.rest_state()
    J = flux = 0.0
    qs = []
    for t in range(T):
        f = o.stream(A, t)
        if adj.obj.in_window(t):
            q = adj.flux(A, f)
            qs.append(q)
            flux += (q - q_target) ** 2
            J += (q - q_target) ** 2 + adj.wss_w * np.sum(adj.wss(f)[adj.dome_idx])
        A = o.collide(f)
    return J, flux, qs


def main():
    g, _, _ = setup()
    io = g.iolets[0]
    theta0 = np.array([io.mean, *io.cos, *io.sin], dtype=np.float64)
    _, _, qs = objective_terms(theta0, 0.0, 0.0)
    q_target = 0.9 * float(np.mean(qs))
    J1, flux, _ = objective_terms(theta0, q_target, 1.0)
    lam = flux / (J1 - flux)  # shear term equal to the flux term
    jobs = [(theta0, q_target, lam)]
    for k in range(len(theta0)):
        for sgn in (1.0, -1.0):
            th = theta0.copy()
            th[k] += sgn * EPS
            jobs.append((th, q_target, lam))
    with ProcessPoolExecutor(max_workers=4) as pool:
        res = list(pool.map(objective_terms, *zip(*jobs)))
    J = res[0][0]
    fd = [(res[1 + 2 * k][0] - res[2 + 2 * k][0]) / (2 * EPS) for k in range(len(theta0))]
    rec = {"workload": "aneurysm_half", "lattice": 15, "T": T, "window": list(WINDOW),
           "alpha": "U[0, 0.01], numpy default_rng(4), rounded to float32",
           "dome": "sites with a wall link within radius + 2 of the sphere's centre",
           "theta": theta0.tolist(), "q_target": q_target, "lam": lam, "J": J, "eps": EPS,
           "dJ_dtheta_fd": fd}
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
