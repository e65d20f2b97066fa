"""Sparse FP64 lattice-BGK step (oracle).

State: post-collision populations A[i, s] (float64 [q, n]); the state after n
steps is A_n, with A_0 = w_i (rest equilibrium at rho = 1).  Step n (n >= 1)
uses boundary time t = n - 1 and maps A_{n-1} to A_n:

1. Pull streaming (Section 2, propagation): for each site s and direction i,
   with upstream point y = x_s - c_i,
   a. y fluid site s':      f_i(s) = A[i, s'];
   b. y wall:               f_i(s) = A[opp(i), s]          (halfway bounce-back,
                                                            the "simple bounce-back"
                                                            of Section 4);
   c. y past pressure iolet k:
                            f_i(s) = f_i^eq(rho_k(t), u_s), u_s the velocity of
                            the site's own stored populations A[:, s];
   d. y past velocity iolet k (Ladd, Section 2):
                            f_i(s) = A[opp(i), s] + 2 w_i rho0 (c_i . u_b) / cs^2,
                            rho0 = 1, u_b = U_k(t) W_s e_k.
2. Moments rho = sum_i f_i, m = sum_i c_i f_i, u = m / rho.
3. Equilibrium f_i^eq(rho, u) = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u).
4. LBGK collision (Section 2, collision): A'[i, s] = f_i - (f_i - f_i^eq(rho, u_b)) / tau,
   with the Brinkman-damped velocity u_b = (1 - alpha_s) u (alpha = 0 by default).

Interpolated walls (the BFL wall boundary Section 3.B selects; Bouzidi,
Firdaouss and Lallemand 2001, linear variant): with ``wall_q`` the wall of link
i at site s lies at fraction q of the way from x_s to x_s - c_i, and with
o = opp(i) (the population that travels into the wall)
   q <  1/2:  f_i(s) = 2q A[o, s] + (1 - 2q) A[o, s'],  s' = x_s + c_i (the site o
              pulls from); halfway bounce-back when s' is not a fluid site;
   q >= 1/2:  f_i(s) = A[o, s] / (2q) + (2q - 1)/(2q) A[i, s].
q = 1/2 gives halfway bounce-back in both branches.

Observables after n steps come from the pre-collision f of step n: pressure
p = rho / 3, velocity u, deviatoric stress
sigma = -(1 - 1/(2 tau)) sum_i c_i c_i (f_i - f_i^eq(rho, u)), and at sites with
at least one wall link the wall shear stress |sigma n - (n.sigma n) n| with
n = normalize(sum of c_i over wall links i) (pointing into the fluid).  The
paper only says that such lattice properties are computed and cached
(Section 3.C.2); these are their textbook definitions.
"""

import math

import numpy as np

from . import lattice as _lattice
from .links import Links, FLUID_LINK, WALL_LINK, IOLET_LINK


class LBGK:
    """The step over all sites, or with ``sites`` over a sample of them: the
    sampled form reads a full state A [q, N] and returns f and A' only at the
    sampled sites (for workloads too large to step whole on the CPU)."""

    def __init__(self, geom, q=15, tau=None, alpha=None, sites=None, wall_q=None):
        self.geom = geom
        self.lat = _lattice.get(q)
        self.q = self.lat.q
        self.links = Links(geom, self.lat, sites)
        self.n = self.links.n
        self.sites = None if sites is None else np.asarray(sites)
        self.tau = float(geom.tau if tau is None else tau)
        self.omega = 0.0 if math.isinf(self.tau) else 1.0 / self.tau
        self.alpha = None if alpha is None else np.asarray(alpha, dtype=np.float64)
        self.W = geom.site_weight()
        if self.sites is not None:
            self.W = self.W[self.sites]
            if self.alpha is not None:
                self.alpha = self.alpha[self.sites]
        self.wall_q = None
        if wall_q is not None:
            wq = np.asarray(wall_q, dtype=np.float64)
            self.wall_q = (wq if self.sites is None else wq[self.sites]).T  # [q, n]
        self.iolets = list(geom.iolets)
        # per direction: iolet link masks, grouped by iolet
        self._io = []
        for i in range(self.q):
            groups = []
            sel_all = self.links.kind[i] == IOLET_LINK
            for k in np.unique(self.links.iolet[i][sel_all]):
                groups.append((int(k), np.nonzero(sel_all & (self.links.iolet[i] == k))[0]))
            self._io.append(groups)
        self._fluid = [np.nonzero(self.links.kind[i] == FLUID_LINK)[0] for i in range(self.q)]
        self._wall = [np.nonzero(self.links.kind[i] == WALL_LINK)[0] for i in range(self.q)]

    # -- lattice functions ------------------------------------------------
    def feq(self, rho, u):
        """Equilibrium [q, n] for density rho [n] and velocity u [3, n]."""
        cu = self.lat.cf @ u
        usq = np.sum(u * u, axis=0)
        return self.lat.w[:, None] * rho[None, :] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq[None, :])

    def moments(self, f):
        rho = np.sum(f, axis=0)
        m = self.lat.cf.T @ f
        return rho, m, m / rho[None, :]

    def rest_state(self):
        return np.repeat(self.lat.w[:, None], self.n, axis=1)

    # -- one step ----------------------------------------------------------
    def stream(self, A, t):
        """Pre-collision populations f of the step that starts at time t."""
        lat, L = self.lat, self.links
        own = A if self.sites is None else A[:, self.sites]  # the sites' own stored populations
        f = np.empty((self.q, self.n))
        f[0] = own[0]
        u_own = None
        for i in range(1, self.q):
            fl = self._fluid[i]
            f[i, fl] = A[i, L.src[i, fl]]
            wl = self._wall[i]
            o = lat.opp[i]
            f[i, wl] = own[o, wl]
            if self.wall_q is not None:
                q = self.wall_q[i, wl]
                near = np.nonzero((q < 0.5) & (L.kind[o, wl] == FLUID_LINK))[0]
                far = np.nonzero(q >= 0.5)[0]
                qn, sn = q[near], wl[near]
                f[i, sn] = 2.0 * qn * own[o, sn] + (1.0 - 2.0 * qn) * A[o, L.src[o, sn]]
                qf, sf = q[far], wl[far]
                f[i, sf] = own[o, sf] / (2.0 * qf) + (2.0 * qf - 1.0) / (2.0 * qf) * own[i, sf]
            for k, sel in self._io[i]:
                io = self.iolets[k]
                if io.kind == "pressure":
                    if u_own is None:
                        u_own = self.moments(own)[2]
                    rho_k = io.value(t)
                    us = u_own[:, sel]
                    cu = lat.cf[i] @ us
                    usq = np.sum(us * us, axis=0)
                    f[i, sel] = lat.w[i] * rho_k * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
                elif io.kind == "velocity":
                    U = io.value(t)
                    ub = U * self.W[sel][None, :] * np.asarray(io.direction, dtype=np.float64)[:, None]
                    f[i, sel] = own[lat.opp[i], sel] + 2.0 * lat.w[i] * (lat.cf[i] @ ub) / _lattice.CS2
                else:
                    raise ValueError(io.kind)
        return f

    def collide(self, f):
        rho, _, u = self.moments(f)
        ub = u if self.alpha is None else u * (1.0 - self.alpha)[None, :]
        return f - self.omega * (f - self.feq(rho, ub))

    def step(self, A, t):
        f = self.stream(A, t)
        return self.collide(f), f

    def run(self, A, t0, nsteps):
        """Advance nsteps from state A at time t0.  Returns (A_end, f_pre_last);
        f_pre_last is None when nsteps == 0."""
        f = None
        for k in range(nsteps):
            A, f = self.step(A, t0 + k)
        return A, f

    # -- observables -------------------------------------------------------
    def wall_normals(self):
        n = np.zeros((3, self.n))
        for i in range(1, self.q):
            wl = self._wall[i]
            n[:, wl] += self.lat.cf[i][:, None]
        nn = np.sqrt(np.sum(n * n, axis=0))
        has = nn > 0
        n[:, has] /= nn[has]
        return n, has

    def observables(self, f):
        """(p [n], u [3, n], sigma [3, 3, n], wss [n]) from pre-collision f."""
        rho, _, u = self.moments(f)
        neq = f - self.feq(rho, u)
        c = self.lat.cf
        pi = np.einsum("ia,ib,in->abn", c, c, neq)
        k = 1.0 - 0.5 * self.omega
        sigma = -k * pi
        nrm, has = self.wall_normals()
        sn = np.einsum("abn,bn->an", sigma, nrm)
        nsn = np.sum(nrm * sn, axis=0)
        tvec = sn - nsn[None, :] * nrm
        wss = np.where(has, np.sqrt(np.sum(tvec * tvec, axis=0)), 0.0)
        return rho / 3.0, u, sigma, wss

    def totals(self, A):
        """Total mass and momentum of a stored state."""
        return float(np.sum(A)), (self.lat.cf.T @ A).sum(axis=1)
