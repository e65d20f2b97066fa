"""Discrete adjoint of the sparse LBGK step and of a flux + wall-shear objective (oracle).

Objective over a window W of steps (step t maps A_t to A_{t+1}, with
pre-collision populations f_t):

    J = sum_{t in W} (Q(t) - Q*)^2 + lam * mean_{t in W} mean_{s in D} WSS_s(f_t)

where Q(t) = sum over the links (s, i) of the outlet iolet of A_t[opp(i), s] - f_t[i, s]
(the mass leaving through the outlet during step t) and D is a set of wall
sites (the aneurysm dome).  Parameters: the Fourier coefficients (mean, cos_h,
sin_h) of every velocity iolet and the per-site Brinkman field alpha.

The adjoint is the exact reverse-mode derivative of the step as ``lbgk``
defines it, written out by hand, operator by operator, in the reverse order
of the forward:

* collision transpose: with g = dJ/dA_{t+1},
  dJ/df_j = (1 - omega) g_j + omega (a + c_j . b), a = sum_i g_i dfeq_i/drho,
  b = sum_i g_i dfeq_i/dm (at fixed momentum m = rho u, Brinkman velocity
  u_b = (1 - alpha) m / rho), and dJ/dalpha_s = sum_i g_i dA'_i/dalpha_s;
* objective terms at the pre-collision populations (wall shear stress) and at
  A_t (outlet flux);
* streaming transpose: every pulled value sends its adjoint back to where it
  was read (upstream site, own opposite population for walls and Ladd links),
  the Ladd term's adjoint goes to the Fourier coefficients, and the pressure
  iolet's equilibrium sends its adjoint to the site's own stored populations
  through the velocity u(A_t[:, s]).
"""

import numpy as np

from . import lattice as _lattice
from .links import FLUID_LINK, WALL_LINK, IOLET_LINK


class Objective:
    """outlet: iolet id of the flux term; q_target: Q*; dome: bool mask [n] of the
    sites whose wall shear stress enters; lam: weight; window: (t0, t1), the
    steps t0 <= t < t1 that contribute."""

    def __init__(self, outlet, q_target, dome, lam, window):
        self.outlet = int(outlet)
        self.q_target = float(q_target)
        self.dome = np.asarray(dome, dtype=bool)
        self.lam = float(lam)
        self.window = (int(window[0]), int(window[1]))

    def in_window(self, t):
        return self.window[0] <= t < self.window[1]


def iolet_basis(io, t):
    """d value(t) / d(mean, cos_1..H, sin_1..H)."""
    H = len(io.cos)
    out = np.empty(1 + 2 * H)
    out[0] = 1.0
    for h in range(1, H + 1):
        ph = 2.0 * np.pi * h * t / io.period
        out[h] = np.cos(ph)
        out[H + h] = np.sin(ph)
    return out


class Adjoint:
    def __init__(self, o, obj):
        self.o = o
        self.obj = obj
        L = o.links
        out = (L.kind == IOLET_LINK) & (L.iolet == obj.outlet)
        self.out_links = [(i, np.nonzero(out[i])[0]) for i in range(o.q)]
        self.nrm, self.has_n = o.wall_normals()
        self.dome_idx = np.nonzero(obj.dome & self.has_n)[0]
        W = obj.window[1] - obj.window[0]
        self.wss_w = obj.lam / (max(W, 1) * max(len(self.dome_idx), 1))

    # -- objective --------------------------------------------------------------
    def flux(self, A, f):
        q = 0.0
        for i, sel in self.out_links:
            if len(sel):
                q += np.sum(A[self.o.lat.opp[i], sel]) - np.sum(f[i, sel])
        return q

    def wss(self, f):
        return self.o.observables(f)[3]

    def forward(self, A0, T):
        """Run T steps from A0 at t = 0; returns (J, tape of A_0..A_T, Q per window step)."""
        o, obj = self.o, self.obj
        tape = [A0]
        A = A0
        J = 0.0
        qs = []
        for t in range(T):
            f = o.stream(A, t)
            if obj.in_window(t):
                q = self.flux(A, f)
                qs.append(q)
                J += (q - obj.q_target) ** 2
                J += self.wss_w * np.sum(self.wss(f)[self.dome_idx])
            A = o.collide(f)
            tape.append(A)
        return J, tape, np.array(qs)

    # -- transposed operators ---------------------------------------------------
    def collide_T(self, f, g):
        """(dJ/df, dJ/dalpha) from g = dJ/dA' for A' = collide(f)."""
        o = self.o
        lat = o.lat
        c = lat.cf
        w = lat.w[:, None]
        om = o.omega
        rho, m, u = o.moments(f)
        keep = np.ones(o.n) if o.alpha is None else 1.0 - o.alpha
        ub = u * keep[None, :]
        cub = c @ ub
        ub2 = np.sum(ub * ub, axis=0)
        dfeq_drho = w * (1.0 - 4.5 * cub * cub + 1.5 * ub2[None, :])
        wg = w * g
        b = keep[None, :] * (3.0 * (c.T @ wg) + 9.0 * (c.T @ (wg * cub)) - 3.0 * ub * wg.sum(axis=0)[None, :])
        a = np.sum(g * dfeq_drho, axis=0)
        fhat = (1.0 - om) * g + om * (a[None, :] + c @ b)
        cu = c @ u
        ubu = np.sum(ub * u, axis=0)
        dA_dalpha = -om * w * rho[None, :] * (3.0 * cu + 9.0 * cub * cu - 3.0 * ubu[None, :])
        return fhat, np.sum(g * dA_dalpha, axis=0)

    def wss_grad(self, f):
        """d WSS_s / d f_j at the dome sites: -(1 - omega/2) (t.(c_j-u)) (n.(c_j-u)),
        t the unit shear direction (zero where the shear vanishes)."""
        o = self.o
        idx = self.dome_idx
        fd = f[:, idx]
        rho, _, u = o.moments(fd)
        neq = fd - o.feq(rho, u)
        c = o.lat.cf
        sigma = -(1.0 - 0.5 * o.omega) * np.einsum("ia,ib,in->abn", c, c, neq)
        n = self.nrm[:, idx]
        sn = np.einsum("abn,bn->an", sigma, n)
        tv = sn - np.sum(n * sn, axis=0)[None, :] * n
        tn = np.sqrt(np.sum(tv * tv, axis=0))
        th = np.where(tn > 0, tv / np.where(tn > 0, tn, 1.0), 0.0)
        cmu = c[:, :, None] - u[None, :, :]          # [q, 3, m]
        return -(1.0 - 0.5 * o.omega) * np.einsum("an,ian->in", th, cmu) * np.einsum("an,ian->in", n, cmu)

    def stream_T(self, fhat, A, t, theta):
        """dJ/dA_t from dJ/df_t; adds the Fourier-coefficient adjoints to theta."""
        o = self.o
        lat, L = o.lat, o.links
        Ahat = np.zeros_like(A)
        Ahat[0] += fhat[0]
        u_own = rho_own = None
        for i in range(1, o.q):
            fl = o._fluid[i]
            Ahat[i, L.src[i, fl]] += fhat[i, fl]
            wl = o._wall[i]
            Ahat[lat.opp[i], wl] += fhat[i, wl]
            for k, sel in o._io[i]:
                io = o.iolets[k]
                if io.kind == "velocity":
                    Ahat[lat.opp[i], sel] += fhat[i, sel]
                    e = np.asarray(io.direction, dtype=np.float64)
                    coef = 2.0 * lat.w[i] * float(lat.cf[i] @ e) / _lattice.CS2
                    theta[k] += np.sum(fhat[i, sel] * coef * o.W[sel]) * iolet_basis(io, t)
                else:
                    if u_own is None:
                        rho_own, _, u_own = o.moments(A)
                    us = u_own[:, sel]
                    ci = lat.cf[i][:, None]
                    gu = lat.w[i] * io.value(t) * (3.0 * ci + 9.0 * (lat.cf[i] @ us)[None, :] * ci - 3.0 * us)
                    # d u / d A_j = (c_j - u) / rho
                    Ahat[:, sel] += fhat[i, sel][None, :] * ((lat.cf @ gu) - np.sum(us * gu, axis=0)[None, :]) / rho_own[sel][None, :]
        return Ahat

    def backward(self, tape, T, g_final=None):
        """Reverse sweep over steps T-1..0.  Returns (dJ/dtheta per velocity
        iolet {k: array}, dJ/dalpha [n], dJ/dA_0)."""
        o, obj = self.o, self.obj
        theta = {k: np.zeros(1 + 2 * len(io.cos)) for k, io in enumerate(o.iolets)
                 if io.kind == "velocity"}
        alpha_hat = np.zeros(o.n)
        g = np.zeros_like(tape[0]) if g_final is None else g_final.copy()
        for t in range(T - 1, -1, -1):
            A = tape[t]
            f = o.stream(A, t)
            fhat, ah = self.collide_T(f, g)
            alpha_hat += ah
            direct = None
            if obj.in_window(t):
                qbar = 2.0 * (self.flux(A, f) - obj.q_target)
                for i, sel in self.out_links:
                    if len(sel):
                        fhat[i, sel] -= qbar
                direct = qbar
                fhat[:, self.dome_idx] += self.wss_w * self.wss_grad(f)
            g = self.stream_T(fhat, A, t, theta)
            if direct is not None:
                for i, sel in self.out_links:
                    if len(sel):
                        g[o.lat.opp[i], sel] += direct
        return theta, alpha_hat, g
