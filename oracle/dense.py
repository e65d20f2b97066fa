"""Dense-box formulation of the same step (oracle cross-check).

The populations live on the whole box, F[i, x, y, z]; streaming shifts each
array by its lattice vector (padding a periodic axis by wrap-around, a
bounded axis by one layer), and the label of the upstream point is read from
the equally shifted label grid.  Non-fluid cells carry no meaning.  The
boundary rules and the collision are those of ``lbgk`` (see there), written
again on dense arrays so that the sparse neighbour lookup is checked by an
independent formulation.
"""

import math

import numpy as np

from . import lattice as _lattice


class DenseLBGK:
    def __init__(self, geom, q=15, tau=None, alpha=None):
        self.geom = geom
        self.lat = _lattice.get(q)
        self.q = self.lat.q
        self.tau = float(geom.tau if tau is None else tau)
        self.omega = 0.0 if math.isinf(self.tau) else 1.0 / self.tau
        X, Y, Z = geom.shape
        lab = geom.labels.copy()
        inner = lab[1:X + 1, 1:Y + 1, 1:Z + 1]
        # a periodic axis takes its padding from the opposite face
        for a, per in enumerate(geom.periodic):
            if per:
                lab = np.moveaxis(lab, a, 0)
                lab[0] = lab[-2]
                lab[-1] = lab[1]
                lab = np.moveaxis(lab, 0, a)
        self.lab = lab
        self.fluid = inner == 1
        self.alpha = None
        if alpha is not None:
            self.alpha = np.zeros(geom.shape)
            c = geom.coords
            self.alpha[c[:, 0], c[:, 1], c[:, 2]] = alpha
        self.W = np.zeros(geom.shape)
        c = geom.coords
        self.W[c[:, 0], c[:, 1], c[:, 2]] = geom.site_weight()
        self.upl = [self._shift_lab(i) for i in range(self.q)]

    def _shift_lab(self, i):
        X, Y, Z = self.geom.shape
        cx, cy, cz = self.lat.c[i]
        return self.lab[1 - cx:1 - cx + X, 1 - cy:1 - cy + Y, 1 - cz:1 - cz + Z]

    def _shift(self, arr, i):
        """out[x] = arr[x - c_i] (wrap on periodic axes; bounded axes read a
        zero layer, which the boundary rules overwrite)."""
        pads = []
        for a, per in enumerate(self.geom.periodic):
            pads.append(per)
        out = arr
        p = np.pad(out, 1, mode="constant")
        for a, per in enumerate(pads):
            if per:
                p = np.moveaxis(p, a, 0)
                p[0] = p[-2]
                p[-1] = p[1]
                p = np.moveaxis(p, 0, a)
        X, Y, Z = self.geom.shape
        cx, cy, cz = self.lat.c[i]
        return p[1 - cx:1 - cx + X, 1 - cy:1 - cy + Y, 1 - cz:1 - cz + Z]

    def to_dense(self, A):
        F = np.zeros((self.q,) + tuple(self.geom.shape))
        c = self.geom.coords
        F[:, c[:, 0], c[:, 1], c[:, 2]] = A
        return F

    def to_sites(self, F):
        c = self.geom.coords
        return F[:, c[:, 0], c[:, 1], c[:, 2]]

    def _feq(self, rho, u):
        out = np.empty((self.q,) + rho.shape)
        usq = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        for i in range(self.q):
            cu = self.lat.cf[i, 0] * u[0] + self.lat.cf[i, 1] * u[1] + self.lat.cf[i, 2] * u[2]
            out[i] = self.lat.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
        return out

    def _moments(self, F):
        rho = F.sum(axis=0)
        m = np.stack([np.tensordot(self.lat.cf[:, a], F, axes=(0, 0)) for a in range(3)])
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(self.fluid[None], m / np.where(rho == 0, 1.0, rho)[None], 0.0)
        return rho, m, u

    def step(self, F, t):
        lat = self.lat
        f = np.empty_like(F)
        f[0] = F[0]
        u_own = None
        for i in range(1, self.q):
            up = self.upl[i]
            fi = self._shift(F[i], i)
            wall = up == 0
            fi = np.where(wall, F[lat.opp[i]], fi)
            for k, io in enumerate(self.geom.iolets):
                sel = up == 2 + k
                if not np.any(sel & self.fluid):
                    continue
                if io.kind == "pressure":
                    if u_own is None:
                        u_own = self._moments(F)[2]
                    rho_k = io.value(t)
                    cu = lat.cf[i, 0] * u_own[0] + lat.cf[i, 1] * u_own[1] + lat.cf[i, 2] * u_own[2]
                    usq = u_own[0] ** 2 + u_own[1] ** 2 + u_own[2] ** 2
                    g = lat.w[i] * rho_k * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq)
                else:
                    U = io.value(t)
                    e = np.asarray(io.direction, dtype=np.float64)
                    g = F[lat.opp[i]] + 2.0 * lat.w[i] * U * self.W * float(lat.cf[i] @ e) / _lattice.CS2
                fi = np.where(sel, g, fi)
            f[i] = np.where(self.fluid, fi, 0.0)
        rho, _, u = self._moments(f)
        ub = u if self.alpha is None else u * (1.0 - self.alpha)[None]
        with np.errstate(invalid="ignore"):
            Fn = f - self.omega * (f - self._feq(rho, ub))
        return np.where(self.fluid[None], Fn, 0.0), f
