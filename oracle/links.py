"""Upstream classification of every (site, direction) pair (oracle).

Pull streaming (Section 2: propagation along the lattice vectors between
fluid sites of the sparse lattice): the population f_i arriving at site x
comes from the upstream point y = x - c_i.  The point y is either

* another fluid site            -> FLUID, with its site index;
* a point past iolet plane k    -> IOLET, with k (label 2 + k);
* anything else (vessel wall)   -> WALL (simple bounce-back, Section 4).

Sites keep the order of ``geometry.coords``.  Fluid neighbours are found by
binary search over the sorted linear keys of the site coordinates.
"""

import numpy as np

FLUID_LINK, WALL_LINK, IOLET_LINK = 0, 1, 2


class Links:
    """Links of every site, or with ``sites`` (indices into geom.coords) of those
    sites only; ``src`` always indexes the full site list."""

    def __init__(self, geom, lat, sites=None):
        X, Y, Z = geom.shape
        all_coords = geom.coords.astype(np.int64)
        keys = (all_coords[:, 0] * Y + all_coords[:, 1]) * Z + all_coords[:, 2]
        order = np.argsort(keys, kind="stable")
        skeys = keys[order]
        if sites is None:
            coords = all_coords
        else:
            coords = all_coords[np.asarray(sites)]
        n = coords.shape[0]
        q = lat.q
        self.n, self.q = n, q
        self.kind = np.zeros((q, n), dtype=np.int8)
        self.src = np.full((q, n), -1, dtype=np.int64)
        self.iolet = np.full((q, n), -1, dtype=np.int64)
        self.src[0] = np.arange(n) if sites is None else np.asarray(sites)
        for i in range(1, q):
            up = coords - lat.c[i]
            for a in range(3):
                if geom.periodic[a]:
                    up[:, a] %= geom.shape[a]
            lab = geom.label_at(up)
            fl = lab == 1
            io = lab >= 2
            self.kind[i][~fl] = WALL_LINK
            self.kind[i][io] = IOLET_LINK
            self.iolet[i][io] = lab[io].astype(np.int64) - 2
            if np.any(fl):
                uk = (up[fl, 0] * Y + up[fl, 1]) * Z + up[fl, 2]
                pos = np.searchsorted(skeys, uk)
                assert np.all(skeys[pos] == uk), "fluid label without a site"
                self.src[i][fl] = order[pos]

    def codes(self):
        """Upstream codes [n, q]: >= 0 fluid site, -1 wall, -2-k iolet k.
        The rest direction (0) holds the site itself."""
        out = np.where(self.kind == FLUID_LINK, self.src,
                       np.where(self.kind == WALL_LINK, -1, -2 - self.iolet))
        out[0] = np.arange(self.n)
        return out.T.copy()
