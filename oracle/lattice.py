"""Lattice velocity sets (oracle).

D3Q19 is the lattice the paper uses (Section 2, Figure 1; Section 4).  D3Q15
is the second lattice of the workloads.  Ordering convention shared by the
interface: index 0 is the rest vector, then opposite pairs (2k-1, 2k).

D3Q15: rest (2/9), 6 face neighbours (1/9), 8 cube corners (1/72).
D3Q19: rest (1/3), 6 face neighbours (1/18), 12 edge neighbours (1/36).
Speed of sound squared: 1/3 for both.
"""

from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0


def _pairs(vecs):
    out = [(0, 0, 0)]
    for v in vecs:
        out.append(v)
        out.append(tuple(-a for a in v))
    return out


_FACES = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
_CORNERS = [(1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1)]
_EDGES = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]


class Lattice:
    def __init__(self, name, vecs, weights_exact):
        self.name = name
        self.c = np.array(vecs, dtype=np.int64)
        self.q = len(vecs)
        self.w_exact = list(weights_exact)
        self.w = np.array([float(x) for x in weights_exact])
        self.opp = np.array([self._find(tuple(-a for a in v)) for v in vecs])
        self.cf = self.c.astype(np.float64)

    def _find(self, v):
        for j, u in enumerate(self.c.tolist()):
            if tuple(u) == tuple(v):
                return j
        raise KeyError(v)


def _weights(vecs, by_norm):
    return [by_norm[sum(a * a for a in v)] for v in vecs]


def d3q15():
    vecs = _pairs(_FACES + _CORNERS)
    return Lattice("D3Q15", vecs,
                   _weights(vecs, {0: Fraction(2, 9), 1: Fraction(1, 9), 3: Fraction(1, 72)}))


def d3q19():
    vecs = _pairs(_FACES + _EDGES)
    return Lattice("D3Q19", vecs,
                   _weights(vecs, {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}))


def get(q):
    if q in (15, "D3Q15"):
        return d3q15()
    if q in (19, "D3Q19"):
        return d3q19()
    raise ValueError(q)
