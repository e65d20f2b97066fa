"""Synthetic vessel geometries as padded voxel label grids.

A geometry is a box of candidate lattice sites with integer coordinates
0 <= x < X, 0 <= y < Y, 0 <= z < Z.  ``labels`` has shape (X+2, Y+2, Z+2): one
layer of padding on every side, ``labels[x+1, y+1, z+1]`` being the label of
point (x, y, z).  Labels:

* ``SOLID`` (0): outside the vessel;
* ``FLUID`` (1): a fluid site of the sparse lattice (only inside the box);
* ``2 + k``: outside the fluid domain but inside the extension of the lumen
  past iolet ``k`` (inlet or outlet plane).  A link whose upstream point has
  this label crosses iolet ``k``; any other non-fluid upstream point is a wall.

Along a periodic axis the padding is unused and coordinates wrap.

The paper's experiments use patient vessels, a D3Q19 lattice and simple
bounce-back walls (Section 4); the patient data is not reproduced.  The
shapes below stand in for it: a straight pipe, a saccular aneurysm on a
half-circle arc, and seeded bifurcating trees that follow Murray's law.
"""

from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SOLID = 0
FLUID = 1


@dataclass(frozen=True)
class Iolet:
    """An inlet/outlet boundary.

    kind: ``"pressure"`` (density imposed) or ``"velocity"`` (velocity imposed
    by moving-wall bounce-back).
    direction: unit vector of the imposed velocity (the inward normal of an
    inlet, or the tangential direction of a moving wall); unused for pressure.
    The imposed scalar (density or speed) at time t is
    ``mean + sum_h cos[h-1]*cos(2 pi h t/period) + sin[h-1]*sin(2 pi h t/period)``.
    """

    kind: str
    direction: tuple = (0.0, 0.0, 0.0)
    mean: float = 1.0
    cos: tuple = ()
    sin: tuple = ()
    period: float = 1.0

    def value(self, t: float) -> float:
        v = float(self.mean)
        for h, (a, b) in enumerate(zip(self.cos, self.sin), start=1):
            ph = 2.0 * math.pi * h * t / self.period
            v += a * math.cos(ph) + b * math.sin(ph)
        return v


@dataclass
class Geometry:
    name: str
    shape: tuple
    labels: np.ndarray
    periodic: tuple = (False, False, False)
    iolets: list = field(default_factory=list)
    tau: float = 0.6
    # inlet velocity profile: (point on axis, unit axis, radius); None -> weight 1
    profile: tuple | None = None
    info: dict = field(default_factory=dict)
    # continuous fluid predicate on float points [M, 3] (the one the labels sample
    # at integer points); None for geometries without a curved wall description
    inside: object = field(default=None, repr=False)

    _coords: np.ndarray | None = field(default=None, repr=False)

    @property
    def coords(self) -> np.ndarray:
        """Fluid sites, int32 [N, 3], lexicographic (x slowest, z fastest)."""
        if self._coords is None:
            X, Y, Z = self.shape
            inner = self.labels[1:X + 1, 1:Y + 1, 1:Z + 1]
            self._coords = np.argwhere(inner == FLUID).astype(np.int32)
        return self._coords

    @property
    def n_sites(self) -> int:
        return int(self.coords.shape[0])

    def site_weight(self) -> np.ndarray:
        """Per-site inlet profile weight W_s = max(0, 1 - r^2/R^2), float64 [N].

        r is the distance of the site from the inlet axis, R the inlet radius.
        Without a profile every weight is 1 (plug flow / moving wall).
        """
        c = self.coords.astype(np.float64)
        if self.profile is None:
            return np.ones(c.shape[0])
        p0, ax, R = self.profile
        v = c - np.asarray(p0, dtype=np.float64)
        a = np.asarray(ax, dtype=np.float64)
        t = v @ a
        r2 = np.einsum("ij,ij->i", v, v) - t * t
        return np.maximum(0.0, 1.0 - r2 / (R * R))

    def wall_fractions(self, dirs, iters=40):
        """Wall position along every wall link, float64 [N, len(dirs)] (NaN where the
        link is not a wall link): for fluid site x and lattice vector c (dirs[i])
        whose point x - c is solid, the fraction q in (0, 1] of the segment from
        x towards x - c at which the continuous wall crosses it (bisection of
        ``inside``).  Interpolated (BFL) walls use it."""
        if self.inside is None:
            raise ValueError(f"{self.name} has no continuous wall description")
        c = self.coords.astype(np.int64)
        dirs = np.asarray(dirs, dtype=np.int64)
        out = np.full((c.shape[0], len(dirs)), np.nan)
        for i, d in enumerate(dirs):
            if not d.any():
                continue
            up = c - d
            lab = self.label_at(up)
            wall = np.nonzero(lab == SOLID)[0]
            if len(wall) == 0:
                continue
            x0 = c[wall].astype(np.float64)
            step = -d.astype(np.float64)
            lo = np.zeros(len(wall))
            hi = np.ones(len(wall))
            for _ in range(iters):
                mid = 0.5 * (lo + hi)
                ins = self.inside(x0 + mid[:, None] * step[None, :])
                lo = np.where(ins, mid, lo)
                hi = np.where(ins, hi, mid)
            out[wall, i] = 0.5 * (lo + hi)
        return out

    def label_at(self, pts: np.ndarray) -> np.ndarray:
        """Labels of integer points [M, 3]; periodic axes wrap, others must lie
        within one layer of the box."""
        p = np.asarray(pts, dtype=np.int64).copy()
        for a in range(3):
            if self.periodic[a]:
                p[:, a] %= self.shape[a]
        return self.labels[p[:, 0] + 1, p[:, 1] + 1, p[:, 2] + 1]


def _empty(shape):
    X, Y, Z = shape
    return np.zeros((X + 2, Y + 2, Z + 2), dtype=np.uint8)


def _grid_points(lo, hi):
    """Integer points of the box lo..hi (inclusive), as float64 component arrays."""
    xs = np.arange(lo[0], hi[0] + 1)
    ys = np.arange(lo[1], hi[1] + 1)
    zs = np.arange(lo[2], hi[2] + 1)
    return np.meshgrid(xs, ys, zs, indexing="ij")


def _in_box(shape, x, y, z):
    X, Y, Z = shape
    return (x >= 0) & (x < X) & (y >= 0) & (y < Y) & (z >= 0) & (z < Z)


# ----------------------------------------------------------------------------
# straight pipe with pressure iolets
# ----------------------------------------------------------------------------

def pipe(X=20, Y=20, Z=64, r2=64.0, rho_in=1.001, rho_out=1.0, tau=0.8, inlet_velocity=None):
    """Straight circular pipe along z: fluid iff (x-cx)^2+(y-cy)^2 < r2, 0<=z<Z.

    Iolet 0 (inlet) lies beyond z = 0, iolet 1 (outlet) beyond z = Z-1, both
    pressure (equilibrium) iolets.  The default is the 20x20x64 pipe with
    radius 8 and 208 sites per cross-section (13,312 sites).  With
    ``inlet_velocity=(mean, cos, sin, period)`` the inlet is instead a Ladd
    velocity iolet along +z with a parabolic profile.
    """
    shape = (X, Y, Z)
    lab = _empty(shape)
    cx, cy = (X - 1) / 2.0, (Y - 1) / 2.0
    x, y, z = _grid_points((-1, -1, -1), (X, Y, Z))
    disc = (x - cx) ** 2 + (y - cy) ** 2 < r2
    inb = _in_box(shape, x, y, z)
    lab[(disc & inb)] = FLUID
    lab[(disc & (z < 0))] = 2
    lab[(disc & (z >= Z))] = 3
    iolets = [Iolet("pressure", mean=rho_in), Iolet("pressure", mean=rho_out)]
    profile = None
    if inlet_velocity is not None:
        mean, cos, sin, period = inlet_velocity
        iolets[0] = Iolet("velocity", direction=(0.0, 0.0, 1.0), mean=mean, cos=tuple(cos),
                          sin=tuple(sin), period=period)
        profile = ((cx, cy, 0.0), (0.0, 0.0, 1.0), float(np.sqrt(r2)))
    def inside(p):
        return (p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2 < r2

    return Geometry("pipe", shape, lab, iolets=iolets, tau=tau, profile=profile,
                    info=dict(r2=r2, rho_in=rho_in, rho_out=rho_out), inside=inside)


# ----------------------------------------------------------------------------
# saccular aneurysm on a half-circle arc
# ----------------------------------------------------------------------------

def aneurysm(half=False, tau=0.6, u_mean=0.02, u_amp=0.01, period=4000.0):
    """Tube of radius r around a half-circle arc of radius R (plane z = zc, half
    y >= y0), plus a spherical dome bulging off the outer wall at mid-arc.

    Full size: box 384x384x192, arc centre (191.5, 112, 95.5), R = 160, r = 24,
    dome radius 56 centred 212 beyond the arc centre along +y (about 1.59M
    sites).  ``half=True`` halves every length (box 192x192x96, about 199k
    sites).  The lumen continues straight along -y past both arc ends; the
    plane y = y0 carries a velocity inlet (end at small x, inward normal +y,
    parabolic profile, pulsatile u(t) = u_mean + u_amp sin(2 pi t/period)) and
    a pressure outlet rho = 1 (end at large x).
    """
    s = 0.5 if half else 1.0
    X, Y, Z = int(384 * s), int(384 * s), int(192 * s)
    shape = (X, Y, Z)
    cx, y0, zc = (X - 1) / 2.0, 112.0 * s, (Z - 1) / 2.0
    R, r = 160.0 * s, 24.0 * s
    sc = np.array([cx, y0 + 212.0 * s, zc])
    rs = 56.0 * s
    lab = _empty(shape)
    zs = np.arange(-1, Z + 1, dtype=np.float64)
    ys = np.arange(-1, Y + 1, dtype=np.float64)
    for xi in range(-1, X + 1):
        x = float(xi)
        y, z = np.meshgrid(ys, zs, indexing="ij")
        rho_xy = np.sqrt((x - cx) ** 2 + (y - y0) ** 2)
        tube = ((rho_xy - R) ** 2 + (z - zc) ** 2 < r * r) & (y >= y0)
        dome = (x - sc[0]) ** 2 + (y - sc[1]) ** 2 + (z - sc[2]) ** 2 < rs * rs
        inb = (xi >= 0) & (xi < X) & (y >= 0) & (y < Y) & (z >= 0) & (z < Z)
        fluid = (tube | dome) & inb
        ext_in = (y < y0) & ((x - (cx - R)) ** 2 + (z - zc) ** 2 < r * r)
        ext_out = (y < y0) & ((x - (cx + R)) ** 2 + (z - zc) ** 2 < r * r)
        plane = np.zeros(y.shape, dtype=np.uint8)
        plane[ext_in] = 2
        plane[ext_out] = 3
        plane[fluid] = FLUID
        lab[xi + 1] = plane
    iolets = [
        Iolet("velocity", direction=(0.0, 1.0, 0.0), mean=u_mean, cos=(0.0,), sin=(u_amp,),
              period=period),
        Iolet("pressure", mean=1.0),
    ]
    profile = ((cx - R, y0, zc), (0.0, 1.0, 0.0), r)
    dome_info = dict(centre=tuple(sc), radius=rs, arc_centre=(cx, y0, zc), R=R, r=r)

    def inside(p):
        rho = np.sqrt((p[:, 0] - cx) ** 2 + (p[:, 1] - y0) ** 2)
        tube = ((rho - R) ** 2 + (p[:, 2] - zc) ** 2 < r * r) & (p[:, 1] >= y0)
        dome = ((p[:, 0] - sc[0]) ** 2 + (p[:, 1] - sc[1]) ** 2 + (p[:, 2] - sc[2]) ** 2) < rs * rs
        return tube | dome

    return Geometry("aneurysm_half" if half else "aneurysm", shape, lab, iolets=iolets,
                    tau=tau, profile=profile, info=dome_info, inside=inside)


# ----------------------------------------------------------------------------
# seeded bifurcating tree (Murray's law)
# ----------------------------------------------------------------------------

def _frame(d):
    ref = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(d, ref)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return e1, e2


def tree_segments(r0, root, generations, seed):
    """Segments of a seeded Murray tree, breadth-first.

    Each segment: dict(a=start, d=unit axis, L=length, r=radius, level,
    open_start, open_end).  At each bifurcation (breadth-first) draw
    k ~ U[0.6, 1], theta_a, theta_b ~ U[25, 45] degrees, phi ~ U[0, 2 pi);
    r_a = r / (1 + k^3)^(1/3), r_b = k r_a (so r^3 = r_a^3 + r_b^3); child a
    leaves at azimuth phi, child b at phi + pi; each child is 8 of its radii
    long.
    """
    rng = np.random.default_rng(seed)
    root_seg = dict(a=np.asarray(root, dtype=np.float64), d=np.array([0.0, 0.0, 1.0]),
                    L=8.0 * r0, r=float(r0), level=0, open_start=True,
                    open_end=(generations == 0))
    segs = [root_seg]
    frontier = [root_seg]
    for level in range(1, generations + 1):
        nxt = []
        for p in frontier:
            k = rng.uniform(0.6, 1.0)
            th_a = math.radians(rng.uniform(25.0, 45.0))
            th_b = math.radians(rng.uniform(25.0, 45.0))
            phi = rng.uniform(0.0, 2.0 * math.pi)
            ra = p["r"] / (1.0 + k ** 3) ** (1.0 / 3.0)
            rb = k * ra
            e1, e2 = _frame(p["d"])
            start = p["a"] + p["L"] * p["d"]
            for rc, th, az in ((ra, th_a, phi), (rb, th_b, phi + math.pi)):
                dc = math.cos(th) * p["d"] + math.sin(th) * (math.cos(az) * e1 + math.sin(az) * e2)
                dc /= np.linalg.norm(dc)
                c = dict(a=start.copy(), d=dc, L=8.0 * rc, r=rc, level=level,
                         open_start=False, open_end=(level == generations))
                segs.append(c)
                nxt.append(c)
        frontier = nxt
    return segs


def _raster_segment(lab, shape, seg, pass_):
    """Rasterise one segment into the padded label grid.

    pass_ 0: fluid (inside the box) and box-crossing lumen (outlet label);
    pass_ 1: inlet/outlet slabs past open ends, only where still SOLID.
    """
    X, Y, Z = shape
    a, d, L, r = seg["a"], seg["d"], seg["L"], seg["r"]
    b = a + L * d
    m = r + 3.0
    lo = np.floor(np.minimum(a, b) - m).astype(np.int64)
    hi = np.ceil(np.maximum(a, b) + m).astype(np.int64)
    lo = np.maximum(lo, -1)
    hi = np.minimum(hi, np.array([X, Y, Z]))
    if np.any(hi < lo):
        return
    # chunk along x to bound memory
    for x0 in range(lo[0], hi[0] + 1, 64):
        x1 = min(hi[0], x0 + 63)
        x, y, z = _grid_points((x0, lo[1], lo[2]), (x1, hi[1], hi[2]))
        vx, vy, vz = x - a[0], y - a[1], z - a[2]
        t = vx * d[0] + vy * d[1] + vz * d[2]
        rad2 = vx * vx + vy * vy + vz * vz - t * t
        r2 = r * r
        if pass_ == 0:
            fl = (t >= 0.0) & (t <= L) & (rad2 < r2)
            if not seg["open_start"]:
                fl |= (vx * vx + vy * vy + vz * vz) < r2
            if not seg["open_end"]:
                fl |= ((x - b[0]) ** 2 + (y - b[1]) ** 2 + (z - b[2]) ** 2) < r2
            inb = _in_box(shape, x, y, z)
            sub = lab[x0 + 1:x1 + 2, lo[1] + 1:hi[1] + 2, lo[2] + 1:hi[2] + 2]
            sub[fl & inb] = FLUID
            sub[fl & ~inb] = 3
        else:
            sl = np.zeros(x.shape, dtype=np.uint8)
            if seg["open_start"]:
                sl[(t >= -2.0) & (t < 0.0) & (rad2 < r * r)] = 2
            if seg["open_end"]:
                sl[(t > L) & (t <= L + 2.0) & (rad2 < r * r)] = 3
            sub = lab[x0 + 1:x1 + 2, lo[1] + 1:hi[1] + 2, lo[2] + 1:hi[2] + 2]
            put = (sl != 0) & (sub == SOLID)
            sub[put] = sl[put]


def tree(box=1024, r0=32.0, root=(512.0, 512.0, 16.0), generations=7, seed=3, tau=0.6,
         u_mean=0.02, name=None):
    """Seeded Murray tree in a cubic box.

    The root starts at ``root`` along +z with an open start carrying a
    velocity inlet (parabolic, constant u_mean).  Inner segments are capsules
    (cylinder plus end spheres); terminal segments are open at their far end,
    where the lumen continues into a pressure outlet rho = 1.  Lumen that
    leaves the box also counts as that outlet.
    """
    shape = (box, box, box)
    lab = _empty(shape)
    segs = tree_segments(r0, root, generations, seed)
    for sg in segs:
        _raster_segment(lab, shape, sg, 0)
    for sg in segs:
        _raster_segment(lab, shape, sg, 1)
    iolets = [
        Iolet("velocity", direction=(0.0, 0.0, 1.0), mean=u_mean),
        Iolet("pressure", mean=1.0),
    ]
    profile = (tuple(root), (0.0, 0.0, 1.0), float(r0))
    return Geometry(name or f"tree{box}", shape, lab, iolets=iolets, tau=tau, profile=profile,
                    info=dict(segments=len(segs), seed=seed, r0=r0, generations=generations))


# ----------------------------------------------------------------------------
# small analytic test geometries
# ----------------------------------------------------------------------------

def couette(H=8, Lx=4, Lz=4, U=0.01, tau=0.8, wall_gap=0.5):
    """Plane Couette cell: periodic in x and z, fluid 0 <= y < H.  A resting
    wall lies beyond y = 0, at y = -wall_gap (the continuous wall used by
    interpolated walls; halfway bounce-back places it at -1/2), a wall moving
    with velocity (U,0,0) beyond y = H-1 (velocity iolet 0, direction +x,
    weight 1)."""
    shape = (Lx, H, Lz)
    lab = _empty(shape)
    lab[:, 1:H + 1, :] = FLUID
    lab[:, H + 1, :] = 2

    def inside(p):
        return p[:, 1] > -wall_gap

    return Geometry("couette", shape, lab, periodic=(True, False, True),
                    iolets=[Iolet("velocity", direction=(1.0, 0.0, 0.0), mean=U)], tau=tau,
                    info=dict(H=H, U=U, wall_gap=wall_gap), inside=inside)


def channel(H=8, L=48, Lx=4, rho_in=1.001, rho_out=1.0, tau=0.6):
    """Plane channel: periodic in x, walls beyond y = 0 and y = H-1, pressure
    inlet beyond z = 0 (iolet 0) and pressure outlet beyond z = L-1 (iolet 1)."""
    shape = (Lx, H, L)
    lab = _empty(shape)
    lab[:, 1:H + 1, 1:L + 1] = FLUID
    lab[:, 1:H + 1, 0] = 2
    lab[:, 1:H + 1, L + 1] = 3
    def inside(p):
        return (p[:, 1] > -0.5) & (p[:, 1] < H - 0.5)

    return Geometry("channel", shape, lab, periodic=(True, False, False),
                    iolets=[Iolet("pressure", mean=rho_in), Iolet("pressure", mean=rho_out)],
                    tau=tau, info=dict(H=H, L=L), inside=inside)


def duct(X=3, Y=4, L=10, rho_in=1.0, rho_out=1.0, tau=0.7):
    """Box periodic in x and y, fluid 0 <= z < L, with a pressure iolet beyond
    z = 0 (iolet 0) and one beyond z = L-1 (iolet 1); no walls."""
    shape = (X, Y, L)
    lab = _empty(shape)
    lab[1:X + 1, 1:Y + 1, 1:L + 1] = FLUID
    lab[1:X + 1, 1:Y + 1, 0] = 2
    lab[1:X + 1, 1:Y + 1, L + 1] = 3
    return Geometry("duct", shape, lab, periodic=(True, True, False),
                    iolets=[Iolet("pressure", mean=rho_in), Iolet("pressure", mean=rho_out)],
                    tau=tau, info=dict(L=L))


def closed_box(X=6, Y=5, Z=7, tau=0.7):
    """All sites of the box are fluid, surrounded by resting walls."""
    shape = (X, Y, Z)
    lab = _empty(shape)
    lab[1:X + 1, 1:Y + 1, 1:Z + 1] = FLUID
    return Geometry("closed_box", shape, lab, tau=tau)


def periodic_box(X=6, Y=5, Z=7, tau=0.7):
    """Fully periodic box: no walls, no iolets."""
    shape = (X, Y, Z)
    lab = _empty(shape)
    lab[1:X + 1, 1:Y + 1, 1:Z + 1] = FLUID
    return Geometry("periodic_box", shape, lab, periodic=(True, True, True), tau=tau)


def config_geometry(name: str) -> Geometry:
    """The named workloads: pipe (13,312 sites), aneurysm (~1.6M), tree1024
    (Murray tree, root radius 32, 7 generations, seed 3), aneurysm_half (~200k),
    tree2048 (root radius 64, 8 generations, seed 5).

    Size-matched variants of the two trees keep the box, seed and branching rules
    and raise only the root radius until the site count reaches the stated ~30M and
    ~400M (branches clipped at the box faces make the count grow more slowly than
    r^3): tree1024_30M (radius 96, 30,090,542 sites) and tree2048_400M (radius 256,
    395,245,440 sites).  As in the originals the root starts half a radius above
    the bottom face."""
    if name == "pipe":
        return pipe()
    if name == "aneurysm":
        return aneurysm(half=False)
    if name == "aneurysm_half":
        return aneurysm(half=True)
    if name == "tree1024":
        return tree(1024, 32.0, (512.0, 512.0, 16.0), 7, seed=3, name="tree1024")
    if name == "tree2048":
        return tree(2048, 64.0, (1024.0, 1024.0, 32.0), 8, seed=5, name="tree2048")
    if name == "tree1024_30M":
        return tree(1024, 96.0, (512.0, 512.0, 48.0), 7, seed=3, name="tree1024_30M")
    if name == "tree2048_400M":
        return tree(2048, 256.0, (1024.0, 1024.0, 128.0), 8, seed=5, name="tree2048_400M")
    raise ValueError(f"unknown workload {name!r}")
