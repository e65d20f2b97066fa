"""Direct volume rendering of a lattice property by ray marching (oracle).

Section 3.C.2: the visualization keeps the voxels of a lattice property (the
"lattice properties computed and cached" of the simulation) in a 3D texture and
renders them with a ray-marching direct volume rendering kernel; the viewing
parameters (zoom, rotation) and a transfer-function look-up table with a
steerable scale and offset are the user's controls.  The paper gives no
formulas; this is the textbook emission-absorption ray marcher (front-to-back
"over" compositing) with the readings below, which the GPU renderer follows.

* Volume: the fluid sites; site s holds value v_s at integer coordinates x_s
  (voxel centres).  Every other point of space is empty (contributes nothing).
* Rays: fixed-point integer vectors, F = 2^20 units per lattice spacing.  Ray
  (i, j) starts at P0 = O + i R + j U and has direction D_ij = D + i DR + j DU;
  its samples are P_k = P0 + k D_ij for k = 0 .. K - 1 (DR = DU = 0: an
  orthographic view; R = U = 0: a pinhole view from the eye O).
* Sampling, nearest voxel: x = floor((P_k + F/2) / F) on each axis.
* Sampling, trilinear (the filtering of a 3D texture): base voxel b = floor(P_k / F)
  and 8-bit fraction a = floor((P_k - b F) / 2^12) in [0, 255] on each axis (the
  weight precision of texture filtering units).  Corner c in {0, 1}^3 has weight
  W_c = prod over axes of (a if c = 1 else 256 - a), an integer; the weights sum
  to 2^24.  Empty voxels hold 0, as in a texture cleared to zero.  The value is
  (sum over c = 0..7, x fastest, of W_c v(b + c)) / 2^24 with the sum in FP64 in
  that order, then rounded to FP32: every product is exact (a 24-bit integer
  times an FP32 value), so the value does not depend on how the products are
  formed.  A corner of zero weight is not read.  A sample contributes only if a
  corner of non-zero weight is a site (so at a voxel centre it is exactly the
  nearest-voxel sample).
* Transfer: t = (v - offset) * scale in FP32; table entry e = floor(256 t)
  clamped to [0, 255] (0 for a NaN); entry e holds (r, g, b, a), straight alpha.
* Compositing, front to back: C <- C + (1 - A) a (r, g, b), A <- A + (1 - A) a.
  Here in FP64 (the GPU composites in FP32).

Output: image [H, W, 4] = (C, A).  Test infrastructure only.
"""

import numpy as np

F = 1 << 20


def transfer_index(values, scale, offset, entries=256):
    """Table entries of FP32 values (the FP32 decision the renderer takes)."""
    v = np.asarray(values, dtype=np.float32)
    t = (v - np.float32(offset)) * np.float32(scale)
    f = np.floor(t * np.float32(entries))
    with np.errstate(invalid="ignore"):
        e = np.where(f >= entries - 1, entries - 1, np.where(f > 0, f, 0))
    e = np.where(np.isnan(f), 0, e)
    return e.astype(np.int64)


def _lookup(x, lo, hi, ext, skeys, order):
    """Site index of integer points x [M, 3] (-1 where no site)."""
    inside = np.all((x >= lo) & (x <= hi), axis=1)
    s = np.full(x.shape[0], -1, dtype=np.int64)
    if np.any(inside):
        y = x[inside]
        kx = ((y[:, 0] - lo[0]) * ext[1] + (y[:, 1] - lo[1])) * ext[2] + (y[:, 2] - lo[2])
        pos = np.minimum(np.searchsorted(skeys, kx), len(skeys) - 1)
        s[inside] = np.where(skeys[pos] == kx, order[pos], -1)
    return s


def trilinear(values, sites, frac):
    """(value float32 [M], hit bool [M]) of samples whose 8 corners are `sites`
    [M, 8] (corner c = x + 2y + 4z offsets, -1 for empty) with 8-bit fractions
    `frac` [M, 3] in [0, 255]; hit: a corner of non-zero weight is a site."""
    v = np.where(sites >= 0, np.asarray(values, dtype=np.float32)[np.maximum(sites, 0)],
                 np.float32(0)).astype(np.float64)
    acc = np.zeros(sites.shape[0])
    hit = np.zeros(sites.shape[0], dtype=bool)
    for c in range(8):
        w = np.ones(sites.shape[0], dtype=np.int64)
        for a in range(3):
            fa = frac[:, a].astype(np.int64)
            w = w * np.where((c >> a) & 1, fa, 256 - fa)
        use = (w > 0) & (sites[:, c] >= 0)  # a corner of zero weight is not read
        acc = acc + np.where(use, w.astype(np.float64) * v[:, c], 0.0)  # exact, in corner order
        hit |= use
    return (acc * 2.0 ** -24).astype(np.float32), hit


def render_rays(coords, values, origins, direction, steps, lut, scale=1.0, offset=0.0,
                filter="nearest"):
    """Composited (r, g, b, a) [M, 4] (float64) of M rays with fixed-point start
    points `origins` [M, 3] and sample steps `direction` ([3], or [M, 3] for one
    per ray)."""
    if filter not in ("nearest", "trilinear"):
        raise ValueError(filter)
    coords = np.asarray(coords, dtype=np.int64).reshape(-1, 3)
    lut = np.asarray(lut, dtype=np.float32).astype(np.float64)
    P0 = np.asarray(origins, dtype=np.int64).reshape(-1, 3)
    D = np.asarray(direction, dtype=np.int64).reshape(-1, 3)  # [1, 3] or [M, 3]
    M, K = P0.shape[0], int(steps)
    C = np.zeros((M, 3))
    A = np.zeros(M)
    if coords.shape[0] == 0 or K == 0:
        return np.concatenate([C, A[:, None]], axis=1)
    lo = coords.min(axis=0)
    hi = coords.max(axis=0)
    ext = hi - lo + 1

    def key(x):  # linear key of points inside the bounding box
        return ((x[:, 0] - lo[0]) * ext[1] + (x[:, 1] - lo[1])) * ext[2] + (x[:, 2] - lo[2])

    keys = key(coords)
    order = np.argsort(keys)
    skeys = keys[order]
    entry = transfer_index(values, scale, offset, lut.shape[0])
    corners = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)
    for k in range(K):
        P = P0 + k * D
        if filter == "nearest":
            s = _lookup((P + F // 2) >> 20, lo, hi, ext, skeys, order)  # floor division by F
            m = s >= 0
            if not np.any(m):
                continue
            e = entry[s[m]]
        else:
            b = P >> 20
            frac = (P - (b << 20)) >> 12
            cs = np.stack([_lookup(b + corners[c], lo, hi, ext, skeys, order) for c in range(8)],
                          axis=1)
            val, m = trilinear(values, cs, frac)
            if not np.any(m):
                continue
            e = transfer_index(val[m], scale, offset, lut.shape[0])
        rgba = lut[e]
        a = rgba[:, 3]
        keep = 1.0 - A[m]
        C[m] += (keep * a)[:, None] * rgba[:, :3]
        A[m] += keep * a
    return np.concatenate([C, A[:, None]], axis=1)


def render(coords, values, view, lut, scale=1.0, offset=0.0):
    """Image [H, W, 4] (float64) of `values` at site `coords` ([N, 3] integers);
    view["filter"] is "nearest" (default) or "trilinear"."""
    W, H, K = int(view["width"]), int(view["height"]), int(view["steps"])
    O, R, U, D = (np.asarray(view[k], dtype=np.int64) for k in ("origin", "right", "up", "dir"))
    DR = np.asarray(view.get("dir_right", (0, 0, 0)), dtype=np.int64)
    DU = np.asarray(view.get("dir_up", (0, 0, 0)), dtype=np.int64)
    jj, ii = np.meshgrid(np.arange(H, dtype=np.int64), np.arange(W, dtype=np.int64), indexing="ij")
    i, j = ii.reshape(-1, 1), jj.reshape(-1, 1)
    P0 = O[None, :] + i * R[None, :] + j * U[None, :]
    Dij = D[None, :] + i * DR[None, :] + j * DU[None, :]
    out = render_rays(coords, values, P0, Dij, K, lut, scale, offset, view.get("filter", "nearest"))
    return out.reshape(H, W, 4)
