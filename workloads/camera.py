"""Views and colour tables for volume rendering (input generation only).

A view is the steerable part of the paper's visualization (Section 3.C.2):
zoom, model rotation, and the scale and offset of the transfer function.  It is
handed to the renderer as fixed-point integer vectors, FIX units per lattice
spacing, so that every sample position along every ray is an exact integer:
ray (i, j) starts at origin + i * right + j * up and its k-th sample lies at
that point + k * (dir + i * dir_right + j * dir_up).  Orthographic views have
dir_right = dir_up = 0; a pinhole (perspective) view starts every ray at the eye
(right = up = 0) and spreads the directions instead.

This module only turns camera parameters into those integers and builds colour
tables; the sampling, transfer and compositing are the renderer's.
"""

import math

import numpy as np

FIX = 1 << 20  # fixed-point units per lattice spacing


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def orbit_view(center, distance, azimuth, elevation, width, height, pixel=1.0, step=0.5,
               steps=None):
    """Orthographic view of `center` from the direction given by `azimuth` and
    `elevation` (degrees; azimuth in the x-y plane from +x, elevation towards +z).

    The image plane lies `distance` lattice units before the centre, with square
    pixels of `pixel` lattice units (the zoom).  Rays march `step` lattice units
    per sample, `steps` samples (default: twice the distance, so the ray ends as
    far behind the centre as it starts before it).
    """
    az, el = math.radians(azimuth), math.radians(elevation)
    toward = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    d = -toward  # the rays travel towards the centre
    world_up = np.array([0.0, 0.0, 1.0]) if abs(toward[2]) < 0.99 else np.array([0.0, 1.0, 0.0])
    r = _unit(np.cross(d, world_up))
    u = np.cross(r, d)
    plane = np.asarray(center, dtype=np.float64) - d * distance
    origin = plane - r * pixel * (width - 1) / 2.0 - u * pixel * (height - 1) / 2.0
    if steps is None:
        steps = int(math.ceil(2.0 * distance / step))

    def fix(v):
        return [int(x) for x in np.rint(np.asarray(v) * FIX).astype(np.int64)]

    return {"origin": fix(origin), "right": fix(r * pixel), "up": fix(u * pixel),
            "dir": fix(d * step), "width": int(width), "height": int(height), "steps": int(steps)}


def perspective_view(center, distance, azimuth, elevation, width, height, fov=40.0, step=0.5,
                     steps=None):
    """Pinhole view of `center` from an eye `distance` lattice units away in the
    direction given by `azimuth` and `elevation` (degrees, as orbit_view), with a
    vertical field of view of `fov` degrees.  The central ray marches `step`
    lattice units per sample; the others the same parameter step along their
    (slightly longer) direction.  `steps` defaults to twice the distance."""
    az, el = math.radians(azimuth), math.radians(elevation)
    toward = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    d = -toward
    world_up = np.array([0.0, 0.0, 1.0]) if abs(toward[2]) < 0.99 else np.array([0.0, 1.0, 0.0])
    r = _unit(np.cross(d, world_up))
    u = np.cross(r, d)
    eye = np.asarray(center, dtype=np.float64) + toward * distance
    s = 2.0 * math.tan(math.radians(fov) / 2.0) / height  # image-plane units per pixel at depth 1
    d0 = d - r * s * (width - 1) / 2.0 - u * s * (height - 1) / 2.0
    if steps is None:
        steps = int(math.ceil(2.0 * distance / step))

    def fix(v):
        return [int(x) for x in np.rint(np.asarray(v) * FIX).astype(np.int64)]

    return {"origin": fix(eye), "right": [0, 0, 0], "up": [0, 0, 0], "dir": fix(d0 * step),
            "dir_right": fix(r * s * step), "dir_up": fix(u * s * step), "width": int(width),
            "height": int(height), "steps": int(steps)}


def axis_view(lo, hi, axis=0, pixel=1.0, step=0.5):
    """View of the box [lo, hi] (lattice coordinates) straight along +axis, one
    pixel row per `pixel` lattice units, covering the whole box."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    a, b, c = axis, (axis + 1) % 3, (axis + 2) % 3
    width = int(math.floor((hi[b] - lo[b]) / pixel)) + 1
    height = int(math.floor((hi[c] - lo[c]) / pixel)) + 1
    origin = np.zeros(3)
    origin[a] = lo[a] - 1.0
    origin[b] = lo[b]
    origin[c] = lo[c]
    right = np.zeros(3)
    right[b] = pixel
    up = np.zeros(3)
    up[c] = pixel
    d = np.zeros(3)
    d[a] = step
    steps = int(math.ceil((hi[a] - lo[a] + 2.0) / step))

    def fix(v):
        return [int(x) for x in np.rint(np.asarray(v) * FIX).astype(np.int64)]

    return {"origin": fix(origin), "right": fix(right), "up": fix(up), "dir": fix(d),
            "width": width, "height": height, "steps": steps}


def ramp_lut(opacity=0.05, entries=256):
    """Colour table of `entries` RGBA rows (straight alpha): blue through white to
    red, opacity rising linearly from 0 to `opacity`."""
    x = np.linspace(0.0, 1.0, entries)
    r = np.clip(2.0 * x, 0.0, 1.0)
    b = np.clip(2.0 - 2.0 * x, 0.0, 1.0)
    g = 1.0 - np.abs(2.0 * x - 1.0)
    a = opacity * x
    return np.stack([r, g, b, a], axis=1).astype(np.float32)
