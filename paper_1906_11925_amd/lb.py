"""Python front end of the C ABI: an `LB` handle over torch device memory.

Argument marshalling only; the neighbour-table build runs in the library's
C++ host code and every time step, observable and reduction in its HIP
kernels.
"""

import ctypes

import numpy as np

from . import lib as L

_STORE = {"f32": L.STORE_F32, "f16": L.STORE_F16, "bf16": L.STORE_BF16}


def _ptr(a, ctype):
    return a.ctypes.data_as(L.P(ctype)) if a is not None else None


def links(labels, shape, periodic, lattice):
    """(coords int32 [N,3], nbr int32 [N,Q]) from a padded label grid (C++ builder)."""
    lib = L.load()
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    X, Y, Z = (int(v) for v in shape)
    if lab.shape != (X + 2, Y + 2, Z + 2):
        raise ValueError(f"labels must have shape {(X + 2, Y + 2, Z + 2)}, got {lab.shape}")
    shp = np.array([X, Y, Z], dtype=np.int32)
    per = np.array([1 if p else 0 for p in periodic], dtype=np.int32)
    n = ctypes.c_int64(0)
    L.check(lib.hemelb_lb_links(_ptr(lab, ctypes.c_uint8), _ptr(shp, L.c_int32), _ptr(per, L.c_int32),
                                lattice, ctypes.byref(n), None, None))
    coords = np.empty((n.value, 3), dtype=np.int32)
    nbr = np.empty((n.value, lattice), dtype=np.int32)
    L.check(lib.hemelb_lb_links(_ptr(lab, ctypes.c_uint8), _ptr(shp, L.c_int32), _ptr(per, L.c_int32),
                                lattice, ctypes.byref(n), _ptr(coords, L.c_int32), _ptr(nbr, L.c_int32)))
    return coords, nbr


def lattice_vectors(lattice):
    """Lattice vectors in the interface ordering (rest, then opposite pairs)."""
    faces = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    second = ([(1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1)] if lattice == 15 else
              [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)])
    out = [(0, 0, 0)]
    for v in faces + second:
        out += [v, tuple(-a for a in v)]
    return np.array(out, dtype=np.int64)


def _torch():
    import torch
    return torch


def _desc(nbr, tau, lattice=15, storage="f32", coords=None, iolets=(), site_weight=None,
          wall_normal=None, alpha=None, stream_ptr=None, scale=True, wall_q=None,
          addressing="auto"):
    """(DescT, arrays it points into) for the arguments of `LB`."""
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    n = nbr.shape[0]
    if nbr.ndim != 2 or nbr.shape[1] != lattice:
        raise ValueError("nbr must be [N, lattice]")
    if addressing not in L.ADDRESSING:
        raise ValueError(f"addressing must be one of {sorted(L.ADDRESSING)}")
    keep = [nbr]
    io_arr = (L.IoletT * max(1, len(iolets)))()
    keep.append(io_arr)
    for k, io in enumerate(iolets):
        cos = np.ascontiguousarray(getattr(io, "cos", ()), dtype=np.float64)
        sin = np.ascontiguousarray(getattr(io, "sin", ()), dtype=np.float64)
        if cos.shape != sin.shape:
            raise ValueError("cos and sin harmonics must have the same length")
        keep += [cos, sin]
        io_arr[k].kind = L.IOLET_PRESSURE if io.kind == "pressure" else L.IOLET_VELOCITY
        for a in range(3):
            io_arr[k].direction[a] = float(io.direction[a])
        io_arr[k].mean = float(io.mean)
        io_arr[k].n_harm = int(cos.size)
        io_arr[k].cos_k = _ptr(cos, L.c_double) if cos.size else None
        io_arr[k].sin_k = _ptr(sin, L.c_double) if sin.size else None
        io_arr[k].period = float(getattr(io, "period", 1.0))
    d = L.DescT()
    d.lattice = lattice
    d.storage = _STORE[storage]
    d.flags = (0 if scale else L.FLAG_NO_SCALE) | L.ADDRESSING[addressing]
    d.n_sites = n
    if coords is not None:
        coords = np.ascontiguousarray(coords, dtype=np.int32)
        keep.append(coords)
        d.coords = _ptr(coords, L.c_int32)
    d.nbr = _ptr(nbr, L.c_int32)
    d.tau = float(tau)
    d.n_iolets = len(iolets)
    d.iolets = io_arr
    if wall_q is not None:
        wall_q = np.nan_to_num(np.asarray(wall_q, dtype=np.float32), nan=0.5)
    for name, arr, ct, dt in (("site_weight", site_weight, L.c_double, np.float64),
                              ("wall_normal", wall_normal, L.c_float, np.float32),
                              ("alpha", alpha, L.c_float, np.float32),
                              ("wall_q", wall_q, L.c_float, np.float32)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=dt)
            keep.append(a)
            setattr(d, name, _ptr(a, ct))
    d.stream = stream_ptr
    return d, keep


def _info_dict(i):
    out = {f: getattr(i, f) for f, _ in L.InfoT._fields_}
    out["addressing_name"] = L.ADDR_NAMES.get(out["addressing"], "?")
    return out


def plan(nbr, tau, **kw):
    """Layout `LB(nbr, tau, **kw)` would build, from the host library alone (no
    GPU needed): n_sites, n_ghosts, pitch, addressing, bytes_per_update and the
    device bytes it would allocate."""
    lib = L.load()
    d, keep = _desc(nbr, tau, **kw)
    i = L.InfoT()
    L.check(lib.hemelb_lb_plan(ctypes.byref(d), ctypes.byref(i)))
    del keep
    return _info_dict(i)


def plan_geometry(geom, lattice=15, storage="f32", tau=None, bfl=False, **kw):
    """`plan` for a workloads.Geometry, with the arguments of LB.from_geometry."""
    coords, nbr = links(geom.labels, geom.shape, geom.periodic, lattice)
    if bfl:
        kw["wall_q"] = geom.wall_fractions(lattice_vectors(lattice))
    return plan(nbr, geom.tau if tau is None else tau, lattice=lattice, storage=storage,
                coords=coords, iolets=list(geom.iolets), site_weight=geom.site_weight(), **kw)


class LB:
    """One simulation handle on the current GPU (see include/hemelb_lb.h)."""

    def __init__(self, nbr, tau, lattice=15, storage="f32", coords=None, iolets=(),
                 site_weight=None, wall_normal=None, alpha=None, stream=None, scale=True,
                 wall_q=None, addressing="auto"):
        torch = _torch()
        self.lib = L.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        d, keep = _desc(nbr, tau, lattice=lattice, storage=storage, coords=coords, iolets=iolets,
                        site_weight=site_weight, wall_normal=wall_normal, alpha=alpha,
                        stream_ptr=ctypes.c_void_p(stream.cuda_stream), scale=scale,
                        wall_q=wall_q, addressing=addressing)
        self.n, self.q, self.storage = d.n_sites, lattice, storage
        self.tau = float(tau)
        h = ctypes.c_void_p()
        L.check(self.lib.hemelb_lb_create(ctypes.byref(h), ctypes.byref(d)))
        self.h = h
        self.iolets = list(iolets)
        del keep

    @classmethod
    def from_geometry(cls, geom, lattice=15, storage="f32", tau=None, alpha=None, bfl=False,
                      **kw):
        """Handle for a workloads.Geometry; bfl=True places the walls where the
        geometry's continuous surface cuts each wall link (interpolated walls)."""
        coords, nbr = links(geom.labels, geom.shape, geom.periodic, lattice)
        if bfl:
            kw["wall_q"] = geom.wall_fractions(lattice_vectors(lattice))
        return cls(nbr, geom.tau if tau is None else tau, lattice=lattice, storage=storage,
                   coords=coords, iolets=list(geom.iolets), site_weight=geom.site_weight(),
                   alpha=alpha, **kw)

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.check(self.lib.hemelb_lb_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping --------------------------------------------------------------
    def step(self, n=1):
        L.check(self.lib.hemelb_lb_step(self.h, int(n)))

    def sync(self):
        L.check(self.lib.hemelb_lb_sync(self.h))

    def set_check(self, every):
        L.check(self.lib.hemelb_lb_set_check(self.h, int(every)))

    def cancel(self):
        L.check(self.lib.hemelb_lb_cancel(self.h))

    def info(self):
        i = L.InfoT()
        L.check(self.lib.hemelb_lb_info(self.h, ctypes.byref(i)))
        return _info_dict(i)

    @property
    def time(self):
        return self.info()["time"]

    # -- rendering --------------------------------------------------------------
    def render(self, values, view, lut, scale=1.0, offset=0.0, image=None):
        """Ray-marched image [H, W, 4] (float32 CUDA tensor) of per-site `values`
        (float32 CUDA tensor [N], caller order) seen through `view` (a dict of the
        fixed-point vectors origin, right, up, dir and width, height, steps, and
        optionally dir_right and dir_up (per-pixel direction increments: a pinhole
        view) and filter: "nearest" (default) or "trilinear"; see
        include/hemelb_lb.h) with the RGBA colour table `lut` ([256, 4])."""
        torch = _torch()
        v = L.ViewT()
        for name in ("origin", "right", "up", "dir", "dir_right", "dir_up"):
            vec = view.get(name, (0, 0, 0)) if name.startswith("dir_") else view[name]
            for a in range(3):
                getattr(v, name)[a] = int(vec[a])
        v.width, v.height, v.steps = int(view["width"]), int(view["height"]), int(view["steps"])
        v.scale, v.offset = float(scale), float(offset)
        f = view.get("filter", "nearest")
        v.filter = L.FILTERS[f] if isinstance(f, str) else int(f)
        lut = np.ascontiguousarray(lut, dtype=np.float32)
        if lut.shape != (256, 4):
            raise ValueError("lut must be [256, 4]")
        v.lut = _ptr(lut, L.c_float)
        values = values.contiguous()
        if values.dtype != torch.float32 or values.numel() != self.n or not values.is_cuda:
            raise ValueError("values must be a float32 CUDA tensor with one entry per site")
        if image is None:
            image = torch.empty((v.height, v.width, 4), dtype=torch.float32, device="cuda")
        L.check(self.lib.hemelb_lb_render(self.h, ctypes.c_void_p(values.data_ptr()), ctypes.byref(v),
                                          ctypes.c_void_p(image.data_ptr())))
        return image

    # -- outputs -----------------------------------------------------------------
    def observables(self):
        """(p_dev [N], u [N, 3], wss [N]) float32 CUDA tensors in caller order."""
        torch = _torch()
        p = torch.empty(self.n, dtype=torch.float32, device="cuda")
        u = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        w = torch.empty(self.n, dtype=torch.float32, device="cuda")
        L.check(self.lib.hemelb_lb_observables(self.h, ctypes.c_void_p(p.data_ptr()),
                                               ctypes.c_void_p(u.data_ptr()),
                                               ctypes.c_void_p(w.data_ptr())))
        return p, u, w

    def observables_into(self, p, u, w):
        """Write the observables into existing float32 CUDA tensors (any may be None)."""
        ptr = lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None  # noqa: E731
        L.check(self.lib.hemelb_lb_observables(self.h, ptr(p), ptr(u), ptr(w)))

    def totals(self):
        out = (ctypes.c_double * 4)()
        L.check(self.lib.hemelb_lb_totals(self.h, out))
        return np.array(list(out))

    def _raw_dtype(self):
        torch = _torch()
        return {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.storage]

    def get_state(self):
        torch = _torch()
        dst = torch.empty((self.q, self.n), dtype=self._raw_dtype(), device="cuda")
        t = ctypes.c_int64(0)
        L.check(self.lib.hemelb_lb_get_state(self.h, ctypes.c_void_p(dst.data_ptr()), ctypes.byref(t)))
        return dst, t.value

    def set_state(self, src, t=0):
        src = src.contiguous()
        if src.dtype != self._raw_dtype() or tuple(src.shape) != (self.q, self.n):
            raise ValueError("state must be [Q, N] in the storage dtype")
        L.check(self.lib.hemelb_lb_set_state(self.h, ctypes.c_void_p(src.data_ptr()), int(t)))
        self._keep = src

    def get_deviations(self):
        torch = _torch()
        dst = torch.empty((self.q, self.n), dtype=torch.float32, device="cuda")
        L.check(self.lib.hemelb_lb_get_deviations(self.h, ctypes.c_void_p(dst.data_ptr())))
        return dst

    def set_deviations(self, src, t=0):
        torch = _torch()
        src = src.to(device="cuda", dtype=torch.float32).contiguous()
        if tuple(src.shape) != (self.q, self.n):
            raise ValueError("deviations must be [Q, N]")
        L.check(self.lib.hemelb_lb_set_deviations(self.h, ctypes.c_void_p(src.data_ptr()), int(t)))
        self._keep = src

    # -- parameters, objective and adjoint -------------------------------------------
    def set_iolet(self, k, io):
        """Replace iolet k's time series (same kind, harmonics count and direction)."""
        cos = np.ascontiguousarray(getattr(io, "cos", ()), dtype=np.float64)
        sin = np.ascontiguousarray(getattr(io, "sin", ()), dtype=np.float64)
        t = L.IoletT()
        t.kind = L.IOLET_PRESSURE if io.kind == "pressure" else L.IOLET_VELOCITY
        for a in range(3):
            t.direction[a] = float(io.direction[a])
        t.mean = float(io.mean)
        t.n_harm = int(cos.size)
        t.cos_k = _ptr(cos, L.c_double) if cos.size else None
        t.sin_k = _ptr(sin, L.c_double) if sin.size else None
        t.period = float(getattr(io, "period", 1.0))
        L.check(self.lib.hemelb_lb_set_iolet(self.h, int(k), ctypes.byref(t)))
        self.iolets[k] = io

    def set_alpha(self, alpha):
        if alpha is None:
            L.check(self.lib.hemelb_lb_set_alpha(self.h, None))
            return
        a = np.ascontiguousarray(alpha, dtype=np.float32)
        if a.shape != (self.n,):
            raise ValueError("alpha must be [N]")
        L.check(self.lib.hemelb_lb_set_alpha(self.h, _ptr(a, L.c_float)))

    def set_objective(self, outlet, q_target, dome, lam, window):
        """J = sum_{t in window} (Q(t) - q_target)^2 + lam * mean_t mean_{dome} WSS."""
        o = L.ObjectiveT()
        o.outlet = int(outlet)
        o.q_target = float(q_target)
        self._dome = None
        if dome is not None:
            self._dome = np.ascontiguousarray(dome, dtype=np.uint8)
            if self._dome.shape != (self.n,):
                raise ValueError("dome must be [N]")
            o.dome = _ptr(self._dome, ctypes.c_uint8)
        o.lam = float(lam)
        o.t0, o.t1 = int(window[0]), int(window[1])
        self.window = (o.t0, o.t1)
        L.check(self.lib.hemelb_lb_set_objective(self.h, ctypes.byref(o)))

    def clear_objective(self):
        L.check(self.lib.hemelb_lb_set_objective(self.h, None))

    def objective_value(self):
        """(J, flux term, shear term) in FP64."""
        v = [ctypes.c_double(0) for _ in range(3)]
        L.check(self.lib.hemelb_lb_objective_value(self.h, *(ctypes.byref(x) for x in v)))
        return tuple(x.value for x in v)

    def objective_flux(self):
        q = np.zeros(max(1, self.window[1] - self.window[0]))
        L.check(self.lib.hemelb_lb_objective_flux(self.h, _ptr(q, L.c_double)))
        return q[: self.window[1] - self.window[0]]

    def adjoint_begin(self, max_segment):
        L.check(self.lib.hemelb_lb_adjoint_begin(self.h, int(max_segment)))

    def adjoint_segment(self, checkpoint, t0, steps):
        checkpoint = checkpoint.contiguous()
        if checkpoint.dtype != self._raw_dtype() or tuple(checkpoint.shape) != (self.q, self.n):
            raise ValueError("checkpoint must be a raw state [Q, N]")
        L.check(self.lib.hemelb_lb_adjoint_segment(self.h, ctypes.c_void_p(checkpoint.data_ptr()),
                                                   int(t0), int(steps)))
        self._keep = checkpoint

    def adjoint_run(self, segments):
        """The whole reverse sweep: `segments` is a list of (t0, steps, checkpoint)
        in forward order (checkpoint = raw state [Q, N] at time t0); each adjoint
        step runs in one launch with a recompute step of the next earlier segment
        (hemelb_lb_adjoint_run)."""
        keep = []
        for _, _, ck in segments:
            ck = ck.contiguous()
            if ck.dtype != self._raw_dtype() or tuple(ck.shape) != (self.q, self.n):
                raise ValueError("checkpoint must be a raw state [Q, N]")
            keep.append(ck)
        k = len(segments)
        ptrs = (ctypes.c_void_p * max(k, 1))(*[c.data_ptr() for c in keep])
        t0 = (ctypes.c_int64 * max(k, 1))(*[int(s[0]) for s in segments])
        st = (ctypes.c_int64 * max(k, 1))(*[int(s[1]) for s in segments])
        L.check(self.lib.hemelb_lb_adjoint_run(self.h, ptrs, t0, st, k))
        self._keep = keep

    def record(self, max_steps):
        """Keep the next `max_steps` states on the device (hemelb_lb_record); with
        FP32 storage also each step's pre-collision populations, when memory allows."""
        L.check(self.lib.hemelb_lb_record(self.h, int(max_steps)))

    def adjoint_recorded(self):
        """Reverse sweep over the recorded states, no recomputation."""
        L.check(self.lib.hemelb_lb_adjoint_recorded(self.h))

    def record_end(self):
        """Free the recorded trajectory; the current state stays."""
        L.check(self.lib.hemelb_lb_record_end(self.h))

    def theta_sizes(self):
        """Number of Fourier coefficients of each velocity iolet, in id order."""
        return [(k, 1 + 2 * len(getattr(io, "cos", ()))) for k, io in enumerate(self.iolets)
                if io.kind == "velocity"]

    def adjoint_grads(self):
        """({velocity iolet k: dJ/d(mean, cos_h, sin_h)}, dJ/dalpha [N]) in FP64."""
        sizes = self.theta_sizes()
        th = np.zeros(max(1, sum(b for _, b in sizes)))
        da = np.zeros(max(1, self.n))
        L.check(self.lib.hemelb_lb_adjoint_grads(self.h, _ptr(th, L.c_double), _ptr(da, L.c_double)))
        out, off = {}, 0
        for k, b in sizes:
            out[k] = th[off:off + b].copy()
            off += b
        return out, da[: self.n]

    def get_adjoint(self):
        torch = _torch()
        dst = torch.empty((self.q, self.n), dtype=torch.float32, device="cuda")
        L.check(self.lib.hemelb_lb_get_adjoint(self.h, ctypes.c_void_p(dst.data_ptr())))
        return dst

    # -- timing -------------------------------------------------------------------
    def kernel_timing(self, max_launches):
        L.check(self.lib.hemelb_lb_kernel_timing(self.h, int(max_launches)))

    def kernel_time(self):
        ms = ctypes.c_double(0)
        k = ctypes.c_int64(0)
        L.check(self.lib.hemelb_lb_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value


def copy_probe(dst, src, nbytes, stream=None):
    """Plain device copy kernel (bandwidth ceiling / counter calibration)."""
    torch = _torch()
    lib = L.load()
    if stream is None:
        stream = torch.cuda.current_stream()
    L.check(lib.hemelb_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                  int(nbytes), ctypes.c_void_p(stream.cuda_stream)))


def relaxation_time(viscosity, step, voxel, density=1000.0):
    """tau = 1/2 + 3 nu dt / dx^2 for a physical dynamic viscosity (Pa s), time
    step (s), voxel size (m) and density (kg/m^3); Table 1 and Section 4 give
    dt = 2e-5 s, dx = 1e-4 m, mu = 0.004 Pa s."""
    nu = viscosity / density
    return 0.5 + 3.0 * nu * step / (voxel * voxel)


__all__ = ["LB", "links", "copy_probe", "relaxation_time"]
