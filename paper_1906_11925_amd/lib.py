"""ctypes binding of libhemelb_lb.so (argument marshalling only).

Every step of the lattice-Boltzmann path runs inside the library's HIP
kernels; this module only converts Python/NumPy/torch arguments into the C
structures of include/hemelb_lb.h.  There is no fallback: if the library
cannot be loaded, ``load()`` raises.
"""

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HEMELB_LIB") or os.path.join(HERE, "libhemelb_lb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hemelb_lb.h")

c_int32, c_int64, c_double, c_float, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                 ctypes.c_float, ctypes.c_void_p)
P = ctypes.POINTER

HEMELB_OK = 0
HEMELB_EINVAL = -1
HEMELB_ENOMEM = -2
HEMELB_EDEVICE = -3
HEMELB_EDIVERGED = -4
HEMELB_EORDER = -5
HEMELB_ECANCELLED = -6

STORE_F32, STORE_F16, STORE_BF16 = 0, 1, 2
FLAG_NO_SCALE = 1
FLAG_BLOCKS, FLAG_TABLE16, FLAG_TABLE32 = 2, 4, 8
ADDR_TABLE32, ADDR_TABLE16, ADDR_BLOCKS = 0, 1, 2
ADDRESSING = {"auto": 0, "blocks": FLAG_BLOCKS, "table16": FLAG_TABLE16, "table32": FLAG_TABLE32}
ADDR_NAMES = {ADDR_TABLE32: "table32", ADDR_TABLE16: "table16", ADDR_BLOCKS: "blocks"}
IOLET_PRESSURE, IOLET_VELOCITY = 0, 1


class IoletT(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("direction", c_double * 3), ("mean", c_double),
                ("n_harm", c_int32), ("cos_k", P(c_double)), ("sin_k", P(c_double)),
                ("period", c_double)]


class DescT(ctypes.Structure):
    _fields_ = [("lattice", c_int32), ("storage", c_int32), ("flags", c_int32),
                ("n_sites", c_int64), ("coords", P(c_int32)), ("nbr", P(c_int32)),
                ("tau", c_double), ("n_iolets", c_int32), ("iolets", P(IoletT)),
                ("site_weight", P(c_double)), ("wall_normal", P(c_float)),
                ("alpha", P(c_float)), ("stream", c_void_p), ("wall_q", P(c_float))]


class InfoT(ctypes.Structure):
    _fields_ = [("n_sites", c_int64), ("n_ghosts", c_int64), ("pitch", c_int64),
                ("time", c_int64), ("lattice", c_int32), ("storage", c_int32),
                ("bytes_per_update", c_double), ("device_bytes", c_int64),
                ("addressing", c_int32)]


class ViewT(ctypes.Structure):
    _fields_ = [("origin", c_int64 * 3), ("right", c_int64 * 3), ("up", c_int64 * 3),
                ("dir", c_int64 * 3), ("width", c_int32), ("height", c_int32), ("steps", c_int32),
                ("scale", c_float), ("offset", c_float), ("lut", P(c_float)), ("filter", c_int32),
                ("dir_right", c_int64 * 3), ("dir_up", c_int64 * 3)]


VIEW_FIX = 1 << 20
FILTER_NEAREST, FILTER_TRILINEAR = 0, 1
FILTERS = {"nearest": FILTER_NEAREST, "trilinear": FILTER_TRILINEAR}


class ObjectiveT(ctypes.Structure):
    _fields_ = [("outlet", c_int32), ("q_target", c_double), ("dome", P(ctypes.c_uint8)),
                ("lam", c_double), ("t0", c_int64), ("t1", c_int64)]


class HemelbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hemelb error {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "hemelb_lb_links": (c_int32, [P(ctypes.c_uint8), P(c_int32), P(c_int32), c_int32, P(c_int64),
                                  P(c_int32), P(c_int32)]),
    "hemelb_lb_create": (c_int32, [P(c_void_p), P(DescT)]),
    "hemelb_lb_destroy": (c_int32, [c_void_p]),
    "hemelb_lb_step": (c_int32, [c_void_p, c_int64]),
    "hemelb_lb_sync": (c_int32, [c_void_p]),
    "hemelb_lb_set_check": (c_int32, [c_void_p, c_int64]),
    "hemelb_lb_cancel": (c_int32, [c_void_p]),
    "hemelb_lb_set_stream": (c_int32, [c_void_p, c_void_p]),
    "hemelb_lb_observables": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "hemelb_lb_totals": (c_int32, [c_void_p, P(c_double)]),
    "hemelb_lb_totals_noalloc": (c_int32, [c_void_p, c_void_p]),
    "hemelb_lb_get_state": (c_int32, [c_void_p, c_void_p, P(c_int64)]),
    "hemelb_lb_set_state": (c_int32, [c_void_p, c_void_p, c_int64]),
    "hemelb_lb_get_deviations": (c_int32, [c_void_p, c_void_p]),
    "hemelb_lb_set_deviations": (c_int32, [c_void_p, c_void_p, c_int64]),
    "hemelb_lb_info": (c_int32, [c_void_p, P(InfoT)]),
    "hemelb_lb_plan": (c_int32, [P(DescT), P(InfoT)]),
    "hemelb_lb_kernel_timing": (c_int32, [c_void_p, c_int64]),
    "hemelb_lb_kernel_time": (c_int32, [c_void_p, P(c_double), P(c_int64)]),
    "hemelb_copy_probe": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "hemelb_lb_render": (c_int32, [c_void_p, c_void_p, P(ViewT), c_void_p]),
    "hemelb_lb_set_iolet": (c_int32, [c_void_p, c_int32, P(IoletT)]),
    "hemelb_lb_set_alpha": (c_int32, [c_void_p, P(c_float)]),
    "hemelb_lb_set_objective": (c_int32, [c_void_p, P(ObjectiveT)]),
    "hemelb_lb_objective_value": (c_int32, [c_void_p, P(c_double), P(c_double), P(c_double)]),
    "hemelb_lb_objective_flux": (c_int32, [c_void_p, P(c_double)]),
    "hemelb_lb_adjoint_begin": (c_int32, [c_void_p, c_int64]),
    "hemelb_lb_adjoint_segment": (c_int32, [c_void_p, c_void_p, c_int64, c_int64]),
    "hemelb_lb_adjoint_run": (c_int32, [c_void_p, P(c_void_p), P(c_int64), P(c_int64), c_int64]),
    "hemelb_lb_record": (c_int32, [c_void_p, c_int64]),
    "hemelb_lb_adjoint_recorded": (c_int32, [c_void_p]),
    "hemelb_lb_record_end": (c_int32, [c_void_p]),
    "hemelb_lb_adjoint_grads": (c_int32, [c_void_p, P(c_double), P(c_double)]),
    "hemelb_lb_get_adjoint": (c_int32, [c_void_p, c_void_p]),
    "hemelb_lb_last_error": (ctypes.c_char_p, []),
    "hemelb_lb_strerror": (ctypes.c_char_p, [c_int32]),
}


def header_functions():
    """Names of the functions include/hemelb_lb.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hemelb_\w+)\s*\(", txt)) - {"HEMELB_LINK_IOLET"})


def load(build_if_missing=True):
    """Load the library; build it first when nothing is built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built")
        from . import build as _build
        _build.build()
    # One HIP runtime per process: torch bundles its own, and the library must bind
    # to it.  Loaded first, the library would bring in the system runtime, and
    # torch would then load a second one beside it (two runtimes cannot share the
    # device), so torch is imported before the library whenever it is installed.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().hemelb_lb_last_error().decode()


def check(rc):
    if rc != HEMELB_OK:
        raise HemelbError(rc, last_error())
    return rc
