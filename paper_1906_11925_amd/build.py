"""Build the C-ABI library libhemelb_lb.so in-tree with hipcc for gfx950."""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhemelb_lb.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "adjoint.hip"),
           os.path.join(CSRC, "render.hip"), os.path.join(CSRC, "host.cpp")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


COMPILE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler away from packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# the profiler's marker library (named ranges around the entry points)
LIBS = ["-lrocprofiler-sdk-roctx", "-lpthread"]


def command(out=LIB):
    """One hipcc command that compiles and links every source."""
    return [hipcc(), *COMPILE_FLAGS, "-shared", *SOURCES, *LIBS, "-o", out]


def compile_command(src, obj):
    return [hipcc(), *COMPILE_FLAGS, "-c", src, "-o", obj]


def link_command(objs, out):
    return [hipcc(), "--offload-arch=gfx950", "-shared", *objs, *LIBS, "-o", out]


# Sanitizer builds of the host code (the planner and its thread pool) for the CPU.
# Only the host library source is compiled, for the host side only; the caller
# supplies a driver program and stand-ins for the kernel launchers, so no device
# code is built and nothing needs a GPU.  Every sanitizer flag is scoped to the
# host pass.
HOST_SOURCE = os.path.join(CSRC, "host.cpp")
SANITIZERS = {
    "address": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined"],
    "thread": ["-Xarch_host", "-fsanitize=thread"],
}


def sanitized_command(kind, sources, out):
    """hipcc command linking host.cpp with `sources` (a driver calling the C ABI and
    the launcher stand-ins) under sanitizer `kind`: "address" (ASan + UBSan) or
    "thread" (TSan)."""
    return [
        hipcc(),
        "--offload-arch=gfx950",
        "--offload-host-only",
        "-O1",
        "-g",
        "-std=c++17",
        "-Xarch_host", "-fno-omit-frame-pointer",
        *SANITIZERS[kind],
        "-I", os.path.join(ROOT, "include"),
        *sources,
        HOST_SOURCE,
        *LIBS,
        "-o", out,
    ]


def build_sanitized(kind, sources, out):
    res = subprocess.run(sanitized_command(kind, sources, out), capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"sanitized build ({kind}) failed")
    return out


def build(verbose: bool = False) -> str:
    """Compile each source to an object in parallel (under _build/), then link the
    library in-tree; the library is replaced only when every step succeeds."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        results = list(pool.map(lambda so: subprocess.run(compile_command(*so), capture_output=True,
                                                          text=True), zip(SOURCES, objs)))
    for src, res in zip(SOURCES, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed on " + src)
        if verbose:
            sys.stderr.write(res.stderr)
    tmp = LIB + ".tmp"
    res = subprocess.run(link_command(objs, tmp), capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
