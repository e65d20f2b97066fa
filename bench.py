#!/usr/bin/env python3
"""Throughput of the sparse lattice-Boltzmann step on one MI355X.

One benchmark step is one full time step of the path: the fused pull-stream +
LBGK collide kernel over every fluid site of the workload, whose epilogue also
writes the next step's incoming iolet populations (site updates counted as in
the paper's Table 3: sites x steps / wall time).  Default workload: the seeded
Murray tree in a 2048^3 box (root radius 64, 8 bifurcation generations, seed 5;
53,020,072 fluid sites), D3Q15, tau 0.6, FP32 storage, inputs resident in HBM,
with velocity, pressure and wall shear stress computed every 100 steps inside the
timed run, as the workload's configuration states.  Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fluid-site updates/s (GLUPS) + % HBM peak, FP32 vs FP16-store; adjoint GLUPS"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_1906_11925_amd", "csrc", f)
               for f in ("kernels.hip", "kernels.hpp", "step.hpp", "lbdev.hpp", "lattice.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def method_bytes(q, storage):
    """Bytes of one site update for the method as stated: every population read
    once and written once, plus an int32 neighbour table entry per moving
    direction (2 Q s + 4 (Q - 1): D3Q15 FP32 176 B, 16-bit 116 B; D3Q19 FP32
    224 B, 16-bit 148 B)."""
    s = 4 if storage == "f32" else 2
    return 2 * q * s + 4 * (q - 1)


def kernel_sha():
    """Hash of the sources the stream-collide kernel is compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_run(lb, steps, warmup, obs_every=0, events=None):
    """Wall time of `steps` steps; with events=(start, end) (HIP events on the
    library's stream, which is torch's current stream) also brackets them on
    the GPU."""
    import torch
    lb.step(warmup)
    lb.sync()
    torch.cuda.synchronize()
    obs = lb.observables() if obs_every > 0 else None  # outputs allocated before timing
    t0 = time.perf_counter()
    if events:
        events[0].record()
    if obs_every > 0:
        done = 0
        while done < steps:
            k = min(obs_every, steps - done)
            lb.step(k)
            done += k
            if done % obs_every == 0:
                lb.observables_into(*obs)
    else:
        lb.step(steps)
    if events:
        events[1].record()
    lb.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def aux_timings(lb, n, q, elem, bpu, reps=20):
    """The on-demand outputs on the benchmark's lattice: one observables pass
    (HIP events around `reps` calls; it re-gathers the last step's pre-collision
    populations and writes p, u, WSS in caller order) and one FP64 totals call
    (host wall time, including its synchronisation and the copy of 4 doubles)."""
    import torch
    obs = lb.observables()
    lb.totals()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lb.observables_into(*obs)
    e1.record()
    torch.cuda.synchronize()
    obs_ms = e0.elapsed_time(e1) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        lb.totals()
    tot_ms = (time.perf_counter() - t0) / reps * 1e3
    obs_bytes = bpu - q * elem + 20.0  # one step's reads (populations + addressing) + 20 B out
    return {"observables_ms": obs_ms,
            "observables_GBs_algorithmic": obs_bytes * n / (obs_ms * 1e-3) / 1e9,
            "totals_ms_incl_sync": tot_ms,
            "totals_GBs_algorithmic": q * elem * n / (tot_ms * 1e-3) / 1e9}


def region_kernel_ms(lb, steps, warmup):
    """Average duration of the fused stream+collide kernel: HIP events on the
    library's stream around `steps` back-to-back steps, each of which is one
    launch of that kernel (plus a ~2.5 us iolet-series kernel per 1024 steps)."""
    import torch
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    timed_run(lb, steps, warmup, 0, ev)
    return ev[0].elapsed_time(ev[1]) / steps


def kernel_avg_ms(lb, steps):
    """Average duration from HIP event pairs recorded around each launch (the
    event records add a few microseconds per launch)."""
    lb.kernel_timing(steps)
    lb.step(steps)
    ms, k = lb.kernel_time()
    lb.kernel_timing(0)
    return ms / max(k, 1)


def traffic_for(workload, storage, addressing):
    """Counter-derived HBM bytes per launch, if taken on the current kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(f"{workload}/{storage}/{addressing}")
    if not entry or rec.get("kernel_sha") != kernel_sha():
        return None
    return entry.get("bytes_per_launch")


def pipe_errors(steps=2000):
    """Error of each storage form against the FP64 oracle on the straight pipe
    (13,312 sites, D3Q15, tau 0.8, pressure iolets) after `steps` steps:
    max_s |x - x_ref| / max_s |x_ref| for velocity, pressure deviation and WSS."""
    import numpy as np
    import workloads as wl
    from oracle.lbgk import LBGK
    from paper_1906_11925_amd import LB
    g = wl.pipe()
    o = LBGK(g, 15)
    _, f = o.run(o.rest_state(), 0, steps)
    op, ou, _, ow = o.observables(f)
    ref = {"u": ou.T, "p": op - 1.0 / 3.0, "wss": ow}

    def rel(a, b):
        if a.ndim == 2:
            return float(np.sqrt(((a - b) ** 2).sum(1)).max() / np.sqrt((b ** 2).sum(1)).max())
        return float(np.abs(a - b).max() / np.abs(b).max())

    out = {}
    # the 16-bit forms also without the per-direction power-of-two scale, which
    # keeps small deviations out of the FP16 subnormals
    for key, st, scaled in (("f32", "f32", True), ("f16", "f16", True), ("bf16", "bf16", True),
                            ("f16_unscaled", "f16", False), ("bf16_unscaled", "bf16", False)):
        lb = LB.from_geometry(g, storage=st, scale=scaled)
        lb.step(steps)
        p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
        out[key] = {"e_u": rel(u, ref["u"]), "e_p": rel(p, ref["p"]), "e_wss": rel(w, ref["wss"])}
        lb.close()
    return out


def cpu_baseline(geom, lattice, sites, seconds=10.0):
    """The FP64 oracle as it stands, one thread.  With `sites` below the
    workload's size it times the oracle's sampled step (the same arithmetic,
    restricted to a contiguous range of `sites` sites in the middle of the site
    list, reading the full-size state) for at least `seconds`; otherwise whole
    steps."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.lbgk import LBGK
    n = geom.n_sites
    with threadpool_limits(limits=1):
        if sites < n:
            a = (n - sites) // 2
            o = LBGK(geom, lattice, sites=np.arange(a, a + sites))
            A = np.repeat(o.lat.w[:, None], n, axis=1)
            what = (f"oracle sampled step over {sites} contiguous sites (of {n}) of the "
                    f"{geom.name} workload, reading the full-size FP64 state")
        else:
            o = LBGK(geom, lattice)
            A = o.rest_state()
            what = f"full oracle steps of the {geom.name} workload ({n} sites)"
        sampled = sites < n
        B, _ = o.step(A, 0)  # warm-up (first-touch allocations)
        k = 0
        t0 = time.perf_counter()
        while True:
            B2, _ = o.step(A if sampled else B, 1 + k)
            if not sampled:
                B = B2
            k += 1
            dt = time.perf_counter() - t0
            if dt >= seconds:
                break
    return {"value": o.n * k / dt / 1e9, "unit": "GLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{k} x {what}; FP64 NumPy, single thread, {dt:.1f} s"}


def storage_errors(make, steps):
    """16-bit storage against FP32 storage on the benchmark's own workload and
    lattice: both run `steps` steps from rest, then
    max_s |x - x_f32| / max_s |x_f32| for velocity, pressure deviation and WSS.
    (The FP32 path itself is held to the FP64 oracle by the parity tests, to
    1e-5 in the same metric, so these figures are the 16-bit forms' error
    against the oracle to within that.)"""
    import numpy as np

    def run(st):
        lb = make(st)
        lb.step(steps)
        out = [x.cpu().numpy().astype(np.float64) for x in lb.observables()]
        lb.close()
        return out

    def rel(a, b):
        if a.ndim == 2:
            return float(np.sqrt(((a - b) ** 2).sum(1)).max() / np.sqrt((b ** 2).sum(1)).max())
        return float(np.abs(a - b).max() / np.abs(b).max())

    ref = run("f32")
    out = {"steps": steps}
    for st in ("f16", "bf16"):
        p, u, w = run(st)
        out[st] = {"e_u": rel(u, ref[1]), "e_p": rel(p, ref[0]), "e_wss": rel(w, ref[2])}
    return out


ADJOINT_RUNS = {"aneurysm_half": dict(name="aneurysm_half", steps=4000, K=200, window=1000),
                "tree1024": dict(name="tree1024", steps=200, K=50, window=100)}


def adjoint_dome(g):
    """Wall sites of the objective's shear term: the aneurysm's dome (sites within
    radius + 2 of the sphere's centre), or on a tree the wall of the root segment
    (the first 8 root radii above its start)."""
    import numpy as np
    c = g.coords.astype(np.float64)
    if "centre" in g.info:
        C, R = g.info["centre"], g.info["radius"]
        return ((c[:, 0] - C[0]) ** 2 + (c[:, 1] - C[1]) ** 2 + (c[:, 2] - C[2]) ** 2) < (R + 2) ** 2
    return c[:, 2] < c[:, 2].min() + 8.0 * g.info["r0"]


def adjoint_run(name="aneurysm_half", steps=4000, K=200, window=1000):
    """Adjoint workload: FP32 forward from rest, outlet flux + wall-shear objective
    over the last `window` steps, gradients with respect to the inlet's Fourier
    coefficients and a Brinkman field alpha ~ U[0, 0.01], checkpoints every K
    steps (the paired sweep: one launch per reverse step, holding that step's
    reverse half and a recompute step of the previous segment), then the same
    gradients with every state kept in HBM (no recompute).  Adjoint GLUPS =
    sites x steps / wall time of the reverse sweep."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_1906_11925_amd import LB
    g = wl.config_geometry(name)
    n = g.n_sites
    dome = adjoint_dome(g)
    alpha = np.random.default_rng(4).uniform(0.0, 0.01, n).astype(np.float32)
    lb = LB.from_geometry(g, alpha=alpha)
    W = (steps - window, steps)
    lb.set_objective(1, 0.0, dome, 1.0, W)

    def forward():
        lb.set_deviations(torch.zeros((lb.q, n), dtype=torch.float32, device="cuda"), t=0)
        cks = []
        for t0 in range(0, steps, K):
            cks.append((t0, min(K, steps - t0), lb.get_state()[0].clone()))
            lb.step(min(K, steps - t0))
        lb.sync()
        return cks

    forward()
    q = lb.objective_flux()
    lb.set_objective(1, 0.9 * float(q.mean()), dome, 1.0, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cks = forward()
    t_fwd = time.perf_counter() - t0
    J = lb.objective_value()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.adjoint_begin(K)
    lb.adjoint_run(cks)  # recompute of segment k-1 overlaps the reverse of segment k
    th, da = lb.adjoint_grads()
    t_bwd = time.perf_counter() - t0
    del cks
    # the same gradients with every state kept in HBM (steps + 1 population
    # buffers): no recomputation in the reverse sweep
    lb.set_deviations(torch.zeros((lb.q, n), dtype=torch.float32, device="cuda"), t=0)
    lb.record(steps)
    rec_gb = lb.info()["device_bytes"] / 1e9
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.step(steps)
    lb.sync()
    t_fwd_rec = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.adjoint_begin(1)
    lb.adjoint_recorded()
    th2, da2 = lb.adjoint_grads()
    t_bwd_rec = time.perf_counter() - t0
    lb.record_end()
    lb.close()
    return {"workload": name, "sites": n, "steps": steps, "checkpoint_every": K,
            "window": window, "J": J[0], "forward_s": t_fwd, "reverse_s": t_bwd,
            "adjoint_GLUPS": n * steps / t_bwd / 1e9,
            "forward_GLUPS_with_objective": n * steps / t_fwd / 1e9,
            "dJ_dtheta": [float(x) for x in th[0]],
            "dJ_dalpha_norm": float(np.linalg.norm(da)),
            "recorded": {"forward_s": t_fwd_rec, "reverse_s": t_bwd_rec,
                         "adjoint_GLUPS": n * steps / t_bwd_rec / 1e9,
                         "device_GB_while_recording": rec_gb,
                         "gradients_identical_to_checkpointed": bool(
                             np.array_equal(th[0], th2[0]) and np.array_equal(da, da2)),
                         "max_rel_diff_dtheta": float(np.abs(np.asarray(th2[0]) - np.asarray(th[0])).max()
                                                      / max(np.abs(np.asarray(th[0])).max(), 1e-300)),
                         "max_rel_diff_dalpha": float(np.abs(np.asarray(da2) - np.asarray(da)).max()
                                                      / max(np.abs(np.asarray(da)).max(), 1e-300))}}


def render_run(lb, geom, size=1024, frames=20):
    """In-situ volume rendering of the flow speed |u| of the benchmark's state:
    a size x size orthographic view of the whole vessel (step half a lattice
    spacing), timed with HIP events over `frames` frames."""
    import numpy as np
    import torch
    from workloads.camera import orbit_view, ramp_lut
    _, u, _ = lb.observables()
    speed = torch.linalg.vector_norm(u, dim=1).contiguous()
    hi = float(speed.max())
    c = geom.coords
    centre = (c.min(axis=0) + c.max(axis=0)) / 2.0
    extent = float(np.linalg.norm(c.max(axis=0) - c.min(axis=0)))
    view = orbit_view(centre, extent, 35, 25, size, size, pixel=extent / size, step=0.5)
    lut = ramp_lut(0.05)
    image = lb.render(speed, view, lut, scale=1.0 / max(hi, 1e-30))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(frames):
        lb.render(speed, view, lut, scale=1.0 / max(hi, 1e-30), image=image)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / frames
    lit = float((image[..., 3] > 0).float().mean())
    tri = dict(view, filter="trilinear")
    lb.render(speed, tri, lut, scale=1.0 / max(hi, 1e-30), image=image)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(frames):
        lb.render(speed, tri, lut, scale=1.0 / max(hi, 1e-30), image=image)
    e1.record()
    torch.cuda.synchronize()
    ms_tri = e0.elapsed_time(e1) / frames
    log(f"[bench] render {size}x{size}: {ms:.3f} ms/frame (nearest), {ms_tri:.3f} (trilinear)")
    return {"field": "speed", "width": size, "height": size, "steps": view["steps"],
            "step_lattice_units": 0.5, "ms_per_frame": ms, "frames_per_s": 1e3 / ms,
            "rays_per_s": size * size / (ms * 1e-3), "lit_fraction": lit,
            "trilinear_ms_per_frame": ms_tri}


def form_timing(make, geom, storage, steps, warmup, addressing="auto", lattice=15, obs_every=0):
    """GLUPS (wall clock over `steps` steps) and the kernel's average duration
    (HIP events around a second pass) of one storage/addressing/lattice form."""
    n = geom.n_sites
    x = make(storage, addressing, lattice)
    d = timed_run(x, steps, warmup, obs_every)
    km = region_kernel_ms(x, steps, 10)
    xi = x.info()
    x.close()
    mb = method_bytes(lattice, storage)
    return {"GLUPS": n * steps / d / 1e9, "ms_per_step": d / steps * 1e3, "kernel_avg_ms": km,
            "addressing": xi["addressing_name"], "bytes_per_update": xi["bytes_per_update"],
            "achieved_GBs": xi["bytes_per_update"] * n / (km * 1e-3) / 1e9,
            "method_bytes_per_update": mb,
            "frac_of_peak_method_bytes": mb * n / (km * 1e-3) / 1e9 / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="tree2048")
    ap.add_argument("--lattice", type=int, default=15)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--cpu-sites", type=int, default=2_000_000,
                    help="sites of the oracle's sampled step for cpu_baseline (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other forms, error legs, smaller workloads and the adjoint")
    ap.add_argument("--size-matched", action="store_true",
                    help="also time the ~400M-site size-matched tree (tree2048_400M)")
    ap.add_argument("--obs-every", type=int, default=100,
                    help="compute velocity/pressure/WSS every k steps inside the timed runs of the "
                         "benchmark's workload, as its configuration states (0: never)")
    ap.add_argument("--addressing", default="auto", choices=["auto", "blocks", "table16", "table32"],
                    help="how the kernels find upstream neighbours (auto: the library's default)")
    ap.add_argument("--adjoint", action="store_true",
                    help="only the adjoint workload (checkpointed and recorded sweeps), one JSON line")
    ap.add_argument("--adjoint-workload", default="aneurysm_half", choices=["aneurysm_half", "tree1024"],
                    help="with --adjoint: aneurysm_half (4000 steps, checkpoints every 200, window "
                         "1000) or tree1024 (200 steps, every 50, window 100)")
    ap.add_argument("--profile", action="store_true",
                    help="only the timed stream+collide steps (for rocprofv3 runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path "
              "(halo exchange over RCCL) is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl
    from paper_1906_11925_amd import LB

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.adjoint:
        log(f"[bench] adjoint workload only: {args.adjoint_workload}")
        out = adjoint_run(**ADJOINT_RUNS[args.adjoint_workload])
        print(json.dumps({k: v for k, v in out.items() if k != "dJ_dtheta"}), flush=True)
        return

    log(f"[bench] building workload {args.workload}")
    t0 = time.perf_counter()
    geom = wl.config_geometry(args.workload)
    n = geom.n_sites
    log(f"[bench] {n} sites ({time.perf_counter() - t0:.1f}s); creating handle")

    def maker(g):
        def make(storage, addressing=args.addressing, lattice=args.lattice):
            return LB.from_geometry(g, lattice=lattice, storage=storage, addressing=addressing)
        return make

    make = maker(geom)
    lb = make(args.storage)
    info = lb.info()
    if args.profile:
        lb.step(args.warmup)
        lb.sync()
        lb.step(args.steps)
        lb.sync()
        log(f"[bench] profile run done: {args.steps} steps")
        # counter calibration: plain copies of a known size (256 MiB each way)
        from paper_1906_11925_amd import copy_probe
        nb = 256 << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            copy_probe(b, a, nb)
        torch.cuda.synchronize()
        log(f"[bench] copy probe done: 3 x {nb} bytes")
        return

    log(f"[bench] timing {args.storage}: warmup {args.warmup}, steps {args.steps}")
    dt = timed_run(lb, args.steps, args.warmup, args.obs_every)
    glups = n * args.steps / dt / 1e9
    ms_step = dt / args.steps * 1e3
    avg_ms = region_kernel_ms(lb, args.steps, 10)
    launch_ms = kernel_avg_ms(lb, args.steps)
    bpu = info["bytes_per_update"]
    mb = method_bytes(args.lattice, args.storage)
    achieved = mb * n / (avg_ms * 1e-3) / 1e9
    achieved_own = bpu * n / (avg_ms * 1e-3) / 1e9
    log(f"[bench] {glups:.2f} GLUPS, {ms_step:.4f} ms/step, kernel {avg_ms:.4f} ms -> "
        f"{achieved:.0f} GB/s at {mb} B/update ({achieved_own:.0f} GB/s at the kernel's own "
        f"{bpu:.1f} B)")
    render = None if args.no_extra else render_run(lb, geom)
    elem = 4 if args.storage == "f32" else 2
    aux = aux_timings(lb, n, args.lattice, elem, info["bytes_per_update"])
    log(f"[bench] observables {aux['observables_ms']:.3f} ms, totals {aux['totals_ms_incl_sync']:.3f} ms")
    lb.close()

    pop_bytes = 2 * args.lattice * elem
    extra = {"bytes_per_update": bpu, "addressing": info["addressing_name"],
             "device_GB": info["device_bytes"] / 1e9,
             "kernel_avg_ms": avg_ms,
             "kernel_avg_ms_per_launch_events": launch_ms,
             "populations_only_GBs": pop_bytes * n / (avg_ms * 1e-3) / 1e9}
    # practical ceiling: plain device copy of the same byte count
    from paper_1906_11925_amd import copy_probe
    nbytes = int(bpu * n // 2 // 16) * 16
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        copy_probe(b, a, nbytes)
    torch.cuda.synchronize()
    reps = 50
    t0 = time.perf_counter()
    for _ in range(reps):
        copy_probe(b, a, nbytes)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * reps / (time.perf_counter() - t0) / 1e9
    extra["outputs"] = aux
    if render:
        extra["render"] = render
    extra["copy_GBs"] = copy_gbs
    extra["frac_of_copy_own_bytes"] = achieved_own / copy_gbs
    del a, b
    torch.cuda.empty_cache()
    if not args.no_extra:
        forms = {}
        for st in ("f16", "bf16"):
            if st != args.storage:
                forms[st] = form_timing(make, geom, st, args.steps, args.warmup,
                                        obs_every=args.obs_every)
                forms[st]["speedup_vs_" + args.storage] = ms_step / forms[st]["ms_per_step"]
                log(f"[bench] {st}: {forms[st]['GLUPS']:.2f} GLUPS")
        for st in ("f32", "f16"):
            # the addressing forms the default does not pick, for comparison
            for ad in ("blocks", "table16"):
                key = f"{st}_{ad}"
                forms[key] = form_timing(make, geom, st, args.steps, args.warmup, ad,
                                         obs_every=args.obs_every)
                log(f"[bench] {key}: {forms[key]['GLUPS']:.2f} GLUPS")
        if args.lattice == 15:
            # the paper's lattice on the same workload
            for st in ("f32", "f16"):
                key = "d3q19_" + st
                forms[key] = form_timing(make, geom, st, args.steps, args.warmup, lattice=19,
                                         obs_every=args.obs_every)
                log(f"[bench] D3Q19 {st}: {forms[key]['GLUPS']:.2f} GLUPS")
        extra["forms"] = forms
        log("[bench] 16-bit storage errors against FP32 storage on the same workload")
        extra["errors_16bit_vs_f32_same_workload"] = storage_errors(make, args.steps)
        log("[bench] storage errors vs oracle (pipe, 2000 steps)")
        extra["errors_vs_oracle_pipe2000"] = pipe_errors()
        small = wl.config_geometry("tree1024")
        mk_small = maker(small)
        extra["tree1024"] = {"sites": small.n_sites}
        for st in ("f32", "f16"):
            extra["tree1024"][st] = form_timing(mk_small, small, st, args.steps, args.warmup)
            log(f"[bench] tree1024 {st}: {extra['tree1024'][st]['GLUPS']:.2f} GLUPS")
        del small, mk_small
        if args.size_matched:
            big = wl.config_geometry("tree2048_400M")
            mk_big = maker(big)
            extra["tree2048_400M"] = {"sites": big.n_sites}
            for st in ("f32", "f16"):
                extra["tree2048_400M"][st] = form_timing(mk_big, big, st, 200, 20,
                                                         obs_every=args.obs_every)
                log(f"[bench] tree2048_400M {st}: {extra['tree2048_400M'][st]['GLUPS']:.2f} GLUPS")
            del big, mk_big
        for key, wname in (("adjoint", "aneurysm_half"), ("adjoint_tree1024", "tree1024")):
            log(f"[bench] adjoint workload {wname}")
            extra[key] = adjoint_run(**ADJOINT_RUNS[wname])
            log(f"[bench] adjoint {wname}: {extra[key]['adjoint_GLUPS']:.3f} GLUPS (reverse incl. "
                f"recompute), {extra[key]['recorded']['adjoint_GLUPS']:.3f} with every state recorded")

    cpu = None
    if args.cpu_sites > 0:
        log(f"[bench] cpu_baseline: oracle, {args.cpu_sites} sites, >= {args.cpu_seconds} s")
        cpu = cpu_baseline(geom, args.lattice, args.cpu_sites, args.cpu_seconds)

    traffic = traffic_for(args.workload, args.storage, info["addressing_name"])
    line = {
        "metric": METRIC,
        "value": glups,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": None,
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": args.workload, "sites": n, "lattice": f"D3Q{args.lattice}",
                   "storage": args.storage, "tau": geom.tau, "collision": "LBGK",
                   "walls": "halfway bounce-back", "addressing": info["addressing_name"],
                   "iolets": "Ladd velocity inlet + equilibrium pressure outlets",
                   "observables_every": args.obs_every},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_update": mb,
                     "own_bytes_per_update": bpu, "achieved_own_bytes": achieved_own,
                     "frac_own_bytes": achieved_own / HBM_PEAK_GBS},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
