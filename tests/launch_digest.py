"""Digest of a short run of the library in one launch mode, for the launch-mode
test (tests/test_gpu_launch_modes.py).

The run: the half aneurysm (D3Q15, pulsatile Ladd inlet, pressure outlets) from
seeded deviations U(-1e-3, 1e-3), `steps` steps, then the raw state, the
observables and the FP64 totals, hashed together.  Modes:
  async   one call for all steps, one synchronisation at the end;
  sync    one call and one synchronisation per step;
  stream  as async, on a stream other than the default one.
Run as a script it prints the digest of the async mode as one JSON line, which
lets the test repeat the run in a process with a different HIP environment.
"""

import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def digest(storage, steps=200, mode="async"):
    import torch
    import workloads as wl
    from paper_1906_11925_amd import LB

    g = wl.aneurysm(half=True)
    d = torch.from_numpy(wl.random_deviations(15, g.n_sites, 41, 1e-3))

    def run():
        lb = LB.from_geometry(g, lattice=15, storage=storage)
        lb.set_deviations(d, t=0)
        if mode == "sync":
            for _ in range(steps):
                lb.step(1)
                lb.sync()
        else:
            lb.step(steps)
            lb.sync()
        raw = lb.get_state()[0]
        if raw.dtype == torch.bfloat16:
            raw = raw.view(torch.int16)
        parts = [raw.cpu().numpy().tobytes()]
        parts += [x.cpu().numpy().tobytes() for x in lb.observables()]
        parts.append(lb.totals().tobytes())
        lb.close()
        return hashlib.sha256(b"".join(parts)).hexdigest()

    if mode == "stream":
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            h = run()
        torch.cuda.synchronize()
        return h
    return run()


if __name__ == "__main__":
    storage = sys.argv[1]
    steps = int(sys.argv[2])
    print(json.dumps({"storage": storage, "steps": steps, "digest": digest(storage, steps)}),
          flush=True)
