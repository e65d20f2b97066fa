"""hemelb_lb_totals_noalloc (the totals for callers that cannot allocate: partial
sums in a per-GPU static scratch array) gives the bits of hemelb_lb_totals, on two
calls in a row, the second on a smaller lattice (the scratch keeps the first
call's contents; the second call must not depend on them)."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from paper_1906_11925_amd import LB  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(g, seed):
    lb = LB.from_geometry(g)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    d = (torch.rand((lb.q, lb.n), generator=gen, device="cuda") - 0.5) * 2e-3
    lb.set_deviations(d, t=0)
    lb.step(5)
    ref = lb.totals()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    rc = L.load().hemelb_lb_totals_noalloc(lb.h, ctypes.c_void_p(out.data_ptr()))
    assert rc == L.HEMELB_OK, L.last_error()
    lb.sync()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    lb.close()
    return ref, got


def test_totals_noalloc_matches_totals_twice_shrinking():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for g, seed in ((wl.aneurysm(half=True), 3), (wl.pipe(), 4)):
        ref, got = _run(g, seed)
        print(f"{g.name}: {g.n_sites} sites, totals {got}", flush=True)
        assert np.array_equal(got, ref), (got, ref)


def test_totals_noalloc_rejects_null():
    lib = L.load()
    assert lib.hemelb_lb_totals_noalloc(None, None) == L.HEMELB_EINVAL
