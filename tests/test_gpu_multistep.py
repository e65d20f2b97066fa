"""Multi-step GPU runs against the FP64 oracle at the sizes and in the storage
forms the benchmark times.

Each case starts GPU and oracle from the same seeded state (deviations
U(-1e-3, 1e-3), rounded so that they are exact in every storage compared),
runs both for a number of steps with the workload's own boundary conditions
(pulsatile Ladd inlet, pressure outlets, halfway walls), and compares the
observables with the error metric used throughout: max_s |x - x_ref| /
max_s |x_ref| for velocity (as a vector), pressure deviation and wall shear
stress.  Bounds: FP32 storage <= 1e-5, FP16 storage <= 2e-3; BF16 (8-bit
mantissa) is reported with a looser bound of 3e-2.  Every GPU run uses the
default addressing (block addressing on these workloads), as the benchmark does.

* the full-size aneurysm (1,590,840 sites), 100 steps: FP32 and FP16;
* the Murray tree in a 1024^3 box (5,598,432 sites), 50 steps: FP32, FP16, BF16;
* the straight pipe in D3Q19 (the paper's lattice), 2000 steps from rest, FP16
  and BF16 (FP32 over 500 steps is in test_gpu_parity.py).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from oracle.lbgk import LBGK  # noqa: E402
from paper_1906_11925_amd import LB  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

from lbtest import quantize, rel_max, rel_l2  # noqa: E402

pytestmark = pytest.mark.gpu

BOUND = {"f32": 1e-5, "f16": 2e-3, "bf16": 3e-2}


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _common_start(q, n, seed):
    """Deviations exactly representable in FP32, FP16 and BF16 storage alike
    (a value that one of the 16-bit roundings would move is set to zero)."""
    d = quantize(wl.random_deviations(q, n, seed, 1e-3), q, "bf16")
    d16 = quantize(d, q, "f16")
    d = np.where(d16 == d, d, 0.0)
    for st in ("f32", "f16", "bf16"):
        assert np.array_equal(quantize(d, q, st), d)
    return d


def _oracle_run(g, q, steps, seed):
    o = LBGK(g, q)
    d = _common_start(q, o.n, seed)
    A, f = o.run(o.lat.w[:, None] + d, 0, steps)
    p, u, _, w = o.observables(f)
    return d, (p - 1.0 / 3.0, u.T, w)


def _gpu_run(g, q, storage, d, steps):
    lb = LB.from_geometry(g, lattice=q, storage=storage)
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    if d is not None:
        lb.set_deviations(torch.from_numpy(d), t=0)
    lb.step(steps)
    out = [x.cpu().numpy().astype(np.float64) for x in lb.observables()]
    lb.close()
    return out


def _compare(tag, got, ref, storage):
    (p, u, w), (op, ou, ow) = got, ref
    eu, ep, ew = rel_max(u, ou), rel_max(p, op), rel_max(w, ow)
    print(f"{tag} {storage}: e_u={eu:.3e} e_p={ep:.3e} e_wss={ew:.3e} "
          f"l2_u={rel_l2(u, ou):.3e}", flush=True)
    tol = BOUND[storage]
    assert eu <= tol and ep <= tol and ew <= tol


@pytest.fixture(scope="module")
def aneurysm_ref():
    g = wl.config_geometry("aneurysm")
    d, ref = _oracle_run(g, 15, 100, seed=31)
    return g, d, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_aneurysm_100_steps_vs_oracle(aneurysm_ref, storage):
    _gpu()
    g, d, ref = aneurysm_ref
    _compare(f"aneurysm ({g.n_sites} sites, 100 steps)", _gpu_run(g, 15, storage, d, 100), ref,
             storage)


@pytest.fixture(scope="module")
def tree1024_ref():
    g = wl.config_geometry("tree1024")
    d, ref = _oracle_run(g, 15, 50, seed=33)
    return g, d, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_tree1024_50_steps_vs_oracle(tree1024_ref, storage):
    _gpu()
    g, d, ref = tree1024_ref
    _compare(f"tree1024 ({g.n_sites} sites, 50 steps)", _gpu_run(g, 15, storage, d, 50), ref,
             storage)


@pytest.fixture(scope="module")
def pipe19_ref():
    g = wl.pipe()
    o = LBGK(g, 19)
    A, f = o.run(o.rest_state(), 0, 2000)
    p, u, _, w = o.observables(f)
    return g, (p - 1.0 / 3.0, u.T, w)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_pipe_d3q19_2000_steps_16bit_vs_oracle(pipe19_ref, storage):
    _gpu()
    g, ref = pipe19_ref
    _compare("pipe D3Q19 (2000 steps)", _gpu_run(g, 19, storage, None, 2000), ref, storage)
