"""GPU path (HIP kernels through the C ABI) against the FP64 oracle.

Bit-exact pins: the rest equilibrium stays exactly zero deviation; with the
collision switched off (tau = infinity) a step is a pure permutation of the
stored values, identical to the oracle's streaming; results do not depend on
the site order given to the library; checkpoint/restore is exact.

Toleranced pins (FP32 arithmetic vs FP64): one step from a random state,
element by element; multi-step runs compared on the observables with the
error metric max_s |x_gpu - x_ref| / max_s |x_ref| (velocity as a vector, and
pressure deviation and wall shear stress likewise): FP32 storage <= 1e-5,
FP16 storage <= 2e-3 after the run.
"""

import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from workloads.geometry import Geometry, Iolet  # noqa: E402
from oracle.lbgk import LBGK  # noqa: E402
from oracle import lattice as olat  # noqa: E402
from paper_1906_11925_amd import LB, HemelbError  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

from lbtest import quantize, rel_max, rel_l2, SCALES  # noqa: E402

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(lb):
    return lb.get_deviations().cpu().numpy().astype(np.float64)


def _walls_only(g):
    lab = g.labels.copy()
    lab[lab >= 2] = 0
    return Geometry(g.name + "_walls", g.shape, lab, periodic=g.periodic, iolets=[], tau=g.tau)


def _still(g):
    ios = [Iolet(io.kind, direction=io.direction, mean=(1.0 if io.kind == "pressure" else 0.0))
           for io in g.iolets]
    return Geometry(g.name + "_still", g.shape, g.labels, periodic=g.periodic, iolets=ios,
                    tau=g.tau, profile=g.profile)


STORAGES = ["f32", "f16", "bf16"]


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("storage", STORAGES)
def test_rest_state_stays_exact(storage, q):
    _gpu()
    for g in (_still(wl.pipe()), _still(wl.aneurysm(half=True)), wl.couette(U=0.0)):
        lb = LB.from_geometry(g, lattice=q, storage=storage)
        lb.step(7)
        raw, t = lb.get_state()
        assert t == 7
        assert torch.count_nonzero(raw.float()) == 0
        p, u, w = lb.observables()
        assert torch.count_nonzero(p) == 0 and torch.count_nonzero(u) == 0
        assert torch.count_nonzero(w) == 0
        lb.close()


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("name", ["closed", "periodic", "pipe_walls", "tree_walls"])
def test_no_collision_is_exact_permutation(name, storage, q):
    """tau = infinity: each step only moves stored values; identical to the
    oracle's pull streaming applied to the same values."""
    _gpu()
    g = {"closed": lambda: wl.closed_box(7, 6, 5), "periodic": lambda: wl.periodic_box(5, 7, 6),
         "pipe_walls": lambda: _walls_only(wl.pipe()),
         "tree_walls": lambda: _walls_only(
             wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1))}[name]()
    o = LBGK(g, q, tau=math.inf)
    d = quantize(wl.random_deviations(q, o.n, 21, 1e-2), q, storage)
    lb = LB.from_geometry(g, lattice=q, storage=storage, tau=math.inf)
    lb.set_deviations(torch.from_numpy(d))
    ref = d
    for t in range(3):
        ref = o.stream(ref, t)
    lb.step(3)
    assert np.array_equal(_dev(lb), ref)
    lb.close()


def fp32_tol(q, amp):
    """Bound on the FP32 error of one step from deviations of size <= amp.

    Summing q terms of size <= amp in FP32 errs by at most (q-1) u sum|d_i|
    <= q^2 amp u (u = 2^-24); the equilibrium and collision reuse these sums
    with O(1) factors, hence 2 q^2 amp u for deviations, velocity and stress
    (and a third of it for the pressure deviation drho/3).  A wrong term, sign
    or weight shows up at the size of w_i * amp ~ 1e-5..1e-4, far above this.
    """
    return 2.0 * q * q * amp * 2.0 ** -24


def _one_step_case(g, q, storage, seed, amp=1e-3, tau=None, alpha=None):
    o = LBGK(g, q, tau=tau, alpha=alpha)
    d = quantize(wl.random_deviations(q, o.n, seed, amp), q, storage)
    t0 = 37
    lb = LB.from_geometry(g, lattice=q, storage=storage, tau=tau,
                          alpha=None if alpha is None else alpha.astype(np.float32))
    lb.set_deviations(torch.from_numpy(d), t=t0)
    lb.step(1)
    gpu = _dev(lb)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    A, f = o.step(o.lat.w[:, None] + d, t0)
    ref = A - o.lat.w[:, None]
    op, ou, _, ow = o.observables(f)
    lb.close()
    return gpu, ref, (p, u, w), (op - 1.0 / 3.0, ou.T, ow), o


@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "couette", "channel", "tree_small"])
def test_one_step_f32_elementwise(name, q):
    _gpu()
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "couette": wl.couette, "channel": wl.channel,
         "tree_small": lambda: wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3,
                                       seed=1)}[name]()
    gpu, ref, (p, u, w), (op, ou, ow), _ = _one_step_case(g, q, "f32", seed=5)
    tol = fp32_tol(q, 1e-3)
    assert np.abs(gpu - ref).max() < tol
    assert np.abs(p - op).max() < tol / 3
    assert np.abs(u - ou).max() < tol
    assert np.abs(w - ow).max() < tol


def _tol16(o, ref, f, storage, q, scaled=True):
    """Bound on one 16-bit step (see test_one_step_16bit_elementwise): the output
    rounding, FP32 collision error, and the rounding of the incoming iolet values
    at iolet sites.  Returns (bound, bound without the iolet term, sites without
    iolet links)."""
    ulp = 2.0 ** -11 if storage == "f16" else 2.0 ** -8
    s = SCALES[q][:, None] if scaled else np.ones((q, 1))
    sub = 2.0 ** -25 / s if storage == "f16" else 0.0 * s
    ghost = o.links.kind == 2
    g_err = np.where(ghost, ulp * np.abs(f - o.lat.w[:, None]) + sub, 0.0).sum(axis=0)
    plain_tol = ulp * np.abs(ref) + sub + fp32_tol(q, 1e-3)
    return plain_tol + 3.0 * g_err[None, :], plain_tol, ~ghost.any(axis=0)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_one_step_16bit_elementwise(storage):
    """16-bit storage: the input is exact, one FP32 collision follows, then one
    rounding of d * scale (relative half-ulp 2^-11 for FP16, 2^-8 for BF16).
    Incoming populations at iolet links are stored in the same format, so
    their rounding (bounded with the oracle's ghost values) also enters the
    collision of their site, with a Jacobian of norm below 3."""
    _gpu()
    q = 15
    g = wl.aneurysm(half=True)
    o = LBGK(g, q)
    d = quantize(wl.random_deviations(q, o.n, 6, 1e-3), q, storage)
    lb = LB.from_geometry(g, lattice=q, storage=storage)
    lb.set_deviations(torch.from_numpy(d), t=37)
    lb.step(1)
    gpu = _dev(lb)
    lb.close()
    A, f = o.step(o.lat.w[:, None] + d, 37)
    ref = A - o.lat.w[:, None]
    tol, plain_tol, plain = _tol16(o, ref, f, storage, q)
    assert np.all(np.abs(gpu - ref) <= tol)
    # away from iolets the bound is the plain rounding bound
    assert np.all(np.abs(gpu - ref)[:, plain] <= plain_tol[:, plain])


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_one_step_16bit_unscaled_elementwise(storage):
    """16-bit storage without the power-of-two scale (HEMELB_FLAG_NO_SCALE): the
    same bound with scale 1, where FP16 keeps small deviations only as
    subnormals (half-spacing 2^-25)."""
    _gpu()
    q = 15
    g = wl.aneurysm(half=True)
    o = LBGK(g, q)
    d = quantize(wl.random_deviations(q, o.n, 6, 1e-3), q, storage, scale=False)
    lb = LB.from_geometry(g, lattice=q, storage=storage, scale=False)
    lb.set_deviations(torch.from_numpy(d), t=37)
    lb.step(1)
    gpu = _dev(lb)
    lb.close()
    A, f = o.step(o.lat.w[:, None] + d, 37)
    ref = A - o.lat.w[:, None]
    tol, plain_tol, plain = _tol16(o, ref, f, storage, q, scaled=False)
    assert np.all(np.abs(gpu - ref) <= tol)
    assert np.all(np.abs(gpu - ref)[:, plain] <= plain_tol[:, plain])


def test_one_step_brinkman_alpha():
    _gpu()
    g = wl.aneurysm(half=True)
    n = g.n_sites
    alpha = np.random.default_rng(4).uniform(0.0, 0.01, n)
    alpha = alpha.astype(np.float32).astype(np.float64)
    gpu, ref, _, _, _ = _one_step_case(g, 15, "f32", seed=8, alpha=alpha)
    assert np.abs(gpu - ref).max() < fp32_tol(15, 1e-3)


def test_site_order_invariance_bit_exact():
    """Morton-ordered and caller-ordered runs give identical bits."""
    _gpu()
    g = wl.aneurysm(half=True)
    from paper_1906_11925_amd import links
    coords, nbr = links(g.labels, g.shape, g.periodic, 15)
    a = LB(nbr, g.tau, coords=coords, iolets=g.iolets, site_weight=g.site_weight())
    b = LB(nbr, g.tau, coords=None, iolets=g.iolets, site_weight=g.site_weight())
    d = torch.from_numpy(quantize(wl.random_deviations(15, g.n_sites, 3, 1e-3), 15, "f32"))
    for lb in (a, b):
        lb.set_deviations(d)
        lb.step(20)
    sa, sb = a.get_state()[0], b.get_state()[0]
    assert torch.equal(sa, sb)
    for x, y in zip(a.observables(), b.observables()):
        assert torch.equal(x, y)


def test_checkpoint_restart_bit_exact():
    _gpu()
    g = wl.aneurysm(half=True)
    a = LB.from_geometry(g, storage="f16")
    a.step(40)
    b = LB.from_geometry(g, storage="f16")
    b.step(20)
    st, t = b.get_state()
    c = LB.from_geometry(g, storage="f16")
    c.set_state(st.clone(), t)
    c.step(20)
    assert c.time == 40
    assert torch.equal(a.get_state()[0], c.get_state()[0])


def test_determinism():
    _gpu()
    g = wl.pipe()
    runs = []
    for _ in range(2):
        lb = LB.from_geometry(g)
        lb.step(50)
        runs.append((lb.get_state()[0], lb.totals()))
    assert torch.equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


@pytest.fixture(scope="module")
def pipe_oracle():
    g = wl.pipe()
    o = LBGK(g, 15)
    A, f = o.run(o.rest_state(), 0, 2000)
    p, u, _, w = o.observables(f)
    return g, A, (p - 1.0 / 3.0, u.T, w)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16", 2e-3)])
def test_pipe_2000_steps_vs_oracle(pipe_oracle, storage, tol):
    """Straight pipe, D3Q15, tau = 0.8, pressure iolets, 2000 steps from rest."""
    _gpu()
    g, A, (op, ou, ow) = pipe_oracle
    lb = LB.from_geometry(g, storage=storage)
    lb.step(2000)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    eu, ep, ew = rel_max(u, ou), rel_max(p, op), rel_max(w, ow)
    print(f"pipe {storage}: e_u={eu:.3e} e_p={ep:.3e} e_wss={ew:.3e} "
          f"l2_u={rel_l2(u, ou):.3e}", flush=True)
    assert eu <= tol and ep <= tol and ew <= tol


def test_pipe_bf16_error_reported(pipe_oracle):
    _gpu()
    g, A, (op, ou, ow) = pipe_oracle
    lb = LB.from_geometry(g, storage="bf16")
    lb.step(2000)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    eu = rel_max(u, ou)
    print(f"pipe bf16: e_u={eu:.3e} e_p={rel_max(p, op):.3e} e_wss={rel_max(w, ow):.3e}", flush=True)
    assert eu < 5e-2


def test_aneurysm_half_pulsatile_vs_oracle():
    """Half-size aneurysm with the pulsatile Ladd inlet, 200 steps from rest."""
    _gpu()
    g = wl.aneurysm(half=True)
    o = LBGK(g, 15)
    A, f = o.run(o.rest_state(), 0, 200)
    op, ou, _, ow = o.observables(f)
    lb = LB.from_geometry(g)
    lb.step(200)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    eu, ep, ew = rel_max(u, ou.T), rel_max(p, op - 1 / 3), rel_max(w, ow)
    print(f"aneurysm_half f32: e_u={eu:.3e} e_p={ep:.3e} e_wss={ew:.3e}", flush=True)
    assert eu <= 1e-5 and ep <= 1e-5 and ew <= 1e-5


def test_pipe_d3q19_vs_oracle():
    _gpu()
    g = wl.pipe()
    o = LBGK(g, 19)
    A, f = o.run(o.rest_state(), 0, 500)
    op, ou, _, ow = o.observables(f)
    lb = LB.from_geometry(g, lattice=19)
    lb.step(500)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    assert rel_max(u, ou.T) <= 1e-5 and rel_max(p, op - 1 / 3) <= 1e-5 and rel_max(w, ow) <= 1e-5


def test_couette_wss_closed_form():
    _gpu()
    H, U, tau = 8, 0.01, 1.0
    g = wl.couette(H=H, Lx=2, Lz=2, U=U, tau=tau)
    lb = LB.from_geometry(g)
    lb.step(1200)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    y = g.coords[:, 1]
    nu = (tau - 0.5) / 3
    assert np.abs(u[:, 0] - U * (y + 0.5) / H).max() / U < 1e-5
    np.testing.assert_allclose(w[y == 0], nu * U / H, rtol=1e-4)


def test_observables_at_time_zero_use_stored_state():
    _gpu()
    g = wl.pipe()
    o = LBGK(g, 15)
    d = quantize(wl.random_deviations(15, o.n, 9, 1e-3), 15, "f32")
    lb = LB.from_geometry(g)
    lb.set_deviations(torch.from_numpy(d), t=5)
    p, u, w = (x.cpu().numpy().astype(np.float64) for x in lb.observables())
    op, ou, _, ow = o.observables(o.lat.w[:, None] + d)
    assert np.abs(p - (op - 1 / 3)).max() < 1e-9
    assert np.abs(u - ou.T).max() < 1e-8


def test_totals_and_mass_conservation():
    _gpu()
    g = wl.closed_box(9, 8, 7)
    o = LBGK(g, 15, tau=0.55)
    d = quantize(wl.random_deviations(15, o.n, 12, 5e-4), 15, "f32")
    lb = LB.from_geometry(g, tau=0.55)
    lb.set_deviations(torch.from_numpy(d))
    t0 = lb.totals()
    m, mom = o.totals(o.lat.w[:, None] + d)
    assert abs(t0[0] - m) < 1e-9 and np.abs(t0[1:] - mom).max() < 1e-12
    lb.step(1000)
    t1 = lb.totals()
    print(f"closed box FP32 mass drift over 1000 steps: {(t1[0] - t0[0]) / t0[0]:.3e}", flush=True)
    assert abs(t1[0] - t0[0]) / t0[0] < 1e-6


def test_divergence_check_reports_nonfinite():
    _gpu()
    g = wl.closed_box(5, 5, 5)
    lb = LB.from_geometry(g)
    d = np.zeros((15, g.n_sites))
    d[3, 10] = np.nan
    lb.set_deviations(torch.from_numpy(d))
    lb.set_check(2)
    lb.step(4)
    with pytest.raises(HemelbError) as ei:
        lb.sync()
    assert ei.value.code == L.HEMELB_EDIVERGED


def test_empty_geometry():
    _gpu()
    lb = LB(np.zeros((0, 15), dtype=np.int32), 0.7)
    lb.step(3)
    p, u, w = lb.observables()
    assert p.numel() == 0
    assert lb.totals()[0] == 0.0
    lb.close()


def test_cancel_stops_step_request():
    _gpu()
    lb = LB.from_geometry(wl.closed_box(4, 4, 4))
    lb.cancel()
    with pytest.raises(HemelbError) as ei:
        lb.step(5)
    assert ei.value.code == L.HEMELB_ECANCELLED
    lb.step(2)
    assert lb.time == 2


def test_kernel_timing_counts_launches():
    _gpu()
    lb = LB.from_geometry(wl.pipe())
    lb.kernel_timing(10)
    lb.step(10)
    ms, k = lb.kernel_time()
    assert k == 10 and ms > 0


@pytest.mark.parametrize("name", ["aneurysm", "tree1024"])
def test_full_size_one_step(name):
    """Full-size workloads, launched as the benchmark launches them: one step
    from a random state compared element by element with the oracle."""
    _gpu()
    g = wl.config_geometry(name)
    gpu, ref, (p, u, w), (op, ou, ow), o = _one_step_case(g, 15, "f32", seed=13)
    print(f"{name}: {o.n} sites", flush=True)
    assert np.abs(gpu - ref).max() < fp32_tol(15, 1e-3)
    assert np.abs(u - ou).max() < fp32_tol(15, 1e-3)


@pytest.mark.parametrize("name", ["aneurysm", "tree1024"])
def test_full_size_one_step_16bit_blocks(name):
    """The FP16 form the benchmark times (block addressing) on the full-size
    workloads: one step from a random state, element by element, to the 16-bit
    bound."""
    _gpu()
    q, storage = 15, "f16"
    g = wl.config_geometry(name)
    o = LBGK(g, q)
    d = quantize(wl.random_deviations(q, o.n, 13, 1e-3), q, storage)
    lb = LB.from_geometry(g, lattice=q, storage=storage)
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    lb.set_deviations(torch.from_numpy(d), t=37)
    lb.step(1)
    gpu = _dev(lb)
    lb.close()
    A, f = o.step(o.lat.w[:, None] + d, 37)
    ref = A - o.lat.w[:, None]
    tol, _, _ = _tol16(o, ref, f, storage, q)
    print(f"{name} f16 blocks: {o.n} sites, worst |err|/tol {np.max(np.abs(gpu - ref) / tol):.3f}",
          flush=True)
    assert np.all(np.abs(gpu - ref) <= tol)


@pytest.fixture(scope="module")
def tree2048():
    return wl.config_geometry("tree2048")


@pytest.mark.parametrize("q", [15, 19])
def test_tree2048_one_step_sampled_16bit_blocks(tree2048, q):
    """The largest workload in FP16 storage with block addressing: one step,
    compared with the oracle's sampled step at 20,000 random sites."""
    _gpu()
    g = tree2048
    n = g.n_sites
    d = quantize(wl.random_deviations(q, n, 19, 1e-3), q, "f16")
    lb = LB.from_geometry(g, lattice=q, storage="f16")
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    lb.set_deviations(torch.from_numpy(d.astype(np.float32)), t=11)
    lb.step(1)
    sites = np.sort(np.random.default_rng(6).choice(n, 20000, replace=False))
    gpu = lb.get_deviations()[:, torch.from_numpy(sites).cuda()].cpu().numpy().astype(np.float64)
    lb.close()
    o = LBGK(g, q, sites=sites)
    A, f = o.step(o.lat.w[:, None] + d.astype(np.float64), 11)
    ref = A - o.lat.w[:, None]
    tol, _, _ = _tol16(o, ref, f, "f16", q)
    assert np.all(np.abs(gpu - ref) <= tol)


@pytest.mark.parametrize("q", [15, 19])
def test_tree2048_one_step_sampled(tree2048, q):
    """The largest workload (seeded Murray tree in a 2048^3 box, 53,020,072
    sites): one step from a random state on the GPU, compared with the oracle's
    sampled step at 20,000 random sites (and all their populations)."""
    _gpu()
    g = tree2048
    n = g.n_sites
    print(f"tree2048 D3Q{q}: {n} sites", flush=True)
    d = wl.random_deviations(q, n, 17, 1e-3).astype(np.float32)
    lb = LB.from_geometry(g, lattice=q)
    lb.set_deviations(torch.from_numpy(d), t=11)
    lb.step(1)
    sites = np.sort(np.random.default_rng(5).choice(n, 20000, replace=False))
    gpu = lb.get_deviations()[:, torch.from_numpy(sites).cuda()].cpu().numpy().astype(np.float64)
    lb.close()
    o = LBGK(g, q, sites=sites)
    A, _ = o.step(o.lat.w[:, None] + d.astype(np.float64), 11)
    ref = A - o.lat.w[:, None]
    assert np.abs(gpu - ref).max() < fp32_tol(q, 1e-3)


def _tree_small():
    return wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1)


def _iolet_only_site():
    around = [((x, y, z), 0) for x in range(-1, 4) for y in range(-1, 4) for z in range(-1, 4)
              if (x, y, z) != (1, 1, 1) and max(abs(x - 1), abs(y - 1), abs(z - 1)) == 1]
    return _lattice_box((3, 3, 3), [(1, 1, 1)], around, tau=0.8,
                        iolets=[Iolet("pressure", mean=1.002)])


ADDR = {"blocks": L.ADDR_BLOCKS, "table16": L.ADDR_TABLE16, "table32": L.ADDR_TABLE32}


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("name", ["pipe", "aneurysm_half", "tree_small", "iolet_only_site"])
def test_addressing_modes_are_bit_identical(name, q, storage):
    """Block addressing, the 16-bit table and the int32 table find the same
    upstream populations: identical bits after 30 steps from a random state
    (pressure and Ladd iolets, walls), observables too.  Block addressing shares
    one ghost cell among the links that pull from one position, so it needs no
    more ghost slots, and it reads fewer addressing bytes."""
    _gpu()
    g = {"pipe": wl.pipe, "aneurysm_half": lambda: wl.aneurysm(half=True),
         "tree_small": _tree_small, "iolet_only_site": _iolet_only_site}[name]()
    d = torch.from_numpy(quantize(wl.random_deviations(q, g.n_sites, 3, 1e-3), q, storage))
    runs = {}
    for mode in ("blocks", "table16", "table32"):
        lb = LB.from_geometry(g, lattice=q, storage=storage, addressing=mode)
        info = lb.info()
        assert info["addressing"] == ADDR[mode]
        lb.set_deviations(d, t=5)
        lb.step(30)
        runs[mode] = (lb.get_state()[0], lb.observables(), info)
        lb.close()
    for mode in ("table16", "table32"):
        assert torch.equal(runs["blocks"][0], runs[mode][0])
        for x, y in zip(runs["blocks"][1], runs[mode][1]):
            assert torch.equal(x, y)
    ib, i16, i32 = (runs[m][2] for m in ("blocks", "table16", "table32"))
    assert ib["n_ghosts"] == i16["n_ghosts"] == i32["n_ghosts"]
    assert ib["pitch"] <= i16["pitch"] == i32["pitch"]
    pops = 2 * q * (4 if storage == "f32" else 2)
    assert i32["bytes_per_update"] == pops + 4 * (q - 1)
    if name != "iolet_only_site":  # per-tile and per-block terms dominate a 1-site lattice
        assert i16["bytes_per_update"] < pops + 2 * (q - 1) + 4
        assert ib["bytes_per_update"] < pops + 8


def test_auto_addressing_prefers_blocks_and_falls_back():
    """The default is block addressing (with coordinates and halfway walls) in
    every storage; a periodic lattice (links that wrap) and interpolated walls use
    the table; asking for blocks where they do not apply is an error that names
    the reason."""
    _gpu()
    lb = LB.from_geometry(wl.pipe(), storage="f16")
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    lb.close()
    lb = LB.from_geometry(wl.pipe())
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    lb.close()
    per = wl.periodic_box(5, 7, 6)
    lb = LB.from_geometry(per, storage="f16")
    assert lb.info()["addressing"] == L.ADDR_TABLE16
    lb.close()
    with pytest.raises(HemelbError) as ei:
        LB.from_geometry(per, addressing="blocks")
    assert ei.value.code == L.HEMELB_EINVAL and "block addressing" in str(ei.value)
    with pytest.raises(HemelbError) as ei:
        LB.from_geometry(wl.pipe(), addressing="blocks", bfl=True)
    assert ei.value.code == L.HEMELB_EINVAL and "interpolated" in str(ei.value)
    lb = LB.from_geometry(wl.pipe(), bfl=True, storage="f16")
    assert lb.info()["addressing"] == L.ADDR_TABLE16
    lb.close()


def _lattice_box(shape, fluid_pts, iolet_pts=(), periodic=(False, False, False), tau=0.7,
                 iolets=()):
    lab = np.zeros(tuple(a + 2 for a in shape), dtype=np.uint8)
    for p in fluid_pts:
        lab[p[0] + 1, p[1] + 1, p[2] + 1] = 1
    for p, k in iolet_pts:
        lab[p[0] + 1, p[1] + 1, p[2] + 1] = 2 + k
    return Geometry("edge", tuple(shape), lab, periodic=periodic, iolets=list(iolets), tau=tau)


@pytest.mark.parametrize("count", [1, 63, 65, 127])
def test_ragged_site_counts(count):
    """Site counts that do not fill the last 64-site tile (and a single site)."""
    _gpu()
    rng = np.random.default_rng(count)
    pts = set()
    while len(pts) < count:
        pts.add(tuple(int(v) for v in rng.integers(0, 9, 3)))
    g = _lattice_box((9, 9, 9), sorted(pts), tau=0.65)
    assert g.n_sites == count
    for q in (15, 19):
        gpu, ref, (p, u, w), (op, ou, ow), _ = _one_step_case(g, q, "f32", seed=count)
        assert np.abs(gpu - ref).max() < fp32_tol(q, 1e-3)
        assert np.abs(w - ow).max() < fp32_tol(q, 1e-3)


def test_isolated_site_is_pure_bounce_back():
    """A single fluid site enclosed by walls: every population bounces back, so
    after two steps with tau = infinity the state returns exactly."""
    _gpu()
    g = _lattice_box((3, 3, 3), [(1, 1, 1)], tau=math.inf)
    d = quantize(wl.random_deviations(15, 1, 2, 1e-2), 15, "f32")
    lb = LB.from_geometry(g, tau=math.inf)
    lb.set_deviations(torch.from_numpy(d))
    lb.step(1)
    once = _dev(lb)
    o = LBGK(g, 15)
    assert np.array_equal(once, d[o.lat.opp])
    lb.step(1)
    assert np.array_equal(_dev(lb), d)


def test_site_with_only_iolet_links():
    """A single site whose every upstream point lies past a pressure iolet."""
    _gpu()
    shape = (3, 3, 3)
    around = [((x, y, z), 0) for x in range(-1, 4) for y in range(-1, 4) for z in range(-1, 4)
              if (x, y, z) != (1, 1, 1) and max(abs(x - 1), abs(y - 1), abs(z - 1)) == 1]
    g = _lattice_box(shape, [(1, 1, 1)], around, tau=0.8, iolets=[Iolet("pressure", mean=1.002)])
    for q in (15, 19):
        gpu, ref, _, _, _ = _one_step_case(g, q, "f32", seed=3)
        assert np.abs(gpu - ref).max() < fp32_tol(q, 2e-3)


@pytest.mark.parametrize("tau", [0.5000001, 0.51, 50.0, 1e6])
def test_extreme_relaxation_times(tau):
    _gpu()
    g = wl.aneurysm(half=True)
    gpu, ref, _, _, _ = _one_step_case(g, 15, "f32", seed=21, tau=tau)
    assert np.abs(gpu - ref).max() < fp32_tol(15, 1e-3)


def test_restore_and_continue_is_exact_over_a_pulsatile_run():
    """A state restored from a checkpoint continues exactly as the run that
    produced it: the ghost fill after a restore and the ghost values the step
    kernel writes for the next step are the same bits (pulsatile Ladd inlet,
    pressure outlet, Brinkman field), at every 200-step checkpoint of 2000 steps."""
    _gpu()
    g = wl.aneurysm(half=True)
    n = g.n_sites
    alpha = np.random.default_rng(4).uniform(0.0, 0.01, n).astype(np.float32)
    a = LB.from_geometry(g, alpha=alpha)
    b = LB.from_geometry(g, alpha=alpha)
    a.set_deviations(torch.zeros((a.q, n), dtype=torch.float32, device="cuda"), t=0)
    states = [a.get_state()[0].clone()]
    for _ in range(10):
        a.step(200)
        states.append(a.get_state()[0].clone())
    bad = []
    for k in range(10):
        b.set_state(states[k].clone(), 200 * k)
        b.step(200)
        if not torch.equal(b.get_state()[0], states[k + 1]):
            bad.append(200 * k)
    assert not bad, f"restored runs differ from t = {bad}"


def test_host_call_before_torch_in_a_fresh_process():
    """A program that calls the host library (links) before it ever imports
    torch still steps on the GPU: the library binds to torch's HIP runtime."""
    _gpu()
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import workloads as wl\n"
        "from paper_1906_11925_amd import links, LB\n"
        "g = wl.pipe(); coords, nbr = links(g.labels, g.shape, g.periodic, 15)\n"
        "lb = LB(nbr, g.tau, coords=coords, iolets=list(g.iolets), site_weight=g.site_weight())\n"
        "lb.step(10); p, u, w = lb.observables(); print(float(u.abs().max()))\n" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert float(r.stdout.strip().splitlines()[-1]) > 0
