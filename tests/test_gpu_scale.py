"""The size-matched tree of about 400M sites (395,245,440; 2048^3 box, root radius
256): more than 2^31 population elements per array, so every offset the kernels
form must be 64-bit.

At this size no oracle state fits beside the lattice, so the check is a property
that holds at any size: with the collision switched off (tau = infinity) one step
moves every stored value along its link, bit for bit.  Fluid link (s, i) with
upstream site s' receives population i of s'; a wall link receives the site's own
opposite population (halfway bounce-back).  Iolet links are covered by the smaller
parity tests.  The link codes are those of the oracle-pinned link builder, checked
here at 200,000 random sites plus the first and last 4,096 sites of the caller's
order, for the FP32 form (16-bit table) and the FP16 form (block addressing).
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from oracle import lattice as olat  # noqa: E402
from paper_1906_11925_amd import LB, links  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def big():
    _gpu()
    g = wl.config_geometry("tree2048_400M")
    print(f"tree2048_400M: {g.n_sites} sites", flush=True)
    coords, nbr = links(g.labels, g.shape, g.periodic, 15)
    return g, coords, nbr


@pytest.mark.parametrize("storage,addressing", [("f32", "table16"), ("f16", "blocks")],
                         ids=["f32-table16", "f16-blocks"])
def test_streaming_is_the_link_permutation_at_400M_sites(big, storage, addressing):
    g, coords, nbr = big
    n, q = g.n_sites, 15
    assert q * n > 2 ** 31
    lb = LB(nbr, math.inf, lattice=q, storage=storage, coords=coords, iolets=list(g.iolets),
            site_weight=g.site_weight(), addressing=addressing)
    assert lb.info()["addressing"] == {"table16": L.ADDR_TABLE16, "blocks": L.ADDR_BLOCKS}[addressing]
    gen = torch.Generator(device="cuda").manual_seed(23)
    d = torch.rand((q, n), generator=gen, device="cuda")
    d.sub_(0.5).mul_(2e-3)
    lb.set_deviations(d, t=0)
    del d
    src = lb.get_deviations()  # the stored values (16-bit rounding applied)
    lb.step(1)
    dst = lb.get_deviations()
    lb.close()
    del lb
    rng = np.random.default_rng(9)
    sites = np.unique(np.concatenate([rng.choice(n, 200000, replace=False),
                                      np.arange(4096), np.arange(n - 4096, n)]))
    code = nbr[sites]  # [S, Q] upstream codes in caller order
    opp = olat.get(q).opp
    s_t = torch.from_numpy(sites).cuda()
    assert torch.equal(dst[0, s_t], src[0, s_t])
    checked = 0
    for i in range(1, q):
        ci = code[:, i]
        fl = ci >= 0
        up = torch.from_numpy(ci[fl].astype(np.int64)).cuda()
        assert torch.equal(dst[i, s_t[fl]], src[i, up]), f"fluid links, direction {i}"
        wl_ = ci == -1
        assert torch.equal(dst[i, s_t[wl_]], src[opp[i], s_t[wl_]]), f"wall links, direction {i}"
        checked += int(fl.sum() + wl_.sum())
    print(f"{storage}: {checked} links checked bit for bit", flush=True)
    assert checked > 0.9 * (q - 1) * len(sites)
