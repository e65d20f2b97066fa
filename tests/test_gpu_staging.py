"""The staged forms of the step give the same bits as the plain four-tile kernel.

With block addressing, a workgroup of W tiles (W = 4, 8 or 16) may first copy its
own tiles' populations into LDS, by loads that write LDS directly or through
registers; pulls from inside the workgroup then read LDS.  The arithmetic is that
of the unstaged kernel, so every form must give the same raw state bit for bit.
Forms are chosen per handle at creation (HEMELB_STAGE_TILES, HEMELB_LDS_DMA).

Cases: the half aneurysm (199,360 sites, 3,115 tiles, so the last workgroup is
ragged for every W; pulsatile Ladd inlet, pressure outlet) and a small tree, 30
steps from a seeded random state, FP32 in D3Q15 and D3Q19 and FP16 (whose staging
copies through registers).  One staged form is also held to the FP64 oracle element
by element after one step, at the bound of the one-step parity tests.
"""

import hashlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as wl  # noqa: E402
from oracle.lbgk import LBGK  # noqa: E402
from paper_1906_11925_amd import LB  # noqa: E402
from paper_1906_11925_amd import lib as L  # noqa: E402

from lbtest import quantize  # noqa: E402

pytestmark = pytest.mark.gpu

GEOMS = {
    "aneurysm_half": lambda: wl.aneurysm(half=True),
    "tree_small": lambda: wl.tree(box=96, r0=6.0, root=(48.0, 48.0, 4.0), generations=3, seed=1),
}
# (HEMELB_STAGE_TILES, HEMELB_LDS_DMA); the first is the unstaged reference
FP32_FORMS = [(0, 1), (4, 1), (8, 1), (16, 1), (4, 0), (8, 0), (16, 0)]
F16_FORMS = [(0, 1), (4, 1), (8, 1)]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _digest(monkeypatch, g, q, storage, form, d, steps):
    monkeypatch.setenv("HEMELB_STAGE_TILES", str(form[0]))
    monkeypatch.setenv("HEMELB_LDS_DMA", str(form[1]))
    lb = LB.from_geometry(g, lattice=q, storage=storage)
    assert lb.info()["addressing"] == L.ADDR_BLOCKS
    lb.set_deviations(torch.from_numpy(d), t=0)
    lb.step(steps)
    raw = lb.get_state()[0].cpu().numpy()
    lb.close()
    return hashlib.sha256(raw.tobytes()).hexdigest()


@pytest.mark.parametrize("name", sorted(GEOMS))
@pytest.mark.parametrize("q,storage,forms", [(15, "f32", FP32_FORMS), (19, "f32", FP32_FORMS[:4]),
                                             (15, "f16", F16_FORMS)])
def test_staged_forms_give_the_same_bits(monkeypatch, name, q, storage, forms):
    _gpu()
    g = GEOMS[name]()
    d = quantize(wl.random_deviations(q, g.n_sites, 23, 1e-3), q, storage)
    ref = _digest(monkeypatch, g, q, storage, forms[0], d, 30)
    for form in forms[1:]:
        assert _digest(monkeypatch, g, q, storage, form, d, 30) == ref, form


def test_widest_staged_form_against_the_oracle(monkeypatch):
    """One step of the 16-tile form with the direct copy, element by element
    against the oracle: deviations within 2 q^2 a 2^-24 (a = 1e-3)."""
    _gpu()
    monkeypatch.setenv("HEMELB_STAGE_TILES", "16")
    monkeypatch.setenv("HEMELB_LDS_DMA", "1")
    g = GEOMS["aneurysm_half"]()
    q = 15
    o = LBGK(g, q)
    d = quantize(wl.random_deviations(q, o.n, 5, 1e-3), q, "f32")
    lb = LB.from_geometry(g, lattice=q, storage="f32")
    lb.set_deviations(torch.from_numpy(d), t=37)
    lb.step(1)
    gpu = lb.get_deviations().cpu().numpy().astype(np.float64)
    lb.close()
    A, _ = o.step(o.lat.w[:, None] + d, 37)
    ref = A - o.lat.w[:, None]
    assert np.abs(gpu - ref).max() < 2.0 * q * q * 1e-3 * 2.0 ** -24
