"""GPU parity of a plan whose spin groups need the full int32 index range of
the engine's decode (csrc/decode.h): a paper-model grid-walk knot (Sec. III.A)
of 770 crossings at q = 2, unsliced, whose min-fill plan holds a tensor of 2^28 entries
and a step contracting a group of 2^27 values (indices far past q * 2^24).
Checked against the sliced plan of the same knot (every tensor <= 2^20
entries, relative error <= 1e-10) and against the exact value V(i) = +-1 that
the Arf invariant fixes."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import invariants
from paper_1807_02119_amd import gen, kn
from tests import image_model as im
from tests.oracle_helpers import oracle_tait, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def test_group_of_2_27_values_q2():
    rng = np.random.default_rng(1000 * 86 + 1)
    d = gen.random_grid_diagram(rng, 86)
    t = kn.Tait(d.pd)
    # the min-fill order: its plan holds the wide group this test needs (the
    # auto order, which also tries separator hierarchies, stays below 2^25)
    p = kn.Plan(t, 2, strategy=2)
    steps = im.Image(p.image()).steps
    widest = max(int(max(s["nb"], s["nm"], s["nn"], s["nk"])) for s in steps)
    assert widest >= 2**27 and p.stats["log2_max_entries"] >= 27
    print(f"n={d.n} widest group {widest}, largest tensor 2^{p.stats['log2_max_entries']:.0f}, "
          f"workspace {p.workspace_bytes / 2**30:.2f} GiB", flush=True)
    z = kn.contract(p)
    torch.cuda.synchronize()
    (m, e), = kn.scalars_from_device(z)
    ps = kn.Plan(t, 2, slice_log2_budget=20)
    assert ps.stats["log2_max_entries"] <= 20 and ps.stats["n_slices"] > 1
    zs = kn.contract(ps)
    torch.cuda.synchronize()
    (ms, es), = kn.scalars_from_device(zs)
    assert rel_err(m * 2.0 ** (e - es), ms) <= 1e-10
    v, _, _ = kn.jones(2, t, m, e)
    tg = oracle_tait(d)
    assert abs(v - invariants.v_at_q2(tg.n_vertices, tg.edges, tg.eps)) < 1e-9
