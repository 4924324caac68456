"""kn_contract_noalloc -- kn_contract with the library's own fixed device
array as its workspace, so that the call allocates no device memory -- checked
through the C ABI against kn_contract on the same plans: two calls in a row,
the second on a smaller knot than the first (the array keeps the first call's
contents), each equal to kn_contract's Z to 1e-10 relative (the kernels are
the same, so the bits agree too); explicit couplings; and a plan whose
workspace exceeds the array rejected with KN_E_BUDGET before any launch."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_02119_amd import gen, kn
from tests.oracle_helpers import rel_err

pytestmark = pytest.mark.gpu

NOALLOC_MAX_BYTES = 64 << 20  # KN_NOALLOC_MAX_BYTES in include/kn.h


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def _host(z):
    torch.cuda.synchronize()
    (m, e), = kn.scalars_from_device(z)
    return m, e, z.cpu().numpy().view(np.int64).copy()


def _same(a, b):
    (ma, ea, ba), (mb, eb, bb) = a, b
    assert np.isfinite(ma.real) and np.isfinite(mb.real)
    assert rel_err(ma * 2.0 ** (ea - eb), mb) <= 1e-10
    assert np.array_equal(ba, bb)


def test_noalloc_two_calls_second_smaller():
    big = kn.Plan(kn.Tait(gen.lattice_knot((950, 0), 300, 420).pd), 3)
    small = kn.Plan(kn.Tait(gen.lattice_knot((950, 1), 30, 60).pd), 3)
    assert small.workspace_bytes < big.workspace_bytes <= NOALLOC_MAX_BYTES
    print(f"workspaces {big.workspace_bytes} then {small.workspace_bytes} bytes", flush=True)
    ref_big = _host(kn.contract(big))
    ref_small = _host(kn.contract(small))
    z_big = _host(kn.contract_noalloc(big))
    z_small = _host(kn.contract_noalloc(small))
    _same(z_big, ref_big)
    _same(z_small, ref_small)
    # and once more in the other order, on the same array
    _same(_host(kn.contract_noalloc(big)), ref_big)


def test_noalloc_couplings_q5():
    rng = np.random.default_rng(951)
    for k, lo, hi in ((0, 120, 200), (1, 20, 40)):
        t = kn.Tait(gen.lattice_knot((951, k), lo, hi).pd)
        p = kn.Plan(t, 5, jones_only=False)
        J = torch.tensor(rng.normal(0.0, 0.3, 2 * t.n_edges), dtype=torch.float64, device="cuda")
        _same(_host(kn.contract_noalloc(p, J)), _host(kn.contract(p, J)))


def test_noalloc_rejects_oversized_plan():
    rng = np.random.default_rng(1000 * 86 + 1)
    t = kn.Tait(gen.random_grid_diagram(rng, 86).pd)
    p = kn.Plan(t, 2)
    assert p.workspace_bytes > NOALLOC_MAX_BYTES
    z = kn.alloc_scalars(1)
    with pytest.raises(kn.KnError) as e:
        kn.contract_noalloc(p, z=z)
    assert e.value.code == -3
