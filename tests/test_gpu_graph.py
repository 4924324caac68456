"""hipGraph capture of a batch launch: every replay (with eager work and
synchronisation between replays) must give the bits of the eager launch."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_02119_amd import gen, kn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def test_graph_replay_matches_eager():
    knots = gen.config_knots("batched", 2, count=96)
    plans = [kn.Plan(kn.Tait(d.pd), q) for d, q in knots]
    b = kn.Batch(plans)
    b.upload()
    z_eager = b.contract()
    torch.cuda.synchronize()
    ref = z_eager.cpu().numpy().copy()
    z = kn.alloc_scalars(len(plans))
    g = b.graph(z)
    for rep in range(4):
        z.fill_(0.0)                        # eager work between replays
        _ = torch.ones(1 << 16, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy().view(np.int64), ref.view(np.int64)), rep


def test_graph_replay_gradients():
    rng = np.random.default_rng(21)
    knots = [gen.lattice_knot((79, k), 20, 70) for k in range(6)]
    plans = [kn.Plan(kn.Tait(d.pd), 3, jones_only=False, gradient=True) for d in knots]
    b = kn.Batch(plans)
    J = torch.tensor(rng.normal(scale=0.3, size=2 * b.stats["total_edges"]), device="cuda")
    b.upload()
    z0, g0 = b.contract_backward(J)
    torch.cuda.synchronize()
    zr, gr = z0.cpu().numpy().copy(), g0.cpu().numpy().copy()
    z = kn.alloc_scalars(len(plans))
    grad = torch.empty_like(g0)
    graph = b.graph(z, J=J, grad=grad)
    for rep in range(3):
        grad.fill_(0.0)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy().view(np.int64), zr.view(np.int64)), rep
        assert np.array_equal(grad.cpu().numpy(), gr), rep
