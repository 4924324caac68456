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


def test_graph_replay_negative_exponent():
    """Result records compare by bit pattern: knot 373 of the mixed batch (q=6,
    21 crossings) has Z = -0.551 * 2^-4, whose int64 exponent read as a double
    is a NaN.  Its value matches the oracle, and graph replays reproduce the
    eager launch bit for bit."""
    from tests.oracle_helpers import oracle_z
    knots = gen.config_knots("batched", 0, count=512)[368:380]
    plans = [kn.Plan(kn.Tait(d.pd), q) for d, q in knots]
    b = kn.Batch(plans)
    b.upload()
    z_eager = b.contract()
    torch.cuda.synchronize()
    ref = z_eager.cpu().numpy().copy()
    exps = ref.view(np.int64)[:, 2]
    assert (exps < 0).any()
    for (d, q), (m, e) in zip(knots, kn.scalars_from_device(z_eager)):
        tg, mo, eo = oracle_z(d, q)
        assert abs(m * 2.0 ** (e - eo) - mo) <= 1e-10 * abs(mo), d.label
    z = kn.alloc_scalars(len(plans))
    g = b.graph(z)
    for rep in range(3):
        z.fill_(0.0)
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
