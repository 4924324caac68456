"""GPU parity of sliced plans: spins fixed, q^k slices run as chains sharing an
arena, slice values summed on the device.  Against the oracle on mid-size
knots, against the unsliced GPU result and the knot invariants on a
paper-model grid-walk knot of 351 crossings (largest tensor 2^25.4 entries
unsliced), and the Arf invariant at q = 2 on one of 574 crossings that does not
plan unsliced at q = 3.  Tolerance 1e-10 relative (complex128)."""

from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import invariants
from paper_1807_02119_amd import gen, kn
from tests.oracle_helpers import oracle_tait, oracle_z, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def _log(msg):
    print(msg, flush=True)


def _z(plan):
    z = kn.contract(plan)
    torch.cuda.synchronize()
    (m, e), = kn.scalars_from_device(z)
    return m, e


@pytest.mark.parametrize("q", [3, 5])
def test_sliced_parity(q):
    chained = False
    for k in range(5):
        d = gen.lattice_knot((82, k), 40, 120)
        t = kn.Tait(d.pd)
        tg, mo, eo = oracle_z(d, q)
        for rank in (1, 2, 3):
            budget = math.ceil(rank * math.log2(q))
            p = kn.Plan(t, q, slice_log2_budget=budget)
            chained |= p.stats["n_slices"] > p.stats["slice_chains"]
            _log(f"sliced q={q} {d.label} budget {budget}: {p.stats['n_slices']} slices, "
                 f"{p.stats['slice_chains']} chains")
            m, e = _z(p)
            assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10, (d.label, budget)
    assert chained


def test_sliced_batch_mixed():
    knots = [gen.lattice_knot((83, k), 30, 90) for k in range(8)]
    taits = [kn.Tait(d.pd) for d in knots]
    plans = [kn.Plan(t, 3, slice_log2_budget=(0 if i % 3 == 0 else 2 + i))
             for i, t in enumerate(taits)]
    b = kn.Batch(plans)
    z = b.contract()
    torch.cuda.synchronize()
    for (m, e), d in zip(kn.scalars_from_device(z), knots):
        tg, mo, eo = oracle_z(d, 3)
        assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10


def test_sliced_wide_grid_knot():
    """351-crossing paper-model knot: sliced (243 slices over 64 chains, every
    tensor <= 2^18 entries) equals the unsliced contraction, and |V| and the
    phase class match the Lickorish-Millett value at q = 3."""
    rng = np.random.default_rng(60)
    d = gen.random_grid_diagram(rng, 60)
    t = kn.Tait(d.pd)
    ps = kn.Plan(t, 3, slice_log2_budget=18)
    assert ps.stats["n_slices"] > ps.stats["slice_chains"] > 1
    _log(f"wide knot n={d.n}: {ps.stats['n_slices']} slices, max 2^{ps.stats['log2_max_entries']:.1f}")
    m, e = _z(ps)
    pu = kn.Plan(t, 3)
    mu, eu = _z(pu)
    assert rel_err(m * 2.0 ** (e - eu), mu) <= 1e-10
    tg = oracle_tait(d)
    v, l2, ar = kn.jones(3, t, m, e)
    dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
    assert abs(l2 - dd * math.log2(3) / 2) < 1e-9
    ratio = complex(math.cos(ar), math.sin(ar)) / unit
    assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9


def test_sliced_q2_arf_574_crossings():
    rng = np.random.default_rng(70)
    d = gen.random_grid_diagram(rng, 70)
    t = kn.Tait(d.pd)
    p = kn.Plan(t, 2, slice_log2_budget=18)
    assert p.stats["n_slices"] > 1
    m, e = _z(p)
    v, _, _ = kn.jones(2, t, m, e)
    tg = oracle_tait(d)
    assert abs(v - invariants.v_at_q2(tg.n_vertices, tg.edges, tg.eps)) < 1e-9


@pytest.mark.parametrize("k,q,budget", [(0, 2, 1), (2, 3, 4)])
def test_long_slice_loops(k, q, budget):
    """Slice counts far beyond the chain count: 16384 slices at q = 2 and
    19683 at q = 3, run as 64 device-side loops and as a single loop (one
    chain, every slice on the same descriptors), against the oracle."""
    d = gen.lattice_knot((84, k), 40, 70)
    t = kn.Tait(d.pd)
    tg, mo, eo = oracle_z(d, q)
    for mem in (None, 1):
        extra = {} if mem is None else {"mem_budget_bytes": mem, "allow_budget": True}
        p = kn.Plan(t, q, slice_log2_budget=budget, **extra)
        assert p.stats["n_slices"] >= 4096
        _log(f"long loop q={q} n={d.n}: {p.stats['n_slices']} slices, "
             f"{p.stats['slice_chains']} chains")
        m, e = _z(p)
        assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10, (d.n, q, mem)


# Paper-model grid-walk knots (Sec. III.A) of 521-574 crossings, too wide for
# one tensor of at most 2^31 entries at q = 3 under the min-fill order: the
# seed and walk size of each, and two plans with different orders and
# slicings (strategy, log2 budget of the largest tensor).
WIDE_Q3 = [(74, 80, (3, 26), (2, 26)), (72, 75, (3, 26), (2, 24)),
           (71, 72, (3, 26), (2, 24)), (70, 70, (3, 26), (3, 24))]


@pytest.mark.parametrize("seed,size,pa,pb", WIDE_Q3)
def test_sliced_q3_paper_model_500_600(seed, size, pa, pb):
    """Two sliced plans of one knot (different orders, spins fixed and slice
    counts) agree to 1e-10, and |V| and the phase class of V(e^{i pi/3}) equal
    the Lickorish-Millett value."""
    import time
    d = gen.random_grid_diagram(np.random.default_rng(seed), size)
    assert 500 <= d.n <= 600
    t = kn.Tait(d.pd)
    vals = []
    for strategy, budget in (pa, pb):
        t0 = time.perf_counter()
        p = kn.Plan(t, 3, strategy=strategy, slice_log2_budget=budget)
        t1 = time.perf_counter()
        assert p.stats["log2_max_entries"] <= budget + 1e-9
        m, e = _z(p)
        t2 = time.perf_counter()
        _log(f"q=3 n={d.n} strategy {strategy} budget {budget}: {p.stats['n_slices']} slices, "
             f"{p.stats['slice_chains']} chains, {p.stats['flops']:.3g} flop, "
             f"plan {t1 - t0:.2f} s, contract {t2 - t1:.2f} s "
             f"({p.stats['flops'] / (t2 - t1) / 1e12:.1f} TFLOP/s)")
        vals.append((m, e))
    (ma, ea), (mb, eb) = vals
    assert rel_err(ma * 2.0 ** (ea - eb), mb) <= 1e-10
    tg = oracle_tait(d)
    v, l2, ar = kn.jones(3, t, ma, ea)
    dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
    assert abs(l2 - dd * math.log2(3) / 2) < 1e-9
    ratio = complex(math.cos(ar), math.sin(ar)) / unit
    assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9
