"""Host-side checks of libkn (no GPU): the C ABI loads and exports every
declared symbol, the C++ Tait builder agrees with the oracle's, the planner's
device program evaluates to the oracle's Z when executed by the CPU model of
the engine, Eq. 4 normalisation, and error handling."""

from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import jones as ojones
from oracle import potts
from paper_1807_02119_amd import gen, kn
from tests import image_model
from tests.oracle_helpers import oracle_tait, oracle_z, rel_err

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kn_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = kn.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(kn.EXPORTED)
    assert "gfx950" in kn.version()


def _same_graph_up_to_relabelling(t, o):
    """C++ and oracle Tait graphs are equal up to a renaming of the vertices.

    Edges are labelled (edge k is crossing k) in both, so a vertex is named by
    the set of edges incident to it; the two graphs agree iff these sets do."""
    uv, eps = t.edges()
    assert t.n_vertices == o.n_vertices
    assert list(eps) == list(o.eps)

    def signature(nv, edges):
        inc = [set() for _ in range(nv)]
        for k, (a, b) in enumerate(edges):
            inc[a].add(k)
            inc[b].add(k)
        return sorted(tuple(sorted(x)) for x in inc)

    return signature(t.n_vertices, [tuple(e) for e in uv]) == signature(o.n_vertices, o.edges)


@pytest.mark.parametrize("outer_side", [0, 1])
def test_tait_graph_matches_oracle(outer_side):
    ds = [gen.trefoil(), gen.figure_eight()] + [gen.lattice_knot((41, k), 3, 150) for k in range(25)]
    rng = np.random.default_rng(2)
    ds += [gen.random_grid_diagram(rng, 9) for _ in range(5)]
    for d in ds:
        if d.n < 2:
            continue
        t = kn.Tait(d.pd, outer_side=outer_side)
        o = oracle_tait(d, outer_left=(outer_side == 0))
        assert (t.writhe, t.tait_number) == (o.writhe, o.tait_number)
        assert _same_graph_up_to_relabelling(t, o)
        # same partition function on the two edge lists (q = 3)
        uv, eps = t.edges()
        x = potts.jones_weights(eps, ojones.t_of_q(3))
        z1 = potts.partition_function(t.n_vertices, [tuple(e) for e in uv], x, 3)
        z2 = potts.partition_function(o.n_vertices, o.edges, x, 3)
        assert rel_err(z1[0] * 2.0 ** (z1[1] - z2[1]), z2[0]) < 1e-12


def test_tait_single_crossing_and_unknot():
    for over_first in (False, True):
        for s in (1, -1):
            d = gen.add_kink(gen.UNKNOT, 0, over_first, s)
            t = kn.Tait(d.pd, d.signs)
            o = oracle_tait(d)
            assert (t.n_vertices, t.writhe, t.tait_number) == (o.n_vertices, o.writhe, o.tait_number)
    t = kn.Tait(np.zeros((0, 4), np.int32))
    assert (t.n_vertices, t.n_edges, t.writhe, t.tait_number) == (1, 0, 0, 0)


def test_tait_rejects_malformed_codes():
    good = gen.trefoil().pd
    with pytest.raises(kn.KnError) as e:
        kn.Tait(np.array([[0, 1, 2, 3]]))  # one crossing without signs
    assert e.value.code == -1
    bad = good.copy()
    bad[0, 0] = 99  # label out of range
    with pytest.raises(kn.KnError):
        kn.Tait(bad)
    bad = good.copy()
    bad[0, 1], bad[0, 3] = bad[0, 3], bad[0, 1]  # label used twice on one side
    bad[1, 1] = bad[0, 1]
    with pytest.raises(kn.KnError):
        kn.Tait(bad)
    # a non-planar code: swap two arcs between crossings
    bad = good.copy()
    bad[0, 1], bad[1, 1] = bad[1, 1], bad[0, 1]
    with pytest.raises(kn.KnError):
        kn.Tait(bad)


def _model_z(plan, J=None):
    (zm, ze), = image_model.run(plan.image(), J)
    return zm, ze


def _check_model(d, q, **kw):
    t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
    p = kn.Plan(t, q, **kw)
    zm, ze = _model_z(p)
    tg, m, e = oracle_z(d, q)
    assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12, (d.label, q, kw)


def test_plan_model_tiny_config():
    for d, q in gen.config_knots("tiny", 0):
        _check_model(d, q)


@pytest.mark.parametrize("q", [2, 3, 5, 6, 8])
def test_plan_model_many_q(q):
    for k in range(6):
        _check_model(gen.lattice_knot((43, k), 30, 120), q)


def test_plan_model_tiled_and_options():
    for k in range(4):
        d = gen.lattice_knot((44, k), 60, 160)
        for kw in (dict(big_step_macs_log2=4, tile_outputs=8),
                   dict(big_step_macs_log2=6, tile_outputs=100),
                   dict(simplify=0, jones_only=True),
                   dict(simplify=1, jones_only=True),
                   dict(simplify=1, jones_only=False),
                   dict(strategy=0), dict(strategy=1), dict(strategy=2),
                   dict(strategy=4, order_trials=3),
                   dict(lds_bytes=512), dict(lds_bytes=98304), dict(precision=1),
                   dict(split_serial_log2=3), dict(split_serial_log2=40),
                   dict(big_step_macs_log2=4, gemm_tasks_log2=1),
                   dict(big_step_macs_log2=4, gemm64_pct=100000),
                   dict(big_step_macs_log2=4, gemm64_pct=1),
                   dict(simplify=7), dict(simplify=5)):
            _check_model(d, 3, **kw)


def _split_gemm_cases():
    """Knots whose plans hold every kind of large step: 32 x 32 GEMM tiles,
    GEMM tiles over a split contracted range, and split output tiles."""
    work = gen.config_knots("q3_200_600", 0, count=72)
    # without the series-parallel reduction (simplify 3) these plans keep the
    # step shapes that split the contracted index of a GEMM step
    cases = [(work[71][0], dict(strategy=0, simplify=3)), (work[11][0], dict(simplify=3)),
             (work[11][0], {})]
    for k in range(2):
        cases.append((gen.lattice_knot((63, k), 100, 400), dict(big_step_macs_log2=4)))
    # segments of 128 contracted entries, so that GEMM steps split too
    return [(d, dict(kw, split_min_log2=7)) for d, kw in cases]


def test_default_split_segments():
    """By default a contracted index of nk entries is split into at most
    nk / 2^12 segments, rounded up (split_min_log2), and the workload's plans
    end with scalar
    products split that way: one output summed over segments of thousands of
    entries, which the engine shares out to the four wavefronts of a task.
    The parity tests of the workload on the GPU run such steps.  The model
    evaluates the default plans of a few of them to the oracle's Z."""
    work = gen.config_knots("q3_200_600", 0, count=24)
    one_output = []
    for i, (d, q) in enumerate(work):
        p = kn.Plan(kn.Tait(d.pd), q)
        for s in image_model.Image(p.image()).steps:
            if int(s["mode"]) == image_model.STEP_SERIAL or int(s["n_ks"]) < 2:
                continue
            nk = int(s["nk"])
            assert int(s["n_ks"]) <= -(-nk // 4096), (i, nk, int(s["n_ks"]))
            if int(s["nb"]) * int(s["nm"]) * int(s["nn"]) == 1:
                one_output.append(i)
    assert len(set(one_output)) >= 2
    for i in sorted(set(one_output))[:2]:
        _check_model(work[i][0], 3)
    # split_min_log2 = 7: segments of 128 entries again, more of them
    d = work[one_output[0]][0]
    fine = kn.Plan(kn.Tait(d.pd), 3, split_min_log2=7)
    assert fine.stats["n_tasks"] > kn.Plan(kn.Tait(d.pd), 3).stats["n_tasks"]
    with pytest.raises(kn.KnError):
        kn.Plan(kn.Tait(d.pd), 3, split_min_log2=31)


def gemm64_cases():
    """(label, knot, q, plan options) whose plans hold 64 x 64 GEMM steps:
    ragged sides, several blocks per task, and a split contracted range."""
    work = gen.config_knots("q3_200_600", 0, count=103)
    # segments of 128 contracted entries, so that GEMM steps split too
    wide = dict(gemm64_pct=100000, split_min_log2=7)
    return [("work71", work[71][0], 3, dict(strategy=0, simplify=3, **wide)),
            ("work94", work[94][0], 3, dict(gemm_tasks_log2=1, **wide)),
            ("work102", work[102][0], 3, dict(strategy=0, simplify=3, **wide)),
            ("lattice61_2", gen.lattice_knot((61, 2), 60, 250), 4,
             dict(big_step_macs_log2=4, **wide)),
            ("lattice61_2", gen.lattice_knot((61, 2), 60, 250), 4,
             dict(big_step_macs_log2=4, gemm_tasks_log2=1, **wide)),
            ("lattice61_5", gen.lattice_knot((61, 5), 150, 400), 3,
             dict(big_step_macs_log2=4, gemm_tasks_log2=1, **wide))]


def test_plan_model_gemm64_steps():
    seen = set()
    for label, d, q, kw in gemm64_cases():
        p = kn.Plan(kn.Tait(d.pd), q, **kw)
        for s in image_model.Image(p.image()).steps:
            if int(s["mode"]) == image_model.STEP_GEMM64:
                seen.add(("split", int(s["n_ks"]) > 1))
                seen.add(("grouped", int(s["tile"]) > 1))
                seen.add(("ragged", int(s["nm"]) % 64 != 0 or int(s["nn"]) % 64 != 0))
        _check_model(d, q, **kw)
    assert {("split", True), ("grouped", True), ("ragged", True)} <= seen
    # gemm64_pct=1 keeps every GEMM step in 32 x 32 blocks
    d = gemm64_cases()[0][1]
    p = kn.Plan(kn.Tait(d.pd), 3, strategy=0, simplify=3, gemm64_pct=1)
    modes = {int(s["mode"]) for s in image_model.Image(p.image()).steps}
    assert image_model.STEP_GEMM in modes and image_model.STEP_GEMM64 not in modes


def test_plan_model_gemm64_split_ragged_full_size():
    """The workload's largest knot (571 crossings) in 64 x 64 blocks, with a
    ragged split GEMM step: too slow for the oracle, so the model's Z is
    checked against the q=3 Lickorish-Millett class of V(e^{i pi/3})."""
    from oracle import invariants
    d = gen.config_knots("q3_200_600", 0, count=79)[78][0]
    t = kn.Tait(d.pd)
    p = kn.Plan(t, 3, gemm64_pct=100000, gemm_tasks_log2=1, split_min_log2=7)
    steps = image_model.Image(p.image()).steps
    assert any(int(s["mode"]) == image_model.STEP_GEMM64 and int(s["n_ks"]) > 1
               and int(s["nm"]) % 64 != 0 for s in steps)
    zm, ze = _model_z(p)
    v, l2, ar = kn.jones(3, t, zm, ze)
    tg = oracle_tait(d)
    dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
    assert abs(l2 - dd * math.log2(3) / 2) < 1e-9
    ratio = complex(math.cos(ar), math.sin(ar)) / unit
    assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9


def test_plan_model_gemm_and_split_steps():
    seen = set()
    for d, kw in _split_gemm_cases():
        p = kn.Plan(kn.Tait(d.pd), 3, **kw)
        for s in image_model.Image(p.image()).steps:
            seen.add((int(s["mode"]), int(s["n_ks"]) > 1))
        _check_model(d, 3, **kw)
    assert {(image_model.STEP_GEMM, False), (image_model.STEP_GEMM, True),
            (image_model.STEP_TILES, True), (image_model.STEP_TILES, False)} <= seen


def test_plan_model_general_couplings():
    rng = np.random.default_rng(7)
    for k in range(5):
        d = gen.lattice_knot((45, k), 20, 90)
        t = kn.Tait(d.pd)
        p = kn.Plan(t, 3, jones_only=False)
        J = rng.normal(scale=0.5, size=2 * t.n_edges)
        zm, ze = _model_z(p, J)
        uv, eps = t.edges()
        x = np.exp(J[0::2] + 1j * J[1::2])
        m, e = potts.partition_function(t.n_vertices, [tuple(a) for a in uv], x, 3)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12


def test_batch_image_model():
    knots = gen.config_knots("batched", 0, count=24)
    plans = [kn.Plan(kn.Tait(d.pd), q, big_step_macs_log2=(8 if i % 3 == 0 else 0))
             for i, (d, q) in enumerate(knots)]
    b = kn.Batch(plans)
    out = image_model.run(b.image())
    for (d, q), (zm, ze) in zip(knots, out):
        tg, m, e = oracle_z(d, q)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12
    assert b.edge_offset(0) == 0
    assert b.edge_offset(1) == plans[0].tait.n_edges


def test_plan_statistics_and_invariants():
    for k in range(8):
        d = gen.lattice_knot((46, k), 100, 300)
        t = kn.Tait(d.pd)
        p = kn.Plan(t, 3)
        s = p.stats
        im = image_model.Image(p.image())
        # every step is a pairwise contraction of live tensors; each consumed once
        steps = p.steps()
        assert len(steps) == s["n_steps"]
        consumed = set()
        n_vt = s["n_vertex_tensors"]
        for i, (a, b) in enumerate(steps):
            assert a != b and a < n_vt + i and b < n_vt + i
            assert a not in consumed and b not in consumed
            consumed |= {a, b}
        # flops and bytes add up over the steps
        fl = sum(8.0 * int(x["nb"]) * int(x["nm"]) * int(x["nn"]) * int(x["nk"]) for x in im.steps)
        assert fl == pytest.approx(s["flops"])
        by = sum(16.0 * (int(im.tensors[x["a"]]["size"]) + int(im.tensors[x["b"]]["size"]) +
                         int(im.tensors[x["c"]]["size"])) for x in im.steps)
        assert by == pytest.approx(s["bytes"])
        assert s["n_components"] >= 1
        assert s["max_rank"] <= 30
        assert s["log2_max_entries"] == pytest.approx(
            max(math.log2(int(x["size"])) for x in im.tensors))


def test_plan_errors():
    t = kn.Tait(gen.trefoil().pd)
    for q in (0, 1, 9, 100):
        with pytest.raises(kn.KnError) as e:
            kn.Plan(t, q)
        assert e.value.code == -6
    with pytest.raises(kn.KnError) as e:
        kn.Plan(t, 3, simplify=3, jones_only=False)  # R-II needs Jones couplings
    assert e.value.code == -1
    d = gen.lattice_knot((47, 0), 150, 250)
    big = kn.Tait(d.pd)
    with pytest.raises(kn.KnError) as e:
        kn.Plan(big, 3, mem_budget_bytes=1024)
    assert e.value.code == -3
    p = kn.Plan(big, 3, mem_budget_bytes=1024, allow_budget=True)
    assert p.stats["workspace_bytes"] > 1024


def test_jones_normalisation_matches_oracle():
    rng = np.random.default_rng(9)
    t = kn.Tait(gen.figure_eight().pd)
    for q in range(2, 9):
        for _ in range(5):
            zm = complex(rng.uniform(0.5, 1) * rng.choice([-1, 1]), rng.uniform(-1, 1))
            ze = int(rng.integers(-300, 300))
            v, l2, ar = kn.jones(q, t, zm, ze)
            vo, l2o = ojones.jones_value(q, t.n_vertices, t.writhe, t.tait_number, zm, ze)
            assert abs(l2 - l2o) < 1e-11
            ph = ar - math.atan2(vo.imag, vo.real) if vo != 0 else 0
            assert abs(math.remainder(ph, 2 * math.pi)) < 1e-11
    # t(q) of Eq. 1
    for q in range(2, 9):
        assert abs(kn.jones_variable(q) - ojones.t_of_q(q)) < 1e-14
    with pytest.raises(kn.KnError):
        kn.jones_variable(9)
    with pytest.raises(kn.KnError) as e:
        kn.jones(3, t, complex(math.nan, 0), 0)
    assert e.value.code == -5


def test_jones_large_knot_phase_exact():
    # phase reduction in integers: same V for huge (n_v, w, tau) offsets that
    # differ by a full period of the phase
    t = kn.Tait(gen.trefoil().pd)
    v, l2, ar = kn.jones(3, t, 0.5 + 0j, 0)
    vo, l2o = ojones.jones_value(3, t.n_vertices, t.writhe, t.tait_number, 0.5 + 0j, 0)
    assert abs(v - vo) < 1e-14 * abs(vo) + 1e-300


def test_status_strings():
    for c in range(-6, 1):
        assert kn.status_string(c)


def _gradient_cases():
    cases = [gen.trefoil(), gen.figure_eight(), gen.add_kink(gen.figure_eight(), 0, True, 1)]
    cases += [gen.lattice_knot((70, k), 8, 16) for k in range(6)]
    cases += [gen.lattice_knot((71, k), 20, 40) for k in range(3)]
    return cases


@pytest.mark.parametrize("q", [2, 3, 5])
def test_gradient_plan_model_matches_oracle(q):
    """Reverse pass of the device program (CPU model) against the oracle's
    d log Z / d J (one elimination per edge), random complex couplings."""
    rng = np.random.default_rng(100 + q)
    for d in _gradient_cases():
        t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
        p = kn.Plan(t, q, jones_only=False, gradient=True)
        J = rng.normal(scale=0.4, size=2 * t.n_edges)
        ((zm, ze),), g = image_model.run(p.image(), J, want_grad=True)
        uv, eps = t.edges()
        x = np.exp(J[0::2] + 1j * J[1::2])
        edges = [tuple(a) for a in uv]
        m, e = potts.partition_function(t.n_vertices, edges, x, q)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12
        go = potts.dlogz_dj(t.n_vertices, edges, x, q)
        assert np.max(np.abs(g - go) / np.abs(go)) < 1e-12, (d.label, q)


def test_gradient_plan_model_jones_point_and_batch():
    """J = NULL (the Jones couplings) on gradient plans, in one batch image."""
    knots = [gen.lattice_knot((72, k), 10, 30) for k in range(4)]
    taits = [kn.Tait(d.pd) for d in knots]
    plans = [kn.Plan(t, 3, gradient=True) for t in taits]
    b = kn.Batch(plans)
    out, g = image_model.run(b.image(), None, want_grad=True)
    tq = ojones.t_of_q(3)
    for i, (t, (zm, ze)) in enumerate(zip(taits, out)):
        uv, eps = t.edges()
        x = potts.jones_weights(eps, tq)
        edges = [tuple(a) for a in uv]
        m, e = potts.partition_function(t.n_vertices, edges, x, 3)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12
        off = b.edge_offset(i)
        go = potts.dlogz_dj(t.n_vertices, edges, x, 3)
        gi = g[off:off + t.n_edges]
        assert np.max(np.abs(gi - go) / np.abs(go)) < 1e-12


def test_gradient_plan_options():
    t = kn.Tait(gen.figure_eight().pd)
    with pytest.raises(kn.KnError):
        kn.Plan(t, 3, gradient=True, simplify=3)  # Reidemeister II drops edges
    p = kn.Plan(t, 3)
    with pytest.raises(kn.KnError) as ei:
        kn.backward_workspace_bytes(p)
    assert ei.value.code == -6
    pg = kn.Plan(t, 3, gradient=True, jones_only=False)
    assert kn.backward_workspace_bytes(pg) == pg.workspace_bytes
    # the reverse pass doubles the steps and adds one seed per component
    pf = kn.Plan(t, 3, jones_only=False, simplify=1)
    assert pg.stats["n_steps"] == 3 * pf.stats["n_steps"]
    assert pg.stats["n_vertex_tensors"] == pf.stats["n_vertex_tensors"] + pf.stats["n_components"]


def test_autotuner_coordinate_descent():
    """The tuner's search on a known cost surface: it reaches the minimum of
    a separable function and measures each setting once."""
    from paper_1807_02119_amd import tune

    calls = []

    def cost(s):
        calls.append(dict(s))
        return (s["a"] - 3) ** 2 + abs(s["b"] - 20) + 0.5 * (s["c"] != "y")

    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": ["x", "y"]}
    best, v, seen = tune.coordinate_descent(cost, space, {"a": 1, "b": 10, "c": "x"})
    assert best == {"a": 3, "b": 20, "c": "y"} and v == 0
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys)) == len(seen)


def test_tile_macs_option():
    d = gen.lattice_knot((44, 0), 60, 160)
    t = kn.Tait(d.pd)
    a = image_model.Image(kn.Plan(t, 3, big_step_macs_log2=4, tile_macs_log2=3).image())
    b = image_model.Image(kn.Plan(t, 3, big_step_macs_log2=4, tile_macs_log2=16).image())
    tiles = lambda im: sum(int(s["n_tiles"]) for s in im.steps if int(s["mode"]) == 1)
    assert tiles(a) > tiles(b) > 0
    with pytest.raises(kn.KnError):
        kn.Plan(t, 3, tile_macs_log2=31)
    _check_model(d, 3, big_step_macs_log2=4, tile_macs_log2=3)


@pytest.mark.parametrize("q", [2, 3, 5])
def test_sliced_plan_model_matches_oracle(q):
    """Slicing (spins fixed, q^k slices, chains of slices sharing an arena)
    through the CPU model of the device program, against the oracle."""
    rng = np.random.default_rng(300 + q)
    cases = [gen.trefoil(), gen.lattice_knot((80, 0), 20, 60), gen.lattice_knot((80, 1), 20, 60),
             gen.random_grid_diagram(rng, 14)]
    seen_chained = False
    for d in cases:
        t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
        tg, m, e = oracle_z(d, q)
        for rank in (1, 2):  # budgets of one and two spins
            budget = math.ceil(rank * math.log2(q))
            p = kn.Plan(t, q, slice_log2_budget=budget)
            assert p.stats["log2_max_entries"] <= budget + 1e-9
            seen_chained |= p.stats["n_slices"] > p.stats["slice_chains"]
            (zm, ze), = image_model.run(p.image())
            assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12, (d.label, budget)
    assert seen_chained or q < 3  # q = 2 slices fit one chain each


def test_sliced_batch_and_couplings():
    """Sliced and unsliced plans in one batch, general couplings."""
    rng = np.random.default_rng(17)
    knots = [gen.lattice_knot((81, k), 15, 50) for k in range(4)]
    taits = [kn.Tait(d.pd) for d in knots]
    plans = [kn.Plan(t, 3, jones_only=False, slice_log2_budget=(3 if i % 2 else 0))
             for i, t in enumerate(taits)]
    assert any(p.stats["n_slices"] > 1 for p in plans)
    b = kn.Batch(plans)
    J = rng.normal(scale=0.3, size=2 * b.stats["total_edges"])
    out = image_model.run(b.image(), J)
    for i, (t, (zm, ze)) in enumerate(zip(taits, out)):
        off = b.edge_offset(i)
        uv, _ = t.edges()
        x = np.exp(J[2 * off:2 * (off + t.n_edges):2] + 1j * J[2 * off + 1:2 * (off + t.n_edges):2])
        m, e = potts.partition_function(t.n_vertices, [tuple(a) for a in uv], x, 3)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12


def test_separator_order_matches_oracle():
    """Separator-hierarchy orders (strategy 4, several hierarchies), also
    sliced, through the CPU model of the device program against the oracle."""
    rng = np.random.default_rng(91)
    cases = [gen.lattice_knot((90, k), 40, 140) for k in range(4)]
    cases += [gen.random_grid_diagram(rng, 16), gen.trefoil()]
    sliced = 0
    for d in cases:
        t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
        for q in (2, 3):
            tg, m, e = oracle_z(d, q)
            # a slicing budget one spin below the width
            r = kn.Plan(t, q, strategy=4).stats["max_rank"]
            budget = max(1, math.floor((r - 1) * math.log2(q)))
            for kw in (dict(strategy=4), dict(strategy=4, order_trials=1),
                       dict(strategy=4, slice_log2_budget=budget)):
                p = kn.Plan(t, q, **kw)
                if p.stats["n_slices"] > 729:  # the CPU model runs slices one by one
                    continue
                sliced += p.stats["n_slices"] > 1
                (zm, ze), = image_model.run(p.image())
                assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12, (d.label, q, kw)
    assert sliced >= 4


def test_separator_order_wins_on_large_grid_knots():
    """On paper-model grid-walk knots of about 900 crossings the separator
    hierarchy needs far less work than the greedy and min-fill orders (the
    paper finds the METIS order ahead of greedy from about 900 crossings),
    and the auto strategy takes it."""
    for seed, size in ((77, 95), (76, 90)):
        d = gen.random_grid_diagram(np.random.default_rng(seed), size)
        assert d.n > 900
        t = kn.Tait(d.pd)
        f = {s: kn.Plan(t, 2, strategy=s, allow_budget=True).stats for s in (0, 2, 3, 4)}
        sep = f[4]["flops"]
        assert sep > 0
        for s in (0, 2):  # a failed plan (a tensor over 2^31 entries) reports 0 flops
            assert f[s]["flops"] == 0 or sep < 0.5 * f[s]["flops"], (seed, s, f[s]["flops"], sep)
        assert f[3]["max_rank"] <= f[4]["max_rank"] + 1


def test_slicing_makes_wide_knots_fit():
    """A paper-model grid-walk knot wider than the int32 tensor limit plans
    only when sliced; the sliced plan keeps every tensor within the budget."""
    rng = np.random.default_rng(70)
    d = gen.random_grid_diagram(rng, 70)
    t = kn.Tait(d.pd)
    with pytest.raises(kn.KnError) as ei:
        kn.Plan(t, 3)
    assert ei.value.code == -3
    p = kn.Plan(t, 3, slice_log2_budget=24)
    assert p.stats["log2_max_entries"] <= 24 + 1e-9
    assert p.stats["n_slices"] == 3 ** round(math.log(p.stats["n_slices"], 3))
    assert 1 <= p.stats["slice_chains"] <= min(64, p.stats["n_slices"])
    with pytest.raises(kn.KnError):
        kn.Plan(t, 3, slice_log2_budget=24, gradient=True)


def test_plan_set_handles():
    """PlanSet: the same plans as plan_many, views that do not free, one batch
    image, and Jones values from the set's Tait graphs."""
    knots = [gen.lattice_knot((85, k), 20, 80) for k in range(6)]
    ncr = np.array([d.n for d in knots], np.int32)
    flat = np.concatenate([np.asarray(d.pd, np.int32).reshape(-1) for d in knots])
    ps = kn.plan_set(ncr, flat, 3)
    _, plans = kn.plan_many([d.pd for d in knots], 3)
    assert len(ps) == len(plans)
    for i, p in enumerate(plans):
        v = ps.plan(i)
        assert v.stats == p.stats
        assert v.image() == p.image()
        del v  # a view: the set still owns the plan
    assert kn.Batch(ps).image() == kn.Batch(plans).image()
    z = np.tile([1.0, 0.0, 0.0], (len(knots), 1))
    a = kn.jones_many(3, ps, z)
    b = kn.jones_many(3, [p.tait for p in plans], z)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_plan_sets_freed_while_planning():
    """The bench's pattern: plan sets and batches released on one thread while
    another plans on the library's thread pool.  Every plan set made
    meanwhile still gives the same batch image."""
    import threading
    knots = [gen.lattice_knot((86, k), 40, 160) for k in range(24)]
    ncr = np.array([d.n for d in knots], np.int32)
    flat = np.concatenate([np.asarray(d.pd, np.int32).reshape(-1) for d in knots])
    ref = kn.Batch(kn.plan_set(ncr, flat, 3, strategy=2)).image()
    old = [kn.plan_set(ncr, flat, 3) for _ in range(6)]
    errors = []

    def release():
        try:
            while old:
                ps = old.pop()
                b = kn.Batch(ps)
                del b, ps
        except Exception as ex:  # pragma: no cover - reported below
            errors.append(ex)

    th = threading.Thread(target=release)
    th.start()
    images = [kn.Batch(kn.plan_set(ncr, flat, 3, strategy=2)).image() for _ in range(6)]
    th.join()
    assert not errors
    assert all(im == ref for im in images)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with a message."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_bench_traffic_record_matches_source(tmp_path, monkeypatch):
    """bench.py reports measured HBM traffic only from a record taken on the
    current kernel source: a record carrying the current source hash is used,
    one with another hash gives none."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_1807_02119_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (csrc / f).write_bytes(open(os.path.join(root, "paper_1807_02119_amd", "csrc", f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"fetch_bytes": 1.0e9, "write_bytes": 0.5e9, "source_hash": bench.source_hash()}
    path = tmp_path / "profiles" / "engine_traffic.json"
    path.write_text(json.dumps({"engine<double>": rec}))
    got = bench.measured_traffic("engine<double>")
    assert got is not None and got["fetch_bytes"] == 1.0e9
    assert bench.measured_traffic("engine<float>") is None
    rec["source_hash"] = "0" * 16
    path.write_text(json.dumps({"engine<double>": rec}))
    assert bench.measured_traffic("engine<double>") is None


def test_tuner_space_is_valid():
    """Every value the autotuner tries, plan-wide and per intermediate-size
    bucket, and its recorded settings, are plan options the planner accepts."""
    from paper_1807_02119_amd import tune
    d = gen.lattice_knot((88, 0), 40, 120)
    t = kn.Tait(d.pd)
    base = tune.plan_options(tune.DEFAULTS)
    for knob, values in tune.SPACE.items():
        for v in values:
            kn.Plan(t, 3, **dict(base, **{knob: v}))
    for coord, values in tune.bucket_space().items():
        for v in values:
            flat = dict(tune.DEFAULTS, **{coord: v})
            kn.Plan(t, 3, **tune.plan_options(tune.split_setting(flat)))
    for workload in ("q3_200_600", "batched"):
        for prec in (0, 1):
            rec = tune.load(workload, prec)
            if workload == "q3_200_600" or rec:
                assert rec, (workload, prec)
                kn.Plan(t, 3, precision=prec, **tune.plan_options(rec))
                # a recorded setting as a search start: every coordinate set,
                # and back to the same setting (defaults filled in)
                flat = tune.flat_setting(rec)
                assert set(flat) == set(tune.DEFAULTS) | set(tune.bucket_space())
                back = tune.split_setting(flat)
                assert back.get("buckets", {}) == rec.get("buckets", {})
                assert all(back[k] == rec.get(k, tune.DEFAULTS[k]) for k in tune.DEFAULTS)


def test_bucket_knobs_change_only_their_bucket():
    """A per-bucket override of the tile shape changes the tiling of the steps
    whose output falls in that bucket and of no other step."""
    from tests import image_model as im
    d = gen.lattice_knot((89, 4), 300, 420)
    t = kn.Tait(d.pd)

    def tiling(**kw):
        st = im.Image(kn.Plan(t, 3, strategy=2, **kw).image()).steps
        return [(int(s["mode"]), int(s["tile"]), int(s["n_tiles"])) for s in st], st

    ref, st = tiling()
    outs = [int(s["nb"]) * int(s["nm"]) * int(s["nn"]) for s in st]
    buckets = [0 if o <= 2**8 else 1 if o <= 2**12 else 2 if o <= 2**16 else 3 if o <= 2**20
               else 4 for o in outs]
    # buckets holding a tiled step whose tiles have more than 8 outputs
    wide = {b for b, r in zip(buckets, ref) if r[0] == 1 and r[1] > 8}
    assert wide
    for b in range(5):
        new, _ = tiling(buckets={b: {"tile_outs_log2": 3}})
        changed = {buckets[i] for i in range(len(ref)) if new[i] != ref[i]}
        assert changed == ({b} if b in wide else set()), (b, changed)


def test_output_heavy_steps_are_tiled():
    """A step with at least 2^big_step_outs_log2 outputs runs as tiles, and no
    tile of a tiled step has more than 2^tile_outs_log2 outputs."""
    from tests import image_model as im
    d = gen.lattice_knot((89, 4), 400, 520)
    t = kn.Tait(d.pd)
    for outs_log2, tile_log2 in ((10, 8), (12, 10), (31, 10)):
        img = im.Image(kn.Plan(t, 3, strategy=2, big_step_outs_log2=outs_log2,
                               tile_outs_log2=tile_log2).image())
        for s in img.steps:
            outs = int(s["nb"]) * int(s["nm"]) * int(s["nn"])
            if outs_log2 < 31 and outs >= 2**outs_log2:
                assert int(s["mode"]) != 0, (outs, int(s["mode"]))
            if int(s["mode"]) == 1 and int(s["tile"]) > 1:
                assert int(s["tile"]) <= 2**tile_log2


def test_series_parallel_reduction():
    """simplify bit 2: fewer spins, the same Z (CPU model against the oracle
    and against the unreduced plan), constants in the image, and only for
    plans bound to the Jones couplings."""
    for k in range(6):
        d = gen.lattice_knot((86, k), 40, 160)
        t = kn.Tait(d.pd)
        p3 = kn.Plan(t, 3, simplify=3)
        p7 = kn.Plan(t, 3, simplify=7)
        assert p7.stats["n_vertices_simplified"] < p3.stats["n_vertices_simplified"]
        im = image_model.Image(p7.image())
        assert int(im.h["n_consts"]) > 0 and (im.medges["y"] == -1).any()
        (m3, e3), = image_model.run(p3.image())
        (m7, e7), = image_model.run(p7.image())
        assert abs(m7 * 2.0 ** (e7 - e3) - m3) <= 1e-12 * abs(m3)
        _check_model(d, 3, simplify=7)
        _check_model(d, 5, simplify=7)
    t = kn.Tait(gen.lattice_knot((86, 0), 40, 160).pd)
    with pytest.raises(kn.KnError):
        kn.Plan(t, 3, jones_only=False, simplify=5)


def test_gradient_recompute_under_budget():
    """Gradient plans under mem_budget_bytes drop forward intermediates after
    their forward use and recompute them before their reverse use: the
    workspace shrinks, the recompute shows in the statistics, and the CPU model
    of the device program gives the unbudgeted Z and gradient (to rounding),
    with the arena reused without overwriting a live tensor."""
    rng = np.random.default_rng(1)
    d = gen.random_grid_diagram(rng, 36)
    t = kn.Tait(d.pd)
    p = kn.Plan(t, 3, jones_only=False, gradient=True)
    W = p.workspace_bytes
    pb = kn.Plan(t, 3, jones_only=False, gradient=True, mem_budget_bytes=int(0.75 * W))
    assert pb.status == 0 and pb.workspace_bytes <= 0.75 * W
    assert pb.stats["n_recompute_steps"] > 0 and pb.stats["flops"] > p.stats["flops"]
    J = rng.normal(scale=0.3, size=2 * t.n_edges)
    ((zm, ze),), g = image_model.run(pb.image(), J, want_grad=True)
    ((zm0, ze0),), g0 = image_model.run(p.image(), J, want_grad=True)
    assert rel_err(zm * 2.0 ** (ze - ze0), zm0) < 1e-12
    assert np.max(np.abs(g - g0) / np.abs(g0)) < 1e-12


def test_gradient_recompute_matches_oracle():
    """A budget below what the gradient plan can reach: the planner keeps the
    setting with the least memory (recompute chains included) and reports
    KN_E_BUDGET; that plan's reverse pass still gives the oracle's
    d log Z / d J_e (CPU model of the device program)."""
    rng = np.random.default_rng(5)
    # knots of 54-59 crossings at q = 5 and 8, whose intermediates (up to
    # 2^14-2^15 entries) are large next to the device program
    for k, q in ((0, 8), (3, 5)):
        d = gen.lattice_knot((75, k), 30, 60)
        t = kn.Tait(d.pd)
        full = kn.Plan(t, q, jones_only=False, gradient=True)
        p = kn.Plan(t, q, jones_only=False, gradient=True,
                    mem_budget_bytes=full.workspace_bytes // 2, allow_budget=True)
        assert p.status == -3 and p.stats["n_recompute_steps"] > 0, d.label
        assert p.workspace_bytes < full.workspace_bytes
        J = rng.normal(scale=0.4, size=2 * t.n_edges)
        ((zm, ze),), g = image_model.run(p.image(), J, want_grad=True)
        uv, eps = t.edges()
        x = np.exp(J[0::2] + 1j * J[1::2])
        edges = [tuple(a) for a in uv]
        m, e = potts.partition_function(t.n_vertices, edges, x, q)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12
        go = potts.dlogz_dj(t.n_vertices, edges, x, q)
        assert np.max(np.abs(g - go) / np.abs(go)) < 1e-12, d.label


def test_slice_loop_on_the_device_model():
    """Slices run as a loop on the device: each chain is one copy of the
    knot's device program whose final task starts the chain's next slice.
    With one chain, every slice runs on the same descriptors (the image does
    not grow with the slice count) and Z matches the oracle."""
    done = 0
    for k, q in ((0, 2), (1, 3), (2, 3), (3, 2), (4, 3)):
        d = gen.lattice_knot((86, k), 30, 70)
        t = kn.Tait(d.pd)
        plain = kn.Plan(t, q)
        # the largest budget that needs between 9 and 729 slices
        p = None
        for budget in range(int(plain.stats["max_rank"] * math.log2(q)), 0, -1):
            c = kn.Plan(t, q, slice_log2_budget=budget, mem_budget_bytes=1, allow_budget=True)
            if 9 <= c.stats["n_slices"] <= 729:
                p = c
                break
        if p is None:
            continue
        st = p.stats
        assert st["slice_chains"] == 1, st
        # one set of descriptors per chain, whatever the slice count
        assert st["image_bytes"] < 4 * plain.stats["image_bytes"] + 65536
        img = image_model.Image(p.image())
        assert int(img.h["n_knots"]) == 1
        assert int(img.h["n_queue"]) == int(img.h["n_tasks"]) * st["n_slices"]
        tg, m, e = oracle_z(d, q)
        (zm, ze), = image_model.run(p.image())
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12, (d.label, q)
        done += 1
    assert done >= 3


def test_forked_runs_on_the_device_model():
    """Long serial runs forked into concurrent subtree tasks: a task for the
    vertex tensors, a group of up to 8 subtree tasks, and the steps above
    them.  The CPU model runs each group's tasks as concurrent (their global
    ranges may not overlap, their outputs are visible only after the group)
    and matches the oracle, also sliced, in complex64 and in a batch."""
    knots = [gen.lattice_knot((44, k), 100, 200) for k in range(4)]
    forked = 0
    for d in knots:
        t = kn.Tait(d.pd)
        tg, m, e = oracle_z(d, 3)
        for kw in (dict(fork_serial_log2=4), dict(fork_serial_log2=6),
                   dict(fork_serial_log2=5, slice_log2_budget=5),
                   dict(fork_serial_log2=3, split_serial_log2=3)):
            p = kn.Plan(t, 3, **kw)
            img = image_model.Image(p.image())
            sizes = [int(g["n_tasks"]) for g in img.groups]
            if p.stats["n_slices"] == 1 and len(sizes) == 3:
                forked += 1
                assert sizes[0] == 1 and 2 <= sizes[1] <= 8 and sizes[2] == 1, sizes
            (zm, ze), = image_model.run(p.image())
            assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12, (d.label, kw)
        p32 = kn.Plan(t, 3, fork_serial_log2=4, precision=1)
        (zm, ze), = image_model.run(p32.image())
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-5
    assert forked >= 4
    b = kn.Batch([kn.Plan(kn.Tait(d.pd), 3, fork_serial_log2=5) for d in knots])
    for (zm, ze), d in zip(image_model.run(b.image()), knots):
        tg, m, e = oracle_z(d, 3)
        assert rel_err(zm * 2.0 ** (ze - e), m) < 1e-12
    # gradient plans are never forked (their tensors are read twice)
    g = kn.Plan(kn.Tait(knots[0].pd), 3, fork_serial_log2=2, gradient=True, jones_only=False)
    assert all(int(x["n_tasks"]) == 1 for x in image_model.Image(g.image()).groups
               if int(image_model.Image(g.image()).tasks[int(x["first_task"])]["kind"]) == 0)


def test_model_catches_overlapping_concurrent_tasks():
    """A planted fault in a copy of a forked image: the output of one subtree
    task moved onto a tensor that another subtree task of the same group
    writes.  The CPU model must reject it."""
    d = gen.lattice_knot((44, 0), 100, 200)
    raw = bytearray(kn.Plan(kn.Tait(d.pd), 3, fork_serial_log2=4).image())
    img = image_model.Image(bytes(raw))
    grp = img.groups[1]
    tasks = [img.tasks[i] for i in range(int(grp["first_task"]), int(grp["first_task"]) + int(grp["n_tasks"]))]
    assert len(tasks) >= 2
    last = lambda task: int(img.steps[int(task["first"]) + int(task["count"]) - 1]["c"])
    a, b = last(tasks[0]), last(tasks[1])
    assert int(img.tensors[a]["lds_off"]) < 0 and int(img.tensors[b]["lds_off"]) < 0
    h = img.h
    tens = np.frombuffer(raw, image_model.TENSOR, int(h["n_tensors"]), int(h["o_tensors"]))
    steps = np.frombuffer(raw, image_model.STEP, int(h["n_steps"]), int(h["o_steps"]))
    tens[b]["off"] = tens[a]["off"]
    for s in steps:  # keep the step homes consistent with the moved tensor
        for f, t in (("home_a", "a"), ("home_b", "b"), ("home_c", "c")):
            if int(s[t]) == b:
                s[f] = int(tens[a]["off"])
    with pytest.raises(AssertionError, match="overlap|overwrites"):
        image_model.run(bytes(raw))
