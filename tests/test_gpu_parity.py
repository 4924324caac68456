"""GPU parity: the HIP engine (through the C ABI) against the CPU oracle.

Tolerance: relative error <= 1e-10 on Z and V for complex128 (the bound the
method's exactness allows: the oracle's own rounding is ~1e-15, see
test_oracle_pins); complex64 results are checked against an error bound
derived in the test.
"""

from __future__ import annotations

import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import exact, invariants, kauffman
from oracle import jones as ojones
from oracle import potts
from paper_1807_02119_amd import gen, kn, tune
from tests.oracle_helpers import TOL32, oracle_tait, oracle_v, oracle_z, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def _log(msg):
    print(msg, flush=True)


def gpu_z(d, q, **kw):
    t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
    p = kn.Plan(t, q, **kw)
    z = kn.contract(p)
    torch.cuda.synchronize()
    (m, e), = kn.scalars_from_device(z)
    return t, p, m, e


def z_close(m, e, mo, eo, tol=TOL):
    if mo == 0:
        return m == 0
    return rel_err(m * 2.0 ** (e - eo), mo) <= tol


def test_tiny_config_parity():
    _log("tiny config, q=3")
    for d, q in gen.config_knots("tiny", 0):
        t, p, m, e = gpu_z(d, q)
        tg, mo, eo = oracle_z(d, q)
        assert z_close(m, e, mo, eo), (d.label, m, e, mo, eo)
        v, l2, ar = kn.jones(q, t, m, e)
        vo, _ = ojones.jones_value(q, tg.n_vertices, tg.writhe, tg.tait_number, mo, eo)
        assert rel_err(v, vo) <= TOL
        if d.n <= 14:
            poly = kauffman.jones_polynomial(d.pd, int(d.signs.sum()))
            assert rel_err(v, kauffman.evaluate(poly, ojones.t_of_q(q))) <= TOL


def test_paper_printed_values():
    golden = os.path.join(os.path.dirname(__file__), "golden", "paper_fig1.txt")
    fx = {"trefoil": gen.trefoil, "unknot": lambda: gen.UNKNOT}
    for line in open(golden):
        if not line.strip() or line.startswith("#"):
            continue
        name, q, re_, im_, src = line.split()
        t, p, m, e = gpu_z(fx[name](), int(q))
        v, _, _ = kn.jones(int(q), t, m, e)
        want = complex(float(re_), float(im_))
        assert abs(v - want) <= 1e-12 * max(1, abs(want)), (name, q, v, want)


@pytest.mark.parametrize("q", [3, 5])
def test_fp64_config_parity(q):
    """The 50-200 crossing workload (64 knots, one knot per launch) against
    the oracle's stored values (tests/golden/oracle_fp64_seed0.json)."""
    import json
    _log(f"fp64 config q={q}")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "oracle_fp64_seed0.json")) as f:
        gold = json.load(f)["knots"]
    knots = gen.config_knots("fp64", 0)
    assert len(knots) == len(gold) == 128
    worst = 0.0
    for (d, qq), g in zip(knots, gold):
        assert (d.label, d.n, qq) == (g["label"], g["crossings"], g["q"])
        if qq != q:
            continue
        t, p, m, e = gpu_z(d, q)
        err = rel_err(m * 2.0 ** (e - g["z_exp2"]), complex(g["z_re"], g["z_im"]))
        worst = max(worst, err)
        assert err <= TOL, (d.label, q, err)
    _log(f"worst relative error {worst:.1e}")


@pytest.mark.parametrize("q", [2, 4, 6, 7, 8])
def test_other_q_parity(q):
    _log(f"q={q}")
    for k in range(6):
        d = gen.lattice_knot((61, k), 40, 150)
        t, p, m, e = gpu_z(d, q)
        tg, mo, eo = oracle_z(d, q)
        assert z_close(m, e, mo, eo), (k, q)


def test_full_size_parity_sample():
    """200-600 crossings at q=3 (the throughput workload): every knot is checked
    against the oracle and the Lickorish-Millett class of V(e^{i pi/3})."""
    _log("200-600 crossings, q=3")
    for d, q in gen.config_knots("q3_200_600", 0, count=24):
        t, p, m, e = gpu_z(d, q)
        tg, mo, eo = oracle_z(d, q)
        assert z_close(m, e, mo, eo), d.label
        v, l2, ar = kn.jones(q, t, m, e)
        dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
        assert abs(l2 - dd * math.log2(3) / 2) < 1e-9
        ratio = complex(math.cos(ar), math.sin(ar)) / unit
        assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9


def test_invariants_q2_q4_large():
    _log("q=2 Arf / q=4 identity on 300-600 crossings")
    for k in range(6):
        d = gen.lattice_knot((62, k), 300, 600)
        tg = oracle_tait(d)
        t, p, m, e = gpu_z(d, 4)
        v, l2, ar = kn.jones(4, t, m, e)
        assert abs(v - 1) < 1e-9
        t, p, m, e = gpu_z(d, 2)
        v, l2, ar = kn.jones(2, t, m, e)
        assert abs(v - invariants.v_at_q2(tg.n_vertices, tg.edges, tg.eps)) < 1e-9


def test_tiled_steps_parity():
    """Force every sizeable step across workgroups (tile tasks + counters)."""
    _log("tiled steps")
    for k in range(6):
        d = gen.lattice_knot((63, k), 100, 400)
        for kw in (dict(big_step_macs_log2=4, tile_outputs=8),
                   dict(big_step_macs_log2=8, tile_outputs=64)):
            t, p, m, e = gpu_z(d, 3, **kw)
            tg, mo, eo = oracle_z(d, 3)
            assert z_close(m, e, mo, eo), (k, kw)


def test_gemm_and_split_parity():
    """32 x 32 GEMM tiles (ragged row and column blocks), GEMM tiles over a
    split contracted range with their reduction, and split output tiles."""
    work = gen.config_knots("q3_200_600", 0, count=72)
    cases = [(71, work[71][0], dict(strategy=0, simplify=3)), (11, work[11][0], dict(simplify=3)),
             (11, work[11][0], {})]
    for k in range(3):
        cases.append((f"lattice{k}", gen.lattice_knot((63, k), 100, 400),
                      dict(big_step_macs_log2=4)))
    # several 32 x 32 blocks per task (ragged last task of a step)
    cases.append((71, work[71][0], dict(strategy=0, simplify=3, gemm_tasks_log2=1)))
    cases.append((11, work[11][0], dict(gemm_tasks_log2=3)))
    cases.append(("lattice0", gen.lattice_knot((63, 0), 100, 400),
                  dict(big_step_macs_log2=4, gemm_tasks_log2=2)))
    for name, d, kw in cases:
        kw = dict(kw, split_min_log2=7)  # segments of 128 entries: GEMM steps split too
        _log(f"gemm/split case {name} {kw}")
        tg, mo, eo = oracle_z(d, 3)
        for prec in (0, 1):
            t, p, m, e = gpu_z(d, 3, precision=prec, **kw)
            tol = TOL if prec == 0 else TOL32
            assert z_close(m, e, mo, eo, tol), (name, kw, prec)


def test_gemm64_parity():
    """64 x 64 GEMM blocks (4 x 4 outputs per thread): ragged sides, several
    blocks per task, a split contracted range with its reduction; complex128
    and complex64."""
    from tests.test_host import gemm64_cases
    for label, d, q, kw in gemm64_cases():
        _log(f"gemm64 case {label} q={q} {kw}")
        tg, mo, eo = oracle_z(d, q)
        for prec in (0, 1):
            t, p, m, e = gpu_z(d, q, precision=prec, **kw)
            tol = TOL if prec == 0 else TOL32
            assert z_close(m, e, mo, eo, tol), (label, kw, prec)


def test_gemm64_split_ragged_full_size():
    """The workload's largest knot (571 crossings) with its ragged split GEMM
    step in 64 x 64 blocks, one block per task and grouped: checked against
    the q=3 Lickorish-Millett class of V(e^{i pi/3}) (the oracle takes too long
    at this size)."""
    d = gen.config_knots("q3_200_600", 0, count=79)[78][0]
    tg = oracle_tait(d)
    dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
    for kw in (dict(gemm64_pct=100000, gemm_tasks_log2=30, split_min_log2=7),
               dict(gemm64_pct=100000, gemm_tasks_log2=1, split_min_log2=7),
               dict(gemm64_pct=100000)):
        _log(f"gemm64 knot 78 {kw}")
        t, p, m, e = gpu_z(d, 3, **kw)
        v, l2, ar = kn.jones(3, t, m, e)
        assert abs(l2 - dd * math.log2(3) / 2) < 1e-9, kw
        ratio = complex(math.cos(ar), math.sin(ar)) / unit
        assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9, kw


# complex64 with the series-parallel reduction at real t (q >= 4): the
# derived couplings x' = (x1 x2 + q - 1) / (x1 + x2 + q - 2) mix terms of
# both signs, and the contraction of such couplings loses a few more bits to
# cancellation than the Jones point of the workloads (measured 1.7e-5 at
# q = 5 against ~2e-6 at q = 3): ten times TOL32.
TOL32_SP = 10 * TOL32


def test_series_parallel_parity():
    """simplify bit 2 (exact series-parallel reduction at the Jones couplings:
    derived edges and constant factors from the plan's constants)."""
    for k in range(6):
        d = gen.lattice_knot((87, k), 40, 200)
        tg, mo, eo = oracle_z(d, 3 + (k % 3))
        for prec in (0, 1):
            t, p, m, e = gpu_z(d, 3 + (k % 3), precision=prec, simplify=7)
            tol = TOL if prec == 0 else TOL32_SP
            _log(f"series-parallel {k} q={3 + k % 3} precision {prec}: "
                 f"{rel_err(m * 2.0 ** (e - eo), mo):.1e}")
            assert z_close(m, e, mo, eo, tol), (d.label, prec)


def test_level_split_parity():
    """Serial runs executed level by level over several workgroups (setup and
    final product as tasks of their own, each level's steps in chunks), for
    single plans and a batch, complex128 and complex64."""
    cases = [gen.lattice_knot((84, k), 60, 200) for k in range(4)]
    cases.append(gen.config_knots("q3_200_600", 0, count=72)[11][0])
    for d in cases:
        tg, mo, eo = oracle_z(d, 3)
        for split in (3, 6):
            _log(f"level split {d.label} n={d.n} split_serial_log2={split}")
            for prec in (0, 1):
                t, p, m, e = gpu_z(d, 3, precision=prec, split_serial_log2=split)
                tol = TOL if prec == 0 else TOL32
                assert z_close(m, e, mo, eo, tol), (d.label, split, prec)
    taits = [kn.Tait(d.pd) for d in cases]
    plans = [kn.Plan(t, 3, split_serial_log2=(3 if i % 2 else 40)) for i, t in enumerate(taits)]
    z = kn.Batch(plans).contract()
    torch.cuda.synchronize()
    for (m, e), d in zip(kn.scalars_from_device(z), cases):
        tg, mo, eo = oracle_z(d, 3)
        assert z_close(m, e, mo, eo, TOL), d.label


def test_exact_ring_parity():
    """Bit-for-bit-exact reference (Z in Z[t]) on mid-size knots."""
    for k in range(4):
        d = gen.lattice_knot((64, k), 40, 100)
        for q in (3, 5):
            t, p, m, e = gpu_z(d, q)
            tg = oracle_tait(d)
            ab = exact.partition_function_exact(tg.n_vertices, tg.edges, tg.eps, q)
            me, ee = exact.to_mant_exp2(ab, q)
            assert z_close(m, e, me, ee), (k, q)


def test_batch_parity():
    _log("batch of 48 mixed knots")
    knots = gen.config_knots("batched", 0, count=48)
    plans = [kn.Plan(kn.Tait(d.pd), q) for d, q in knots]
    b = kn.Batch(plans)
    z = b.contract()
    torch.cuda.synchronize()
    out = kn.scalars_from_device(z)
    for (d, q), (m, e) in zip(knots, out):
        tg, mo, eo = oracle_z(d, q)
        assert z_close(m, e, mo, eo), (d.label, q)
    # a second launch on the same workspace gives identical bits
    z2 = b.contract()
    torch.cuda.synchronize()
    assert torch.equal(z.view(torch.int64), z2.view(torch.int64))


def test_forked_runs_parity():
    """Long serial runs forked into concurrent subtree tasks (the vertex
    tensors, up to 8 subtree tasks on their own workgroups, the steps above
    them), alone and in a batch, complex128 and complex64, against the
    oracle; a second launch gives identical bits."""
    knots = gen.config_knots("q3_200_600", 0, count=24)
    for prec, tol in ((0, TOL), (1, TOL32)):
        for fork in (6, 9):
            _log(f"forked runs: 2^{fork}, precision {prec}")
            plans = [kn.Plan(kn.Tait(d.pd), q, fork_serial_log2=fork, precision=prec)
                     for d, q in knots]
            b = kn.Batch(plans)
            z = b.contract()
            torch.cuda.synchronize()
            for (d, q), (m, e) in zip(knots, kn.scalars_from_device(z)):
                tg, mo, eo = oracle_z(d, q)
                assert rel_err(m * 2.0 ** (e - eo), mo) <= tol, (d.label, fork, prec)
            z2 = b.contract()
            torch.cuda.synchronize()
            assert torch.equal(z.view(torch.int64), z2.view(torch.int64))
    d, q = knots[3]
    t, p, m, e = gpu_z(d, q, fork_serial_log2=5)
    tg, mo, eo = oracle_z(d, q)
    assert z_close(m, e, mo, eo)


def test_bench_configuration_parity():
    """The batch exactly as bench.py times it: the 256 knots of the 200-600
    crossing workload planned as one PlanSet (min-fill orders, the tuned
    setting and grid), uploaded on a side stream and contracted on another
    behind the upload event; complex128 and complex64.  The first 24 knots are
    checked against the oracle; every fourth knot and the largest (571
    crossings) against the q=3 Lickorish-Millett class of V(e^{i pi/3})."""
    _log("bench configuration: 256 knots, plan set, tuned setting")
    knots = gen.config_knots("q3_200_600", 0, count=256)
    ncr = np.array([d.n for d, _ in knots], np.int32)
    flat = np.concatenate([np.asarray(d.pd, np.int32).reshape(-1) for d, _ in knots])
    oracle = {i: oracle_z(knots[i][0], 3) for i in range(24)}
    inv = {}
    for i in sorted(set(range(0, 256, 4)) | {78}):
        tg = oracle_tait(knots[i][0])
        inv[i] = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
    for prec in (0, 1):
        _log(f"bench configuration, precision {prec}")
        setting = tune.load("q3_200_600", prec)
        opts = {k: v for k, v in setting.items() if k != "grid"}
        ps = kn.plan_set(ncr, flat, 3, strategy=2, precision=prec, **opts)
        b = kn.Batch(ps)
        if setting.get("grid"):
            b.set_grid(int(setting["grid"]))
        side, main = torch.cuda.Stream(), torch.cuda.current_stream()
        ws = kn.alloc_workspace(b.workspace_bytes)
        b.upload(ws, side)
        uploaded = torch.cuda.Event()
        uploaded.record(side)
        main.wait_event(uploaded)
        z = b.contract(stream=main)
        torch.cuda.synchronize()
        out = kn.scalars_from_device(z)
        tol, itol = (TOL, 1e-9) if prec == 0 else (TOL32, TOL32)
        for i, (tg, mo, eo) in oracle.items():
            m, e = out[i]
            assert z_close(m, e, mo, eo, tol), (i, prec)
        for i, (dd, unit) in inv.items():
            m, e = out[i]
            v, l2, ar = kn.jones(3, ps.tait(i), m, e)
            assert abs(l2 - dd * math.log2(3) / 2) < itol, (i, prec)
            ratio = complex(math.cos(ar), math.sin(ar)) / unit
            assert min(abs(ratio - 1), abs(ratio + 1)) < itol, (i, prec)


def test_batch_small_grid():
    """Any grid size completes (tasks are taken in dependency order)."""
    knots = gen.config_knots("batched", 1, count=12)
    plans = [kn.Plan(kn.Tait(d.pd), q, big_step_macs_log2=6, tile_outputs=32) for d, q in knots]
    b = kn.Batch(plans)
    for g in (1, 3, 64):
        b.set_grid(g)
        z = b.contract()
        torch.cuda.synchronize()
        for (d, q), (m, e) in zip(knots, kn.scalars_from_device(z)):
            tg, mo, eo = oracle_z(d, q)
            assert z_close(m, e, mo, eo), (g, d.label)


def test_general_couplings_parity():
    rng = np.random.default_rng(5)
    for k in range(5):
        d = gen.lattice_knot((65, k), 30, 200)
        t = kn.Tait(d.pd)
        p = kn.Plan(t, 3, jones_only=False)
        Jh = rng.normal(scale=0.4, size=2 * t.n_edges)
        J = torch.tensor(Jh, dtype=torch.float64, device="cuda")
        z = kn.contract(p, J=J)
        torch.cuda.synchronize()
        (m, e), = kn.scalars_from_device(z)
        uv, eps = t.edges()
        x = np.exp(Jh[0::2] + 1j * Jh[1::2])
        mo, eo = potts.partition_function(t.n_vertices, [tuple(a) for a in uv], x, 3)
        assert z_close(m, e, mo, eo), k


def test_fp32_path_error_bound():
    """complex64 tensors, FP32 accumulation: error against the FP64 oracle,
    per knot within TOL32 (a few times the FP32 rounding random walk along
    the contraction; see tests/oracle_helpers)."""
    errs = []
    for d, q in gen.config_knots("q3_200_600", 0, count=8):
        t, p, m, e = gpu_z(d, q, precision=1)
        tg, mo, eo = oracle_z(d, q)
        errs.append(rel_err(m * 2.0 ** (e - eo), mo))
    _log(f"fp32 rel errors: {['%.1e' % x for x in errs]}")
    assert max(errs) < TOL32


def test_special_cases():
    for d in (gen.UNKNOT, gen.add_kink(gen.UNKNOT, 0, True, 1),
              gen.add_kink(gen.add_kink(gen.UNKNOT, 0, False, -1), 1, True, 1)):
        for q in (2, 3, 5):
            t, p, m, e = gpu_z(d, q)
            v, _, _ = kn.jones(q, t, m, e)
            assert abs(v - 1) < 1e-12, (d.label, q)


def test_api_errors():
    t = kn.Tait(gen.figure_eight().pd)
    p = kn.Plan(t, 3)
    J = torch.zeros(2 * t.n_edges, dtype=torch.float64, device="cuda")
    with pytest.raises(kn.KnError) as e:
        kn.contract(p, J=J)     # Jones-only plan with explicit couplings
    assert e.value.code == -6
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(kn.KnError) as e:
        kn.contract(p, workspace=small)
    assert e.value.code == -3


def test_staged_serial_steps_same_bits():
    """Serial steps that the whole workgroup computes copy their global
    operands into the LDS staging area after the tensor arena when they fit.
    The staging changes where a step reads its operands, not what it adds:
    the same knots planned with a 48 KiB tensor arena (a 64 KiB staging area)
    and with a 128 KiB one (a 1.75 KiB staging area, so that almost nothing
    is staged) give the same bits, in complex128 and complex64, and the first
    knots match the oracle."""
    from tests import image_model as im

    knots = gen.config_knots("q3_200_600", 5, count=32)
    ncr = np.array([d.n for d, _ in knots], np.int32)
    flat = np.concatenate([np.asarray(d.pd, np.int32).reshape(-1) for d, _ in knots])
    oracle = {i: oracle_z(knots[i][0], 3) for i in range(4)}
    for prec in (0, 1):
        bits = []
        for lds in (49152, 131072):
            ps = kn.plan_set(ncr, flat, 3, strategy=2, precision=prec, lds_bytes=lds)
            b = kn.Batch(ps)
            if lds == 49152:
                # whole-workgroup serial steps (one step in its level, or at
                # least 2048 products) with a global operand that fits 4096
                # entries: steps that take the staging path
                img = im.Image(b.image())
                st = img.steps
                ser = st[st["mode"] == 0]
                macs = ser["nb"].astype(np.int64) * ser["nm"] * ser["nn"] * ser["nk"]
                na = ser["nb"].astype(np.int64) * ser["nm"] * ser["nk"]
                glob_a = (ser["home_a"] >= 0) & (na <= 4096)
                assert int((glob_a & (macs >= 2048)).sum()) > 0
            _log(f"staging: precision {prec}, lds_bytes {lds}")
            z = b.contract()
            torch.cuda.synchronize()
            bits.append(z.cpu().numpy().view(np.int64).copy())
            out = kn.scalars_from_device(z)
            tol = TOL if prec == 0 else TOL32
            for i, (tg, mo, eo) in oracle.items():
                m, e = out[i]
                assert z_close(m, e, mo, eo, tol), (i, prec, lds)
        assert np.array_equal(bits[0], bits[1]), prec
