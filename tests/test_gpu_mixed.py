"""The mixed-precision workload: 16 seeded lattice knots of 300-600 crossings
(at least 4 of 560-600), q = 3.  Every knot contracted on the GPU in
complex128 and in complex64 (FP32 tensors and FP32 accumulation on the
matrix cores, power-of-two exponents and the final normalisation in
FP64/int64), in one batch and one knot per launch, against the oracle's
stored values (tests/golden/oracle_mixed_seed0.json, written by
tests/golden/make_oracle_values.py from oracle/ alone): complex128 to 1e-10
relative per knot, complex64 to TOL32 per knot (Z and V)."""

from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_02119_amd import gen, kn, tune
from tests.oracle_helpers import TOL32, TOL64, close_log, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_mixed_seed0.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def _workload():
    with open(GOLDEN) as f:
        gold = json.load(f)["knots"]
    knots = gen.config_knots("mixed", 0)
    assert len(knots) == len(gold) == 16
    for (d, q), g in zip(knots, gold):
        assert (d.label, d.n, q) == (g["label"], g["crossings"], g["q"])
    assert sum(d.n >= 560 for d, _ in knots) >= 4
    return knots, gold


def _errors(out, gold, taits):
    ez, ev = [], []
    for (m, e), g, t in zip(out, gold, taits):
        mo = complex(g["z_re"], g["z_im"])
        ez.append(rel_err(m * 2.0 ** (e - g["z_exp2"]), mo))
        v, l2, ar = kn.jones(g["q"], t, m, e)
        dv = 2.0 ** (l2 - g["v_log2_abs"]) * complex(math.cos(ar - g["v_arg"]),
                                                     math.sin(ar - g["v_arg"]))
        ev.append(abs(dv - 1.0))
    return np.array(ez), np.array(ev)


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_workload_batch(precision):
    knots, gold = _workload()
    pds = [np.ascontiguousarray(d.pd, np.int32) for d, _ in knots]
    setting = tune.load("q3_200_600", precision)
    taits, plans = kn.plan_many(pds, 3, precision=precision, **tune.plan_options(setting))
    b = kn.Batch(plans)
    if setting.get("grid"):
        b.set_grid(int(setting["grid"]))
    z = b.contract()
    torch.cuda.synchronize()
    ez, ev = _errors(kn.scalars_from_device(z), gold, taits)
    tol = TOL64 if precision == 0 else TOL32
    print(f"precision {precision}: per-knot rel. error of Z "
          f"{' '.join('%.1e' % x for x in ez)}; max V error {ev.max():.2e}", flush=True)
    assert ez.max() <= tol and ev.max() <= tol


def test_mixed_workload_one_knot_per_launch():
    knots, gold = _workload()
    for precision in (0, 1):
        tol = TOL64 if precision == 0 else TOL32
        for (d, q), g in zip(knots, gold):
            t = kn.Tait(d.pd)
            p = kn.Plan(t, q, precision=precision)
            z = kn.contract(p)
            torch.cuda.synchronize()
            ez, ev = _errors(kn.scalars_from_device(z), [g], [t])
            assert ez[0] <= tol and ev[0] <= tol, (d.label, precision, ez[0], ev[0])
