"""The per-task trace tool (paper_1807_02119_amd/trace.py) on the CPU: its
decoding of the device program agrees with the independent image model, and
its report reads a synthetic trace (the GPU capture itself is exercised by
the profiling runs)."""

from __future__ import annotations

import numpy as np

from paper_1807_02119_amd import gen, kn, trace
from tests import image_model as im


def _batch(count=12):
    knots = gen.config_knots("q3_200_600", 0, count=count)
    _, plans = kn.plan_many([np.ascontiguousarray(d.pd, np.int32) for d, _ in knots], 3,
                            strategy=2)
    return knots, kn.Batch(plans)


def test_decode_matches_image_model():
    _, b = _batch()
    raw = b.image()
    h, tasks, steps = trace._decode(raw)
    ref = im.Image(raw)
    assert int(h["n_tasks"]) == len(ref.tasks) and int(h["n_steps"]) == len(ref.steps)
    for f in trace._TASK.names:
        assert (tasks[f] == ref.tasks[f]).all(), f
    for f in trace._STEP.names:
        assert (steps[f] == ref.steps[f]).all(), f


def test_report_on_a_synthetic_trace():
    knots, b = _batch()
    _, tasks, steps = trace._decode(b.image())
    n = len(tasks)
    rng = np.random.default_rng(0)
    # every group after its predecessor: tasks in image order, 5 us apart
    start = np.arange(n) * 5.0
    t = dict(t_claim=start - 1.0, t_start=start, t_end=start + rng.uniform(1, 4, n),
             ph=np.zeros((n, 4)), kind=tasks["kind"], knot=tasks["knot"], group=tasks["group"],
             first=tasks["first"], count=tasks["count"],
             mode=np.where(tasks["kind"] == 0, -1,
                           steps["mode"][np.minimum(tasks["first"], len(steps) - 1)]),
             ncr=np.array([d.n for d, _ in knots]), steps=steps, grid=None)
    text = trace.report(t, 1.0, n_wg=4)
    last = int(tasks["knot"][n - 1])
    assert f"Group chain of knot {last}" in text
    assert "| serial |" in text and "Busy workgroups" in text
