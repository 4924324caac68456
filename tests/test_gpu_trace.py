"""Per-task tracing of a batch launch (kn.Batch.set_trace, used by
paper_1807_02119_amd.trace): a traced launch gives the bits of an untraced
one, every task has one record with claim <= start <= end, the phases of a
tile task fit inside its run time, and the trace tool's report reads it."""

from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_02119_amd import gen, kn, trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def test_traced_launch_records_every_task_and_keeps_the_bits():
    knots = gen.config_knots("q3_200_600", 3, count=24)
    _, plans = kn.plan_many([np.ascontiguousarray(d.pd, np.int32) for d, _ in knots], 3,
                            strategy=2)
    b = kn.Batch(plans)
    _, tasks, steps = trace._decode(b.image())
    n = len(tasks)
    assert (tasks["kind"] == 1).any(), "the batch should hold tiled steps"
    b.upload()
    z0 = b.contract()
    torch.cuda.synchronize()
    ref = z0.cpu().numpy().copy()
    buf = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    b.set_trace(buf)
    z1 = b.contract()
    torch.cuda.synchronize()
    b.set_trace(None)
    assert np.array_equal(z1.cpu().numpy().view(np.int64), ref.view(np.int64))
    rec = kn.Batch.decode_trace(buf.cpu().numpy().tobytes())
    print(f"{n} tasks, {int(((rec['t_end'] - rec['t_start']) // 100).max())} us longest",
          flush=True)
    assert np.array_equal(np.sort(rec["task"]), np.arange(n))
    assert (rec["t_claim"] > 0).all()
    assert (rec["t_claim"] <= rec["t_start"]).all() and (rec["t_start"] <= rec["t_end"]).all()
    order = np.argsort(rec["task"])
    run = (rec["t_end"] - rec["t_start"])[order]
    ph = rec["ph"][order]
    tile = tasks["kind"] == 1
    assert (ph[tile][:, :3] >= 0).all() and (ph[tile][:, 3] == 0).all()
    assert (ph[tile][:, :3].sum(axis=1) <= run[tile]).all()
    assert (ph[tasks["kind"] == 2] == 0).all()
    t0 = rec["t_claim"].min()
    us = lambda x: (x.astype(np.int64)[order] - t0) * 0.01  # noqa: E731
    t = dict(t_claim=us(rec["t_claim"]), t_start=us(rec["t_start"]), t_end=us(rec["t_end"]),
             ph=rec["ph"][order] * 0.01, kind=tasks["kind"], knot=tasks["knot"],
             group=tasks["group"], first=tasks["first"], count=tasks["count"],
             mode=np.where(tasks["kind"] == 0, -1,
                           steps["mode"][np.minimum(tasks["first"], len(steps) - 1)]),
             ncr=np.array([d.n for d, _ in knots]), steps=steps, grid=None)
    text = trace.report(t, 1.0)
    assert "Group chain of knot" in text and "Tile tasks, mean us" in text
