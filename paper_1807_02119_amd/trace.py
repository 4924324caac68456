"""Per-task trace of one persistent batch launch, and where its time goes.

    python -m paper_1807_02119_amd.trace [--batch 256] [--seed 0] [--grid G]
                                         [--fork-log2 F] [--md FILE]

Plans the bench's workload (seeded lattice-walk knots of 200-600 crossings,
q = 3, complex128, min-fill orders, the autotuned setting of
``tuned/q3_200_600.json``), launches the batch a few times, then once more
with per-task timing on (``kn.Batch.set_trace``: the device clock at claim,
start and end of every task, and the phases of serial tasks).  Printed: the
launch time, busy time per task kind, the knots that finish last, the chain
of task groups of the last one (start, duration and the gap before each
group) and the number of busy workgroups over the launch.  Needs a GPU.
"""

from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1807_02119_amd import gen, kn, tune  # noqa: E402

# The leading fields of the device-program header (csrc/program.h ImgHeader):
# 22 int32 counts, then the int64 section offsets in declaration order.
_HDR = np.dtype([(f, "<i4") for f in (
    "magic", "precision", "n_tasks", "n_knots", "n_tensors", "n_steps", "n_vtx", "n_medges",
    "n_members", "n_factors", "n_strides", "n_groups", "n_edges", "n_roots", "lds_bytes",
    "n_pins", "n_wslots", "n_outputs", "sliced", "n_consts", "n_queue", "n_zslice")]
    + [(f, "<i8") for f in ("o_tasks", "o_groups", "o_roots", "o_knots", "o_tensors",
                             "o_steps")])
_TASK = np.dtype([(f, "<i4") for f in ("kind", "knot", "group", "first", "count", "flags",
                                       "state_lo", "state_len")])
_STEP = np.dtype([(f, "<i4") for f in ("a", "b", "c", "nb", "nm", "nn", "nk", "str", "ranks",
                                       "n_tiles", "tile", "home_a", "home_b", "home_c", "mode",
                                       "n_mb", "n_nb", "n_ks", "kseg", "partial", "lvl")])
_KINDS = {0: "serial", 1: "tile", 2: "reduce"}
_MODES = {0: "serial", 1: "tiles", 2: "gemm32", 3: "gemm64"}
_TICK_US = 0.01  # the device clock runs at 100 MHz


def _decode(raw: bytes):
    h = np.frombuffer(raw, _HDR, 1)[0]
    tasks = np.frombuffer(raw, _TASK, int(h["n_tasks"]), int(h["o_tasks"]))
    steps = np.frombuffer(raw, _STEP, int(h["n_steps"]), int(h["o_steps"]))
    return h, tasks, steps


def capture(batch_size=256, seed=0, grid=0, fork_log2=0, warm=3, timed=10):
    """Trace one launch of the bench's batch; returns a dict of numpy arrays
    (times in microseconds from the first claim) and the launch time."""
    import torch

    knots = gen.config_knots("q3_200_600", seed, count=batch_size)
    pds = [np.ascontiguousarray(d.pd, dtype=np.int32) for d, _ in knots]
    ncr = np.asarray([d.n for d, _ in knots], np.int32)
    flat = np.concatenate([p.reshape(-1) for p in pds])
    tuned = tune.load("q3_200_600", 0)
    opts = {k: v for k, v in tuned.items() if k != "grid"}
    opts["strategy"] = 2
    if fork_log2:
        opts["fork_serial_log2"] = fork_log2
    ps = kn.plan_set(ncr, flat, 3, **opts)
    b = kn.Batch([ps.plan(i) for i in range(len(ps))])
    g = grid or int(tuned.get("grid") or 0)
    if g:
        b.set_grid(g)
    h, tasks, steps = _decode(b.image())
    b.upload()
    z = kn.alloc_scalars(len(ps))
    for _ in range(warm):
        b.contract(z=z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    e0.record(st)
    for _ in range(timed):
        b.contract(z=z)
    e1.record(st)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / timed
    buf = torch.zeros(64 * int(h["n_tasks"]), dtype=torch.uint8, device="cuda")
    b.set_trace(buf)
    b.contract(z=z)
    torch.cuda.synchronize()
    b.set_trace(None)
    rec = kn.Batch.decode_trace(buf.cpu().numpy().tobytes())
    t0 = rec["t_claim"].min()
    us = lambda x: (x.astype(np.int64) - t0) * _TICK_US  # noqa: E731
    # (a serial task's first step may be one past the last: it is not looked up)
    mode = np.where(tasks["kind"] == 0, -1,
                    steps["mode"][np.minimum(tasks["first"], max(len(steps) - 1, 0))])
    return dict(t_claim=us(rec["t_claim"]), t_start=us(rec["t_start"]), t_end=us(rec["t_end"]),
                ph=rec["ph"] * _TICK_US, kind=tasks["kind"].copy(), knot=tasks["knot"].copy(),
                group=tasks["group"].copy(), first=tasks["first"].copy(),
                count=tasks["count"].copy(), mode=mode, ncr=ncr, steps=steps,
                grid=g or None), launch_ms


def report(t, launch_ms, n_wg=256):
    """Text summary of a trace from capture()."""
    ts, te, tc = t["t_start"], t["t_end"], t["t_claim"]
    kind, knot, group, mode, steps = t["kind"], t["knot"], t["group"], t["mode"], t["steps"]
    span = te.max()
    busy = te - ts
    out = [f"launch {launch_ms * 1e3:.0f} us (events, mean of the timed launches); traced "
           f"launch {span:.0f} us, {len(te)} tasks, grid {t['grid'] or 'one workgroup per CU'}",
           f"workgroups busy {100 * busy.sum() / (n_wg * span):.1f} % of {n_wg} x the traced "
           f"launch; claim-to-start waits {(ts - tc).sum() / 1e3:.1f} WG-ms", "",
           "| task kind | tasks | busy WG-ms | mean us |", "|---|---|---|---|"]
    for k in (0, 1, 2):
        m = kind == k
        if m.any():
            out.append(f"| {_KINDS[k]} | {m.sum()} | {busy[m].sum() / 1e3:.1f} | "
                       f"{busy[m].mean():.1f} |")
    for md in (1, 2, 3):
        m = (kind == 1) & (mode == md)
        if m.any():
            out.append(f"| tile, {_MODES[md]} | {m.sum()} | {busy[m].sum() / 1e3:.1f} | "
                       f"{busy[m].mean():.1f} |")
    m = kind == 1
    if m.any():
        ph = t["ph"][m]
        rest = busy[m] - ph[:, :3].sum(axis=1)
        out += ["", "Tile tasks, mean us: descriptors, tables and operand states "
                f"{ph[:, 0].mean():.1f}; products {ph[:, 1].mean():.1f}; publish of C's shift "
                f"{ph[:, 2].mean():.1f}; release and enqueue {rest.mean():.1f}"]
    nk = int(knot.max()) + 1
    kend = np.zeros(nk)
    np.maximum.at(kend, knot, te)
    order = np.argsort(-kend)
    out += ["", "Knots finishing last: " + ", ".join(
        f"knot {k} ({t['ncr'][k]} crossings) at {kend[k]:.0f} us" for k in order[:6])]
    k = int(order[0])
    out += ["", f"Group chain of knot {k} ({t['ncr'][k]} crossings):", "",
            "| group | kind | tasks | steps or step shape (nb nm nn nk) | start us | duration us "
            "| gap before us |", "|---|---|---|---|---|---|---|"]
    idx = np.where(knot == k)[0]
    prev = 0.0
    run = gaps = 0.0
    for g in sorted(set(group[idx].tolist())):
        m = idx[group[idx] == g]
        g0, g1 = ts[m].min(), te[m].max()
        i = m[0]
        if kind[i] == 0:
            what = f"{int(t['count'][m].sum())} steps"
            if len(m) == 1:
                what += " (phases us: setup {:.0f}, tables {:.0f}, products {:.0f}, other {:.0f})" \
                    .format(*t["ph"][i])
        else:
            s = steps[t["first"][i]]
            what = f"{_MODES[int(s['mode'])]} {s['nb']} {s['nm']} {s['nn']} {s['nk']}"
        out.append(f"| {g} | {_KINDS[int(kind[i])]} | {len(m)} | {what} | {g0:.0f} | "
                   f"{g1 - g0:.0f} | {g0 - prev:.0f} |")
        run += g1 - g0
        gaps += max(0.0, g0 - prev)
        prev = g1
    out += ["", f"Chain: {run:.0f} us running, {gaps:.0f} us waiting between groups."]
    bins = np.linspace(0, span, 21)
    occ = [np.clip(np.minimum(te, bins[j + 1]) - np.maximum(ts, bins[j]), 0, None).sum()
           / (bins[j + 1] - bins[j]) for j in range(20)]
    out += ["", "Busy workgroups in each twentieth of the launch: "
            + " ".join(f"{x:.0f}" for x in occ)]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="persistent grid (0: tuned / one per CU)")
    ap.add_argument("--fork-log2", type=int, default=0,
                    help="fork threshold of serial runs (0: tuned setting)")
    ap.add_argument("--md", default="", help="also write the summary to this file")
    args = ap.parse_args()
    t, ms = capture(args.batch, args.seed, args.grid, args.fork_log2)
    text = report(t, ms, n_wg=args.grid or 256)
    print(text, flush=True)
    if args.md:
        with open(args.md, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
