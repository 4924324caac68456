"""Autotuner for batched contraction.

How a step runs is decided by planner knobs:
- big_step_macs_log2 / big_step_outs_log2: the multiply-add count, and the
  output count, from which a step is split into tiles over workgroups
  instead of running inside a serial task;
- tile_macs_log2 / tile_outs_log2: how much work, and at most how many
  outputs, one tile of outputs carries;
- lds_bytes: the per-workgroup LDS arena for tensors that stay inside one
  serial task, which also sets how many workgroups fit on a compute unit;
- gemm_tasks_log2: how many tasks a step computed in output blocks is cut
  into (several blocks per task above that);
- gemm64_pct: how much padding a step accepts to use 64 x 64 output blocks
  instead of 32 x 32 ones;
- split_serial_log2: from which estimated length a run of small steps is
  executed level by level over several workgroups;
- split_min_log2: how many contracted entries (at least) one segment of a
  split contracted index holds;
- fork_serial_log2: from which estimated length a run of small steps is
  forked into concurrent subtree tasks.
The persistent kernel's grid is one more knob.  The tile-shape knobs
(tile_macs_log2, tile_outs_log2, gemm64_pct, gemm_tasks_log2) can also be
set per intermediate-size bucket (steps whose output has at most 2^8, 2^12,
2^16, 2^20 or more entries).

The tuner times kn_batch_contract with HIP events (on the launch stream) on
a sample of a workload.  It searches the plan-wide knobs and the grid by
coordinate descent from the defaults, then the per-bucket knobs by
coordinate descent from that setting.  At the end it times the defaults and
the best setting again, alternately, to state the gain against run-to-run
noise.  It writes the best setting, with the full table of measurements, to
a JSON file.  bench.py and users load it with ``load``.

    python -m paper_1807_02119_amd.tune --workload q3_200_600 --count 256 --strategy 2
    python -m paper_1807_02119_amd.tune --workload batched --count 512 --precisions 0
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

SPACE = {
    "big_step_macs_log2": [14, 15, 16, 17, 18],
    "big_step_outs_log2": [10, 11, 12, 13, 14, 31],
    "tile_macs_log2": [13, 14, 15, 16, 17],
    "tile_outs_log2": [8, 9, 10, 11, 12, 14],
    "lds_bytes": [16384, 24576, 32768, 49152],
    "gemm_tasks_log2": [4, 5, 6, 7, 30],
    "gemm64_pct": [1, 150, 300],
    "split_serial_log2": [8, 10, 12, 40],
    "split_min_log2": [9, 10, 11, 12, 13, 14],
    "fork_serial_log2": [8, 9, 10, 11, 40],
}
BUCKET_SPACE = {
    "tile_macs_log2": [12, 13, 14, 15, 16, 17],
    "tile_outs_log2": [7, 8, 9, 10, 11, 12],
    "gemm64_pct": [1, 150, 300, 1000],
    "gemm_tasks_log2": [3, 4, 5, 6, 7, 30],
}
N_BUCKETS = 5
DEFAULTS = {"big_step_macs_log2": 16, "big_step_outs_log2": 12, "tile_macs_log2": 15,
            "tile_outs_log2": 10, "lds_bytes": 24576, "gemm_tasks_log2": 5, "gemm64_pct": 300,
            "split_serial_log2": 40, "split_min_log2": 12, "fork_serial_log2": 10, "grid": 0}
DEFAULTS_KEY = json.dumps(DEFAULTS, sort_keys=True)
TUNED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")


def coordinate_descent(measure, space, start, passes=2):
    """Minimise measure(setting) one knob at a time (all values of a knob,
    the others held), `passes` sweeps over the knobs.  Returns (best setting,
    best value, {setting key: value} of every distinct setting measured)."""
    seen = {}

    def key(s):
        return json.dumps(s, sort_keys=True)

    def value(s):
        k = key(s)
        if k not in seen:
            seen[k] = measure(dict(s))
        return seen[k]

    best = dict(start)
    best_v = value(best)
    for _ in range(passes):
        changed = False
        for knob, values in space.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = dict(best)
                cand[knob] = v
                cv = value(cand)
                if cv < best_v:
                    best, best_v, changed = cand, cv, True
        if not changed:
            break
    return best, best_v, seen


def bucket_space(bucket_space=None, n_buckets=N_BUCKETS):
    """The per-bucket knobs as flat coordinates "knob@bucket" (value 0 = the
    plan-wide setting)."""
    bs = BUCKET_SPACE if bucket_space is None else bucket_space
    return {f"{k}@{b}": [0] + list(vals) for b in range(n_buckets) for k, vals in bs.items()}


def split_setting(flat):
    """A flat setting (plan-wide knobs and "knob@bucket" coordinates) as plan
    options: the per-bucket values go to ``buckets`` ({bucket: {knob: value}},
    zero entries dropped)."""
    out, buckets = {}, {}
    for k, v in flat.items():
        if "@" in k:
            knob, b = k.split("@")
            if v:
                buckets.setdefault(str(int(b)), {})[knob] = v
        else:
            out[k] = v
    if buckets:
        out["buckets"] = buckets
    return out


def plan_options(setting):
    """Planner keyword arguments of a recorded setting (everything but grid)."""
    return {k: v for k, v in setting.items() if k != "grid"}


def make_measure(pds, qs, precision=0, reps=5, threads=0, strategy=3):
    """measure(setting) -> ms per kn_batch_contract of the sample."""
    import torch

    from . import kn

    stream = torch.cuda.current_stream()

    def measure(setting):
        setting = split_setting(setting)
        _, plans = kn.plan_many(pds, qs, n_threads=threads, precision=precision,
                                strategy=strategy, **plan_options(setting))
        b = kn.Batch(plans)
        if setting.get("grid", 0):
            b.set_grid(int(setting["grid"]))
        b.upload(stream=stream)
        z = kn.alloc_scalars(len(plans))
        b.contract(stream=stream, z=z)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.contract(stream=stream, z=z)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    return measure


def flat_setting(setting):
    """A setting as ``load`` returns it (plan-wide knobs and ``buckets``) as a
    flat setting over every coordinate the search moves: knobs it lacks take
    the defaults, bucket coordinates it lacks 0 (the plan-wide value)."""
    flat = dict(DEFAULTS)
    flat.update({k: v for k, v in setting.items() if k != "buckets" and k in DEFAULTS})
    flat.update({k: 0 for k in bucket_space()})
    for b, knobs in (setting.get("buckets") or {}).items():
        for knob, v in knobs.items():
            flat[f"{knob}@{int(b)}"] = v
    return flat


def tune(pds, qs, precision=0, reps=5, space=None, grids=None, buckets=True, threads=0,
         confirm=5, strategy=3, start=None, log=print):
    """Coordinate descent from the defaults, or from ``start`` (a setting as
    ``load`` returns it, e.g. the one recorded before); the confirmation
    times the defaults, the start and the best alternately."""
    space = dict(SPACE if space is None else space)
    measure = make_measure(pds, qs, precision=precision, reps=reps, threads=threads,
                           strategy=strategy)

    def logged(s):
        v = measure(s)
        log(f"  {json.dumps(split_setting(s), sort_keys=True)}: {v:.4f} ms")
        return v

    first = dict(DEFAULTS) if start is None else flat_setting(start)
    best, best_v, seen = coordinate_descent(logged, space, first)
    if grids:
        best, best_v, more = coordinate_descent(logged, {"grid": list(grids)}, best, passes=1)
        seen.update(more)
    plan_wide = {k: v for k, v in best.items() if "@" not in k}
    if buckets:
        bspace = bucket_space()
        flat = dict({k: 0 for k in bspace}, **best)
        best, best_v, more = coordinate_descent(logged, bspace, flat, passes=1)
        seen.update(more)
    # defaults (and the start) against the best, timed alternately
    d_ms, b_ms, s_ms = [], [], []
    for _ in range(confirm):
        d_ms.append(measure(dict(DEFAULTS)))
        if start is not None:
            s_ms.append(measure(dict(first)))
        b_ms.append(measure(dict(best)))
    if DEFAULTS_KEY not in seen:
        seen[DEFAULTS_KEY] = statistics.median(d_ms)
    table = [dict(split_setting(json.loads(k)), ms=v)
             for k, v in sorted(seen.items(), key=lambda kv: kv[1])]
    return {"best": split_setting(best), "best_ms": best_v, "plan_wide": split_setting(plan_wide),
            "default_ms": seen[DEFAULTS_KEY],
            "confirm": dict({"default_ms": d_ms, "best_ms": b_ms,
                             "default_median_ms": statistics.median(d_ms),
                             "best_median_ms": statistics.median(b_ms),
                             "default_spread_ms": max(d_ms) - min(d_ms),
                             "best_spread_ms": max(b_ms) - min(b_ms)},
                            **({"start": split_setting(first), "start_ms": s_ms,
                                "start_median_ms": statistics.median(s_ms)} if s_ms else {})),
            "table": table}


def save(result, path, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(dict(meta, **result), f, indent=1)


def load(workload, precision=0):
    """The tuned setting of a workload ({} when none was recorded): planner
    keyword arguments (``buckets`` included) plus ``grid``."""
    path = os.path.join(TUNED_DIR, f"{workload}.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    rec = d.get("by_precision", {}).get(str(precision))
    return dict(rec["best"]) if rec else {}


def main():
    ap = argparse.ArgumentParser(description="tune the batch contraction knobs on a workload")
    ap.add_argument("--workload", default="q3_200_600")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--precisions", default="0,1")
    ap.add_argument("--no-buckets", action="store_true")
    ap.add_argument("--strategy", type=int, default=3,
                    help="contraction-order strategy the plans are made with (kn_plan_opts)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--from-tuned", action="store_true",
                    help="start the search from the setting recorded for the workload")
    args = ap.parse_args()

    import numpy as np
    import torch

    from . import gen, kn

    if not torch.cuda.is_available():
        print("tune.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    kn.lib()
    knots = gen.config_knots(args.workload, args.seed, count=args.count)
    qs = [q for _, q in knots]
    pds = [np.ascontiguousarray(d.pd, dtype=np.int32) for d, _ in knots]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"workload": args.workload, "seed": args.seed, "count": args.count,
           "q": sorted(set(qs)), "strategy": args.strategy,
           "device": torch.cuda.get_device_name(0),
           "when": time.strftime("%Y-%m-%d"), "by_precision": {}}
    for precision in (int(p) for p in args.precisions.split(",")):
        print(f"precision {precision}", flush=True)
        start = load(args.workload, precision) if args.from_tuned else None
        res = tune(pds, qs, precision=precision, reps=args.reps,
                   grids=[0, cus, 2 * cus, 4 * cus], buckets=not args.no_buckets,
                   strategy=args.strategy, start=start or None,
                   log=lambda m: print(m, flush=True))
        c = res["confirm"]
        print(f"best {res['best']} {res['best_ms']:.4f} ms (defaults {res['default_ms']:.4f} ms); "
              f"confirmed medians {c['best_median_ms']:.4f} vs {c['default_median_ms']:.4f} ms"
              + (f", start {c['start_median_ms']:.4f} ms" if "start_median_ms" in c else ""),
              flush=True)
        out["by_precision"][str(precision)] = res
    path = args.out or os.path.join(TUNED_DIR, f"{args.workload}.json")
    save({}, path, out)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
