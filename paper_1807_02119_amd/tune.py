"""Autotuner for batched contraction.

How a step runs is decided by a few planner knobs:
- big_step_macs_log2: the multiply-add count above which a step is split
  into tiles over workgroups instead of running inside a serial task;
- tile_macs_log2: how much work one tile of outputs carries;
- lds_bytes: the per-workgroup LDS arena for tensors that stay inside one
  serial task, which also sets how many workgroups fit on a compute unit;
- gemm_tasks_log2: how many tasks a step computed in output blocks is cut
  into (several blocks per task above that);
- gemm64_pct: how much padding a step accepts to use 64 x 64 output blocks
  instead of 32 x 32 ones.
The persistent kernel's grid is the last knob.  The tuner times
kn_batch_contract with HIP events (on the launch stream) on a sample of a
workload, searches the knobs by coordinate descent from the defaults, and
writes the best setting with the full table of measurements to a JSON file.
bench.py and users load it with ``load``.

    python -m paper_1807_02119_amd.tune --workload q3_200_600 --count 256 \\
        --out paper_1807_02119_amd/tuned/q3_200_600.json
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

SPACE = {
    "big_step_macs_log2": [14, 15, 16, 17, 18],
    "tile_macs_log2": [13, 14, 15, 16, 17],
    "lds_bytes": [16384, 24576, 32768, 49152],
    "gemm_tasks_log2": [4, 5, 6, 7, 30],
    "gemm64_pct": [1, 150, 300],
}
DEFAULTS = {"big_step_macs_log2": 16, "tile_macs_log2": 15, "lds_bytes": 24576,
            "gemm_tasks_log2": 5, "gemm64_pct": 300, "grid": 0}
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


def make_measure(pds, q, precision=0, reps=5, threads=0):
    """measure(setting) -> ms per kn_batch_contract of the sample."""
    import torch

    from . import kn

    stream = torch.cuda.current_stream()

    def measure(setting):
        opts = {k: v for k, v in setting.items() if k != "grid"}
        _, plans = kn.plan_many(pds, q, n_threads=threads, precision=precision, **opts)
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


def tune(pds, q, precision=0, reps=5, space=None, grids=None, threads=0, log=print):
    space = dict(SPACE if space is None else space)
    measure = make_measure(pds, q, precision=precision, reps=reps, threads=threads)

    def logged(s):
        v = measure(s)
        log(f"  {json.dumps(s, sort_keys=True)}: {v:.4f} ms")
        return v

    best, best_v, seen = coordinate_descent(logged, space, DEFAULTS)
    if grids:
        best, best_v, more = coordinate_descent(logged, {"grid": list(grids)}, best, passes=1)
        seen.update(more)
    table = [dict(json.loads(k), ms=v) for k, v in sorted(seen.items(), key=lambda kv: kv[1])]
    return {"best": best, "best_ms": best_v, "default_ms": seen[json.dumps(DEFAULTS, sort_keys=True)],
            "table": table}


def save(result, path, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(dict(meta, **result), f, indent=1)


def load(workload, precision=0):
    """The tuned setting of a workload ({} when none was recorded)."""
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
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    import numpy as np
    import torch

    from . import gen, kn

    if not torch.cuda.is_available():
        print("tune.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    kn.lib()
    knots = gen.config_knots(args.workload, args.seed, count=args.count)
    qs = sorted({q for _, q in knots})
    if len(qs) != 1:
        print("tune.py tunes single-q workloads", file=sys.stderr)
        sys.exit(2)
    pds = [np.ascontiguousarray(d.pd, dtype=np.int32) for d, _ in knots]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"workload": args.workload, "seed": args.seed, "count": args.count,
           "device": torch.cuda.get_device_name(0), "when": time.strftime("%Y-%m-%d"),
           "by_precision": {}}
    for precision in (0, 1):
        print(f"precision {precision}", flush=True)
        res = tune(pds, qs[0], precision=precision, reps=args.reps,
                   grids=[0, cus, 2 * cus, 4 * cus], log=lambda m: print(m, flush=True))
        print(f"best {res['best']} {res['best_ms']:.4f} ms (defaults {res['default_ms']:.4f} ms)",
              flush=True)
        out["by_precision"][str(precision)] = res
    path = args.out or os.path.join(TUNED_DIR, f"{args.workload}.json")
    save({}, path, out)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
