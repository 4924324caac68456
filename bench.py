#!/usr/bin/env python3
"""Throughput of exact Jones-polynomial evaluation V_K(t(3)) on one MI355X.

Workload: seeded lattice-walk knot diagrams with 200-600 raw crossings
(``paper_1807_02119_amd.gen``, workload ``q3_200_600``), q = 3
(t = e^{i pi/3}), complex128.  One step = the whole pipeline for one batch of
knots: signed Tait graphs and plans on the host thread pool (kn_plan_many),
the batch device program (kn_batch_create + upload), the persistent GPU
contraction of every tensor network (kn_batch_contract) and the
normalisation V = A(q) Z (kn_jones_many).  The PD codes (the input) are
generated before timing.

Printed: one JSON line.  ``value`` is knots/s of the whole step; the line
also carries the GPU contraction alone (events around the persistent
kernel), the complex64 path with its error against complex128, the
one-knot-per-call path, the roofline of the contraction kernel and the CPU
oracle timed on a bounded sample of the same knots.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "knots/s + achieved TFLOP/s for exact Z, q=3, 200–600 crossings; FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256, help="knots per step")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0, help="host planning threads (0 = all)")
    ap.add_argument("--strategy", type=int, default=2, choices=(0, 1, 2, 3),
                    help="contraction-order strategy of the planner (kn_plan_opts.strategy); "
                         "default min-fill only: the pipeline is bound by host planning, and "
                         "the greedy alternative that auto also builds for the heaviest knots "
                         "costs more host time than it saves on the device")
    ap.add_argument("--prefetch", type=int, default=2, choices=(1, 2, 3),
                    help="batches the helper thread prepares ahead of the launch thread")
    ap.add_argument("--kernel-reps", type=int, default=20,
                    help="launches of the contraction kernel timed for the roofline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget for the CPU oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the one-knot-per-call comparison")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the mixed batch (512 knots of 20-250 crossings, q in 2,3,5,6) "
                         "launched through a captured graph")
    ap.add_argument("--untuned", action="store_true",
                    help="ignore the autotuner's recorded setting (library defaults)")
    ap.add_argument("--pmc-calibrate", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (a plain copy of known "
                         "size, to scale the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


# the sources the contraction kernel is compiled from
KERNEL_SOURCES = ("engine.hip", "program.h", "decode.h")


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1807_02119_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "engine_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    rec = d.get(kernel)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the contraction runs on one GPU only (asked for --gpus {args.gpus}); "
              "knots are independent and would shard across GPUs with no communication, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1807_02119_amd import gen, kn, tune

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.pmc_calibrate:
        n = args.pmc_calibrate // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": 4 * n, "launches": 3}), flush=True)
        return
    kn.lib()
    q = 3
    B = args.batch
    knots = gen.config_knots("q3_200_600", args.seed, count=B)
    pds = [np.ascontiguousarray(d.pd, dtype=np.int32) for d, _ in knots]
    ncross = [d.n for d, _ in knots]
    # the batch's input as the library takes it: crossing counts and the PD
    # codes concatenated
    ncr_arr = np.asarray(ncross, np.int32)
    flat_pd = np.concatenate([p.reshape(-1) for p in pds])
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------------- pipeline
    # Two threads.  A helper prepares batches i+1 .. i+prefetch back to back
    # (Tait graphs and plans on the library's thread pool, the batch device
    # program, its upload on a side stream into one of prefetch + 1 workspaces
    # in turn) while
    # the launch thread contracts batch i and, while the GPU runs it, forms
    # V = A Z of batch i - 1 and releases that batch.  The library calls
    # release the GIL.
    state = {}
    # the threads hand the interpreter lock to each other often: switch fast
    sys.setswitchinterval(1e-4)
    pool = ThreadPoolExecutor(max_workers=1)
    up_stream = torch.cuda.Stream()

    # knob settings recorded by the autotuner for this workload (plan options
    # and the persistent grid), per precision; defaults when none was recorded
    tuned = {p: tune.load("q3_200_600", p) for p in (0, 1)} if not args.untuned else {0: {}, 1: {}}

    # wall time of each part of the pipeline, summed over the timed steps
    phase = {k: 0.0 for k in ("prepare", "plan", "batch", "upload", "handoff", "device", "launch",
                              "submit", "finish", "wait", "jones", "release", "gpu")}
    counter = [0]

    def workspace(slot, need, precision):
        ws = state.get(("ws", precision, slot))
        if ws is None or ws.numel() < need + 256:
            ws = kn.alloc_workspace(need)
            state[("ws", precision, slot)] = ws
        return ws

    def prepare(precision=0):
        tp = time.perf_counter()
        opts = {k: v for k, v in tuned[precision].items() if k != "grid"}
        opts["strategy"] = args.strategy
        plans = kn.plan_set(ncr_arr, flat_pd, q, n_threads=args.threads, precision=precision,
                            **opts)
        taits = plans  # the set holds the Tait graphs too
        t1 = time.perf_counter()
        batch = kn.Batch(plans)
        if tuned[precision].get("grid"):
            batch.set_grid(int(tuned[precision]["grid"]))
        t2 = time.perf_counter()
        # prefetch + 1 workspaces in turn: the upload into this one waits (on
        # the GPU, not here) for the contraction that used it last, prefetch + 1
        # batches ago; that contraction's launch came before this preparation
        # was queued
        slot = counter[0] % (args.prefetch + 1)
        counter[0] += 1
        ws = workspace(slot, batch.workspace_bytes, precision)
        last = state.get(("done", precision, slot))
        if last is not None:
            up_stream.wait_event(last)
        batch.upload(ws, up_stream)
        uploaded = torch.cuda.Event()
        uploaded.record(up_stream)
        t3 = time.perf_counter()
        phase["plan"] += t1 - tp
        phase["batch"] += t2 - t1
        phase["upload"] += t3 - t2
        phase["prepare"] += t3 - tp
        return taits, plans, batch, uploaded, slot

    def launch(prepared, precision=0):
        """Queue batch i's contraction behind its upload."""
        taits, plans, batch, uploaded, slot = prepared
        z = state.get(("z", precision))
        if z is None:
            z = kn.alloc_scalars(B)
            state[("z", precision)] = z
        t1 = time.perf_counter()
        stream.wait_event(uploaded)
        start = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        batch.contract(stream=stream, z=z)
        done = torch.cuda.Event(enable_timing=True)
        done.record(stream)
        state["start"] = start
        state[("done", precision, slot)] = done
        phase["launch"] += time.perf_counter() - t1
        return done, z

    def release(box):
        box.pop()

    def finish(prepared, done, z, hand=None):
        """While the GPU runs batch i: form V = A Z of batch i - 1 (handed over
        in the list `hand`, which holds the only reference) and release that
        batch; then wait for batch i's Z."""
        taits, plans, batch = prepared[:3]
        previous = hand.pop() if hand else None
        t2 = time.perf_counter()
        if previous is not None:
            kn.jones_many(q, previous[0], previous[3])
        t21 = time.perf_counter()
        # batch i - 1 (plans, Tait graphs, device program) is released by the
        # helper thread between two preparations: freed while the planning
        # threads allocate, its many small blocks would contend for the
        # allocator's locks (several ms instead of a fraction of one)
        if previous is not None:
            pool.submit(release, [previous])
        del previous
        t3 = time.perf_counter()
        phase["release"] += t3 - t21
        # wait without spinning: the planning threads need every core
        while not done.query():
            time.sleep(50e-6)
        zh = z.cpu().numpy()
        t4 = time.perf_counter()
        # the contraction's own time inside the pipeline (device clock)
        phase["gpu"] += state["start"].elapsed_time(done) / 1e3
        phase["jones"] += t21 - t2
        phase["wait"] += t4 - t3
        return taits, plans, batch, zh

    def run_steps(n, precision=0):
        """n whole batches, host preparation (and upload) of batch i+1
        overlapped with the device work of batch i; returns the last batch's
        results (every batch's V is formed before this returns)."""
        # the helper runs up to two preparations ahead, back to back (one
        # worker), so it never waits for the launch thread
        futs = [pool.submit(prepare, precision) for _ in range(min(args.prefetch, n))]
        cur = None
        for i in range(n):
            t0 = time.perf_counter()
            prepared = futs.pop(0).result()
            t1 = time.perf_counter()
            done, z = launch(prepared, precision)
            ts = time.perf_counter()
            if i + args.prefetch < n:
                futs.append(pool.submit(prepare, precision))
            hand = [cur] if cur is not None else None
            cur = None
            tf = time.perf_counter()
            cur = finish(prepared, done, z, hand)
            del prepared
            te = time.perf_counter()
            phase["handoff"] += t1 - t0
            phase["submit"] += tf - ts
            phase["finish"] += te - tf
            phase["device"] += te - t1
        taits, plans, batch, zh = cur
        v, l2, ar = kn.jones_many(q, taits, zh)
        return taits, plans, batch, zh, v, l2, ar

    run_steps(max(1, args.warmup))
    torch.cuda.synchronize()
    for k in phase:
        phase[k] = 0.0
    t0 = time.perf_counter()
    taits, plans, batch, zh, v, l2, ar = run_steps(args.steps)
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    pipeline_ms = {k: round(1e3 * t / args.steps, 3) for k, t in phase.items()}
    value = B / (ms_step / 1e3)

    # ---------------------------------------------------------------- GPU contraction alone
    def time_kernel(batch, reps):
        z = kn.alloc_scalars(B)
        batch.contract(stream=stream, z=z)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            batch.contract(stream=stream, z=z)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, z

    ms_gpu, z64 = time_kernel(batch, args.kernel_reps)
    st = batch.stats
    flops, bytes_alg = st["flops"], st["bytes"]
    zh64 = z64.cpu().numpy()
    # (re, im, exp2) records: compare bit patterns (an int64 exponent read as a
    # double can be a NaN, which never compares equal)
    assert np.array_equal(zh64.view(np.int64), zh.view(np.int64)), \
        "repeated launches must give identical bits"

    # host-only breakdown of one step: plans, then plans + device program
    t0 = time.perf_counter()
    kn.plan_set(ncr_arr, flat_pd, q, n_threads=args.threads, strategy=args.strategy,
                **{k: v for k, v in tuned[0].items() if k != "grid"})
    ms_plan = 1e3 * (time.perf_counter() - t0)
    t0 = time.perf_counter()
    prepare()
    ms_prepare = 1e3 * (time.perf_counter() - t0)

    roofline_gbs = bytes_alg / (ms_gpu * 1e-3) / 1e9
    rec = measured_traffic("engine<double>")
    traffic = None
    if rec is not None:
        traffic = rec["fetch_bytes"] + rec["write_bytes"]
    roofline = {
        "kernel": "kn::engine<double> (persistent contraction, batch launch)",
        "bound": "hbm",
        "achieved": round(roofline_gbs, 3),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": roofline_gbs / HBM_PEAK_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": bytes_alg,
        "flops_per_launch": flops,
        "avg_launch_ms": ms_gpu,
        "achieved_tflops": flops / (ms_gpu * 1e-3) / 1e12,
        "fp64_peak_tflops": FP64_PEAK_TFLOPS,
    }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "knots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "q3_200_600: seeded lattice-walk knots, 200-600 raw crossings, q=3, "
                        "complex128, whole pipeline (Tait graph, plan, device program, "
                        "persistent GPU contraction, V = A Z) per batch",
            "q": q,
            "knots_per_step": B,
            "crossings_min": int(min(ncross)),
            "crossings_max": int(max(ncross)),
            "crossings_mean": float(np.mean(ncross)),
            "seed": args.seed,
        },
        "achieved_tflops": flops / (ms_step * 1e-3) / 1e12,
        "host_plan_ms": ms_plan,
        "host_prepare_ms": ms_prepare,
        "host_threads": args.threads if args.threads > 0 else len(os.sched_getaffinity(0)),
        "pipelined": f"host preparation of batches i+1..i+{args.prefetch} overlaps the GPU work "
                     "of batch i",
        "pipeline_ms": pipeline_ms,
        "tuned": tuned[0] or None,
        "gpu_contract": {
            "ms_per_batch": ms_gpu,
            "knots_per_s": B / (ms_gpu * 1e-3),
            "tflops": flops / (ms_gpu * 1e-3) / 1e12,
            "n_tasks": st["n_tasks"],
        },
        "roofline": roofline,
    }

    # ---------------------------------------------------------------- FP32 path
    def rel_errs(za, zb):
        ea = za.view(np.int64)[:, 2]
        eb = zb.view(np.int64)[:, 2]
        ma = za[:, 0] + 1j * za[:, 1]
        mb = zb[:, 0] + 1j * zb[:, 1]
        return np.abs(ma * np.exp2((ea - eb).astype(np.float64)) - mb) / np.abs(mb)

    if not args.no_fp32:
        run_steps(1, precision=1)
        n32 = max(1, args.steps // 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        taits32, plans32, batch32, zh32, v32, _, _ = run_steps(n32, precision=1)
        torch.cuda.synchronize()
        t32 = (time.perf_counter() - t0) / n32
        ms32, _ = time_kernel(batch32, args.kernel_reps)
        err = rel_errs(zh32, zh)
        out["fp32"] = {
            "dtype": "f32",
            "knots_per_s": B / t32,
            "gpu_contract_ms": ms32,
            "gpu_knots_per_s": B / (ms32 * 1e-3),
            "gpu_speedup_vs_fp64": ms_gpu / ms32,
            "tflops": batch32.stats["flops"] / (ms32 * 1e-3) / 1e12,
            "rel_err_vs_fp64_max": float(err.max()),
            "rel_err_vs_fp64_median": float(np.median(err)),
        }

    # ---------------------------------------------------------------- one knot per call
    if not args.no_single:
        single = [plans.plan(i) for i in range(len(plans))]
        ws = kn.alloc_workspace(max(p.workspace_bytes for p in single))
        z1 = kn.alloc_scalars(1)
        for p in single[:4]:
            kn.contract(p, workspace=ws, stream=stream, z=z1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in single:
            kn.contract(p, workspace=ws, stream=stream, z=z1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["one_at_a_time"] = {
            "knots_per_s": B / dt,
            "ms_per_knot": 1e3 * dt / B,
            "batched_gpu_speedup": (dt * 1e3) / ms_gpu,
        }

    # ---------------------------------------------------------------- mixed batch, graph launch
    # 512 knots of 20-250 crossings with q drawn from {2, 3, 5, 6}, complex128,
    # contracted in one persistent launch replayed from a captured hipGraph,
    # against eager launches of the same batch and one knot per call
    if not args.no_batched:
        mixed = gen.config_knots("batched", args.seed, count=512)
        mtaits, mplans = kn.plan_many([np.ascontiguousarray(d.pd, dtype=np.int32)
                                       for d, _ in mixed], [mq for _, mq in mixed])
        mb = kn.Batch(mplans)
        mb.upload(stream=stream)
        zm = kn.alloc_scalars(len(mplans))
        mb.contract(stream=stream, z=zm)
        torch.cuda.synchronize()
        zref = zm.cpu().numpy().copy()
        g = mb.graph(zm)
        reps = 20

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_graph = timed(g.replay)
        replay_ok = bool(np.array_equal(zm.cpu().numpy().view(np.int64), zref.view(np.int64)))
        ms_eager = timed(lambda: mb.contract(stream=stream, z=zm))
        sample = mplans[:64]
        wsm = kn.alloc_workspace(max(p.workspace_bytes for p in sample))
        z1m = kn.alloc_scalars(1)
        for p in sample[:4]:
            kn.contract(p, workspace=wsm, stream=stream, z=z1m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in sample:
            kn.contract(p, workspace=wsm, stream=stream, z=z1m)
        torch.cuda.synchronize()
        single_kps = len(sample) / (time.perf_counter() - t0)
        out["batched_mixed"] = {
            "workload": "512 seeded lattice-walk knots, 20-250 crossings, q in {2,3,5,6}, "
                        "complex128, one persistent launch",
            "graph_ms_per_launch": ms_graph,
            "graph_knots_per_s": len(mplans) / (ms_graph * 1e-3),
            "eager_ms_per_launch": ms_eager,
            "one_at_a_time_knots_per_s": single_kps,
            "one_at_a_time_sample": len(sample),
            "speedup_vs_one_at_a_time": len(mplans) / (ms_graph * 1e-3) / single_kps,
            "graph_replays_equal_eager_bits": replay_ok,
            "tflops": mb.stats["flops"] / (ms_graph * 1e-3) / 1e12,
        }

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu_baseline:
        from oracle import diagram, jones, potts

        t_cpu = 0.0
        n_done = 0
        worst = 0.0
        for i, (d, _) in enumerate(knots):
            t0 = time.perf_counter()
            tg = diagram.tait_graph(d.pd)
            x = potts.jones_weights(tg.eps, jones.t_of_q(q))
            mo, eo = potts.partition_function(tg.n_vertices, tg.edges, x, q)
            jones.jones_value(q, tg.n_vertices, tg.writhe, tg.tait_number, mo, eo)
            t_cpu += time.perf_counter() - t0
            n_done += 1
            m = complex(zh[i, 0], zh[i, 1])
            e = int(zh.view(np.int64)[i, 2])
            worst = max(worst, abs(m * 2.0 ** (e - eo) - mo) / abs(mo))
            if t_cpu >= args.cpu_seconds:
                break
        out["cpu_baseline"] = {
            "value": n_done / t_cpu,
            "unit": "knots/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"first {n_done} of the {B} knots of the step (same seed), numpy "
                      f"complex128 min-fill variable elimination, single thread, "
                      f"{t_cpu:.1f} s",
            "gpu_vs_oracle_max_rel_err": worst,
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
