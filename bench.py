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
import queue
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "knots/s + achieved TFLOP/s for exact Z, q=3, 200–600 crossings; FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256, help="knots per step")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0, help="host planning threads (0 = all)")
    ap.add_argument("--strategy", type=int, default=2, choices=(0, 1, 2, 3, 4),
                    help="contraction-order strategy of the planner (kn_plan_opts.strategy); "
                         "default min-fill only: the pipeline is bound by host planning, and "
                         "the greedy alternative that auto also builds for the heaviest knots "
                         "costs more host time than it saves on the device")
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
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision workload (16 knots of 300-600 crossings)")
    ap.add_argument("--no-fp64-single", action="store_true",
                    help="skip the 50-200 crossing workload at q=3 and 5, one knot per launch")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the gradient workload (32 knots of 150-300 crossings)")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the unsliced 351-crossing grid-walk knot (GEMM-heavy)")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the 351-crossing knot leg (for counter profiles) and print "
                         "its record")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-cores CPU oracle leg (0 = the host's CPUs, "
                         "at most 16)")
    ap.add_argument("--untuned", action="store_true",
                    help="ignore the autotuner's recorded setting (library defaults)")
    ap.add_argument("--pmc-calibrate", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers (a plain copy of known "
                         "size, to scale the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


# the sources the contraction kernel is compiled from
KERNEL_SOURCES = ("engine.hip", "program.h", "decode.h", "checks.h")


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


def oracle_knot(pd, q):
    """(seconds, Z mantissa, Z exponent) of one knot by the CPU oracle."""
    import numpy as np

    from oracle import diagram, jones, potts

    t0 = time.perf_counter()
    tg = diagram.tait_graph(np.asarray(pd))
    x = potts.jones_weights(tg.eps, jones.t_of_q(q))
    mo, eo = potts.partition_function(tg.n_vertices, tg.edges, x, q)
    jones.jones_value(q, tg.n_vertices, tg.writhe, tg.tait_number, mo, eo)
    return time.perf_counter() - t0, mo, eo


def _one_blas_thread():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"


def _oracle_job(job):
    return oracle_knot(*job)[0]


def cpu_parallel(knots, q, workers, seconds):
    """The oracle on `workers` fresh processes (spawned: they never touch the
    GPU), knots handed out in order, until `seconds` of wall time have
    passed; returns the knots finished and the wall time."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_one_blas_thread) as pool:
        pool.map(_oracle_job, [(knots[0][0].pd, q)] * workers)  # start-up outside the timing
        t0 = time.perf_counter()
        done = 0
        for _ in pool.imap(_oracle_job, [(d.pd, q) for d, _ in knots], chunksize=1):
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
        wall = time.perf_counter() - t0
        pool.terminate()
    return {"knots": done, "wall_s": wall, "knots_per_s": done / wall}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
            else:
                name = "unknown"
    except OSError:
        name = "unknown"
    return {"model": name, "usable_cpus": len(os.sched_getaffinity(0)),
            "os_cpu_count": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the contraction runs on one GPU only (asked for --gpus {args.gpus}); "
              "knots are independent and would shard across GPUs with no communication, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_1807_02119_amd import gen

    q = 3
    B = args.batch
    knots = gen.config_knots("q3_200_600", args.seed, count=B)
    # the all-cores CPU oracle leg runs first, before this process touches the
    # GPU (its worker processes are spawned fresh and never use the GPU)
    cpu_par = None
    if not args.no_cpu_baseline and not args.pmc_calibrate and not args.wide_only:
        workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        cpu_par = dict(cpu_parallel(knots, q, workers, args.cpu_seconds), workers=workers)

    import torch

    from paper_1807_02119_amd import kn, tune

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

    def wide_knot_leg(reps=5):
        """The paper-model grid walk of Sec. III.A with L = 60 (351 crossings,
        seed 60), q = 3, unsliced: its largest tensor has 2^25.4 entries and its
        big steps run as GEMM blocks on the matrix cores."""
        rng = np.random.default_rng(60)
        d = gen.random_grid_diagram(rng, 60)
        t = kn.Tait(d.pd)
        leg = {"workload": f"paper-model grid-walk knot L=60 ({d.n} crossings, seed 60), q=3, "
                           "unsliced, one knot per launch"}
        st_ = torch.cuda.current_stream()
        for prec, name in ((0, "c128"), (1, "c64")):
            p_ = kn.Plan(t, 3, precision=prec)
            ws_ = kn.alloc_workspace(p_.workspace_bytes)
            z_ = kn.alloc_scalars(1)
            kn.contract(p_, workspace=ws_, stream=st_, z=z_)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st_)
            for _ in range(reps):
                kn.contract(p_, workspace=ws_, stream=st_, z=z_)
            e1.record(st_)
            torch.cuda.synchronize()
            ms_ = e0.elapsed_time(e1) / reps
            leg[name] = {"ms": ms_, "gflop": p_.stats["flops"] / 1e9,
                         "tflops": p_.stats["flops"] / (ms_ * 1e-3) / 1e12,
                         "log2_max_entries": p_.stats["log2_max_entries"]}
            leg[name]["frac_of_peak"] = leg[name]["tflops"] / (FP64_PEAK_TFLOPS if prec == 0
                                                                 else FP32_PEAK_TFLOPS)
        # grid-walk knots of 521-574 crossings at q = 3, too wide for one
        # tensor of at most 2^31 entries: sliced (largest tensor <= 2^26
        # entries), auto order, slices as device-side loops over chains
        leg["sliced_q3_500_600"] = []
        for seed_, size_ in ((74, 80), (72, 75), (71, 72), (70, 70)):
            d_ = gen.random_grid_diagram(np.random.default_rng(seed_), size_)
            t0_ = time.perf_counter()
            p_ = kn.Plan(kn.Tait(d_.pd), 3, slice_log2_budget=26)
            plan_s = time.perf_counter() - t0_
            ws_ = kn.alloc_workspace(p_.workspace_bytes)
            z_ = kn.alloc_scalars(1)
            kn.contract(p_, workspace=ws_, stream=st_, z=z_)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st_)
            for _ in range(2):
                kn.contract(p_, workspace=ws_, stream=st_, z=z_)
            e1.record(st_)
            torch.cuda.synchronize()
            ms_ = e0.elapsed_time(e1) / 2
            leg["sliced_q3_500_600"].append({
                "crossings": d_.n, "seed": seed_, "walk": size_, "slices": p_.stats["n_slices"],
                "chains": p_.stats["slice_chains"], "gflop": p_.stats["flops"] / 1e9,
                "plan_s": plan_s, "ms": ms_, "tflops": p_.stats["flops"] / (ms_ * 1e-3) / 1e12,
                "log2_max_entries": p_.stats["log2_max_entries"]})
            del ws_
        return leg

    if args.wide_only:
        print(json.dumps({"wide_knot": wide_knot_leg()}), flush=True)
        return
    pds = [np.ascontiguousarray(d.pd, dtype=np.int32) for d, _ in knots]
    ncross = [d.n for d, _ in knots]
    # the batch's input as the library takes it: crossing counts and the PD
    # codes concatenated
    ncr_arr = np.asarray(ncross, np.int32)
    flat_pd = np.concatenate([p.reshape(-1) for p in pds])
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------------- pipeline
    # Three threads joined by bounded queues.  The planner thread makes the
    # Tait graphs and plans of one batch after another on the library's thread
    # pool; between two plan sets it frees the batches the launch thread is
    # done with (freed while the planning threads allocate, their many blocks
    # would contend for the allocator's locks).  The builder thread makes each
    # batch's device program and uploads it on a side stream into one of
    # N_SLOTS workspaces in turn.  The launch thread queues batch i + 1's
    # contraction behind batch i's on the stream, forms V = A Z of batch i - 1
    # while the GPU works, then waits for batch i.  The library calls release
    # the GIL.
    #
    # Workspace slots: the builder starts batch j only once batch j - 1 is in
    # the (one-deep) built queue, so batch j - 2 has been taken and batch
    # j - 3, the last user of slot j % 3, launched: the upload waits (on the
    # GPU) for that launch's contraction.  Batch j's Z buffer (one per slot)
    # is written by a launch that comes after batch j - 3's Z was read.
    N_SLOTS = 3
    state = {}
    # the threads hand the interpreter lock to each other often: switch fast
    sys.setswitchinterval(1e-4)
    up_stream = torch.cuda.Stream()

    # knob settings recorded by the autotuner for this workload (plan options
    # and the persistent grid), per precision; defaults when none was recorded
    tuned = {p: tune.load("q3_200_600", p) for p in (0, 1)} if not args.untuned else {0: {}, 1: {}}

    # wall time of each part of the pipeline, summed over the timed steps
    phase = {k: 0.0 for k in ("plan", "plan_blocked", "free", "prepare", "batch", "upload",
                              "handoff", "launch", "finish", "wait", "jones", "gpu", "gpu_start")}

    def workspace(slot, need, precision):
        ws = state.get(("ws", precision, slot))
        if ws is None or ws.numel() < need + 256:
            ws = kn.alloc_workspace(need)
            state[("ws", precision, slot)] = ws
        return ws

    def plan_stage(precision=0):
        opts = {k: v for k, v in tuned[precision].items() if k != "grid"}
        opts["strategy"] = args.strategy
        return kn.plan_set(ncr_arr, flat_pd, q, n_threads=args.threads, precision=precision,
                           **opts)

    def build_stage(plans, slot, precision=0):
        """A plan set's batch device program, uploaded into workspace `slot`
        behind the contraction that used that workspace last."""
        t1 = time.perf_counter()
        batch = kn.Batch(plans)
        if tuned[precision].get("grid"):
            batch.set_grid(int(tuned[precision]["grid"]))
        t2 = time.perf_counter()
        ws = workspace(slot, batch.workspace_bytes, precision)
        last = state.get(("done", precision, slot))
        if last is not None:
            up_stream.wait_event(last)
        batch.upload(ws, up_stream)
        uploaded = torch.cuda.Event()
        uploaded.record(up_stream)
        t3 = time.perf_counter()
        phase["batch"] += t2 - t1
        phase["upload"] += t3 - t2
        phase["prepare"] += t3 - t1
        return plans, plans, batch, uploaded, slot  # the set holds the Tait graphs too

    def prepare(precision=0):
        """One batch planned, built and uploaded on the calling thread (into a
        workspace of its own)."""
        return build_stage(plan_stage(precision), "host", precision)

    def launch(prepared, precision=0):
        """Queue batch i's contraction behind its upload (and behind what the
        stream already holds: batch i - 1's contraction)."""
        taits, plans, batch, uploaded, slot = prepared
        z = state.get(("z", precision, slot))
        if z is None:
            z = kn.alloc_scalars(B)
            state[("z", precision, slot)] = z
        t1 = time.perf_counter()
        pre = torch.cuda.Event(enable_timing=True)
        pre.record(stream)
        stream.wait_event(uploaded)
        start = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        batch.contract(stream=stream, z=z)
        done = torch.cuda.Event(enable_timing=True)
        done.record(stream)
        state[("done", precision, slot)] = done
        phase["launch"] += time.perf_counter() - t1
        return dict(z=z, pre=pre, start=start, done=done)

    def finish(prepared, launched, to_free, hand=None):
        """While the device runs batch i (and has batch i + 1 queued): form
        V = A Z of batch i - 1 (handed over in the list `hand`, which holds
        the only reference) and pass that batch on to be freed; then wait for
        batch i's Z."""
        taits, plans, batch = prepared[:3]
        done, z = launched["done"], launched["z"]
        previous = hand.pop() if hand else None
        t2 = time.perf_counter()
        if previous is not None:
            kn.jones_many(q, previous[0], previous[3])
            to_free.put([previous])
        del previous
        t3 = time.perf_counter()
        # wait without spinning: the planning threads need every core
        while not done.query():
            time.sleep(50e-6)
        zh = z.cpu().numpy()
        t4 = time.perf_counter()
        # the contraction's own time inside the pipeline (device clock), and
        # how long it waited on the device for its upload once the stream
        # reached it
        phase["gpu"] += launched["start"].elapsed_time(done) / 1e3
        phase["gpu_start"] += launched["pre"].elapsed_time(launched["start"]) / 1e3
        phase["jones"] += t3 - t2
        phase["wait"] += t4 - t3
        return taits, plans, batch, zh

    def prime(precision=0):
        """Set-up before the warmup: every workspace slot and Z buffer
        allocated, and the library's pool of page-locked image buffers filled
        with as many buffers as batches can be alive at once in run_steps (one
        in each queue, one being built, two launched, two waiting to be
        freed), so that the timed steps allocate nothing on the device or in
        page-locked memory."""
        plans = plan_stage(precision)
        held = [kn.Batch(plans) for _ in range(N_SLOTS + 4)]
        for slot in range(N_SLOTS):
            workspace(slot, held[0].workspace_bytes, precision)
            if state.get(("z", precision, slot)) is None:
                state[("z", precision, slot)] = kn.alloc_scalars(B)
        del held, plans

    def run_steps(n, precision=0):
        """n whole batches through the three threads; returns the last batch's
        results (every batch's V is formed before this returns)."""
        plan_q = queue.Queue(maxsize=1)   # planned, not yet being built
        built_q = queue.Queue(maxsize=1)  # built and uploaded, not yet launched
        free_q = queue.SimpleQueue()      # done with: freed by the planner thread
        stop = threading.Event()

        def put(dst, item):
            """Blocking put that gives up once the run has stopped."""
            while not stop.is_set():
                try:
                    dst.put(item, timeout=0.05)
                    return True
                except queue.Full:
                    pass
            return False

        def get(src):
            while True:
                try:
                    item = src.get(timeout=0.05)
                except queue.Empty:
                    if stop.is_set():
                        raise RuntimeError("pipeline stopped")
                    continue
                if isinstance(item, BaseException):
                    raise item
                return item

        def drain_free():
            while True:
                try:
                    free_q.get_nowait().clear()
                except queue.Empty:
                    return

        def planner():
            try:
                for _ in range(n):
                    t0 = time.perf_counter()
                    drain_free()
                    t1 = time.perf_counter()
                    plans = plan_stage(precision)
                    t2 = time.perf_counter()
                    ok = put(plan_q, plans)
                    del plans
                    phase["free"] += t1 - t0
                    phase["plan"] += t2 - t1
                    phase["plan_blocked"] += time.perf_counter() - t2
                    if not ok:
                        return
            except BaseException as e:  # handed to the launch thread
                put(plan_q, e)

        def builder():
            try:
                for j in range(n):
                    prepared = build_stage(get(plan_q), j % N_SLOTS, precision)
                    ok = put(built_q, prepared)
                    del prepared
                    if not ok:
                        return
            except BaseException as e:
                put(built_q, e)

        helpers = [threading.Thread(target=planner, daemon=True),
                   threading.Thread(target=builder, daemon=True)]
        for t in helpers:
            t.start()

        def take_and_launch():
            t0 = time.perf_counter()
            prepared = get(built_q)
            phase["handoff"] += time.perf_counter() - t0
            return prepared, launch(prepared, precision)

        try:
            cur = None
            nxt = take_and_launch()
            for i in range(n):
                prepared, launched = nxt
                nxt = take_and_launch() if i + 1 < n else None
                hand = [cur] if cur is not None else None
                cur = None
                tf = time.perf_counter()
                cur = finish(prepared, launched, free_q, hand)
                del prepared, launched
                phase["finish"] += time.perf_counter() - tf
        finally:
            stop.set()
            for t in helpers:
                t.join()
        drain_free()
        taits, plans, batch, zh = cur
        v, l2, ar = kn.jones_many(q, taits, zh)
        return taits, plans, batch, zh, v, l2, ar

    prime()
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
        "pipelined": "three threads: planning batch i+2 and building and uploading batch i+1 "
                     "overlap the GPU work of batch i; batch i+1 is queued on the stream "
                     "behind batch i",
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
        prime(precision=1)
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
        mtuned = tune.load("batched", 0) if not args.untuned else {}
        mtaits, mplans = kn.plan_many([np.ascontiguousarray(d.pd, dtype=np.int32)
                                       for d, _ in mixed], [mq for _, mq in mixed],
                                      **tune.plan_options(mtuned))
        mb = kn.Batch(mplans)
        if mtuned.get("grid"):
            mb.set_grid(int(mtuned["grid"]))
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
            "tuned": mtuned or None,
        }

    def golden(workload):
        """Oracle values stored for seed 0 of a workload (written by
        tests/golden/make_oracle_values.py from the oracle alone), or None."""
        path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_seed{args.seed}.json")
        try:
            with open(path) as f:
                return json.load(f)["knots"]
        except (OSError, ValueError):
            return None

    def errs_vs(zh_, gold):
        ez = []
        for i, g in enumerate(gold):
            m = complex(zh_[i, 0], zh_[i, 1])
            e = int(zh_.view(np.int64)[i, 2])
            mo = complex(g["z_re"], g["z_im"])
            ez.append(abs(m * 2.0 ** (e - g["z_exp2"]) - mo) / abs(mo))
        return ez

    def time_batch(b, reps=20):
        z = kn.alloc_scalars(len(b.plans))
        b.contract(stream=stream, z=z)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.contract(stream=stream, z=z)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, z.cpu().numpy()

    # ---------------------------------------------------------------- mixed precision workload
    # 16 knots of 300-600 crossings (at least 4 of 560-600), q = 3, one batch
    # launch in complex128 and in complex64, each knot against the oracle
    if not args.no_mixed:
        mk = gen.config_knots("mixed", args.seed)
        mpds = [np.ascontiguousarray(d.pd, np.int32) for d, _ in mk]
        gold = golden("mixed")
        leg = {"workload": "16 seeded lattice-walk knots, 300-600 raw crossings (>= 4 of "
                           "560-600), q=3, one batch launch",
               "crossings": [d.n for d, _ in mk]}
        ms_by = {}
        for prec, name in ((0, "c128"), (1, "c64")):
            setting = tuned[prec]
            _, plans_m = kn.plan_many(mpds, 3, precision=prec, **tune.plan_options(setting))
            bm = kn.Batch(plans_m)
            if setting.get("grid"):
                bm.set_grid(int(setting["grid"]))
            bm.upload(stream=stream)
            ms_m, zm_h = time_batch(bm)
            ms_by[prec] = ms_m
            rec_m = {"ms_per_launch": ms_m, "knots_per_s": len(mk) / (ms_m * 1e-3),
                     "tflops": bm.stats["flops"] / (ms_m * 1e-3) / 1e12}
            if gold is not None:
                ez = errs_vs(zm_h, gold)
                rec_m["rel_err_vs_oracle_per_knot"] = [float("%.3g" % x) for x in ez]
                rec_m["rel_err_vs_oracle_max"] = max(ez)
            leg[name] = rec_m
        leg["c64_speedup_vs_c128"] = ms_by[0] / ms_by[1]
        out["mixed_precision"] = leg

    # ---------------------------------------------------------------- 50-200 crossings, one knot per launch
    if not args.no_fp64_single:
        fk = gen.config_knots("fp64", args.seed)
        gold = golden("fp64")
        leg = {"workload": "64 seeded lattice-walk knots, 50-200 raw crossings, q=3 and q=5, "
                           "complex128, one knot per launch (kn_contract)"}
        for qv in (3, 5):
            idx = [i for i, (_, qq) in enumerate(fk) if qq == qv]
            single = [kn.Plan(kn.Tait(fk[i][0].pd), qv) for i in idx]
            wsf = kn.alloc_workspace(max(p_.workspace_bytes for p_ in single))
            zf = kn.alloc_scalars(len(single))
            for p_ in single[:4]:
                kn.contract(p_, workspace=wsf, stream=stream, z=zf[:1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j, p_ in enumerate(single):
                kn.contract(p_, workspace=wsf, stream=stream, z=zf[j:j + 1])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec_f = {"knots_per_s": len(single) / dt, "ms_per_knot": 1e3 * dt / len(single),
                     "tflops": sum(p_.stats["flops"] for p_ in single) / dt / 1e12}
            if gold is not None:
                rec_f["rel_err_vs_oracle_max"] = max(errs_vs(zf.cpu().numpy(),
                                                             [gold[i] for i in idx]))
            leg[f"q{qv}"] = rec_f
        out["fp64_one_knot_per_launch"] = leg

    # ---------------------------------------------------------------- gradients
    if not args.no_grad:
        gk = gen.config_knots("grad", args.seed)
        gpds = [np.ascontiguousarray(d.pd, np.int32) for d, _ in gk]
        _, gplans = kn.plan_many(gpds, 3, gradient=True, jones_only=False)
        gb = kn.Batch(gplans)
        gb.upload(stream=stream)
        zg = kn.alloc_scalars(len(gplans))
        gg = torch.empty((max(1, int(gb.stats["total_edges"])), 2), dtype=torch.float64,
                         device="cuda")
        gb.contract_backward(stream=stream, z=zg, grad=gg)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            gb.contract_backward(stream=stream, z=zg, grad=gg)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_g = e0.elapsed_time(e1) / reps
        out["gradient"] = {
            "workload": "32 seeded lattice-walk knots, 150-300 raw crossings, q=3, d log Z / d J_e "
                        "for every edge (forward and reverse sweep, one batch launch), complex128",
            "ms_per_launch": ms_g, "knots_per_s": len(gplans) / (ms_g * 1e-3),
            "edges_per_s": int(gb.stats["total_edges"]) / (ms_g * 1e-3),
            "tflops": gb.stats["flops"] / (ms_g * 1e-3) / 1e12,
        }

    if not args.no_wide:
        out["wide_knot"] = wide_knot_leg()

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        # single thread: the oracle knot after knot, BLAS limited to one thread
        t_cpu = 0.0
        n_done = 0
        worst = 0.0
        with threadpool_limits(limits=1):
            for i, (d, _) in enumerate(knots):
                dt, mo, eo = oracle_knot(d.pd, q)
                t_cpu += dt
                n_done += 1
                m = complex(zh[i, 0], zh[i, 1])
                e = int(zh.view(np.int64)[i, 2])
                worst = max(worst, abs(m * 2.0 ** (e - eo) - mo) / abs(mo))
                if t_cpu >= args.cpu_seconds:
                    break
        single = {"value": n_done / t_cpu, "unit": "knots/s", "cores": 1,
                  "sample": f"first {n_done} of the {B} knots of the step, {t_cpu:.1f} s",
                  "gpu_vs_oracle_max_rel_err": worst}
        # all cores: one oracle process per usable CPU (at most 16), each with
        # one BLAS thread, over the knots of the step in order, for a bounded
        # wall time; whole-job knots/s
        par = cpu_par
        workers = par["workers"]
        out["cpu_baseline"] = {
            "value": par["knots_per_s"],
            "unit": "knots/s",
            "cores": workers,
            "kind": "oracle",
            "sample": f"first {par['knots']} of the {B} knots of the step (same seed), numpy "
                      f"complex128 min-fill variable elimination, {workers} processes with one "
                      f"BLAS thread each, {par['wall_s']:.1f} s wall",
            "cpu": cpu_model(),
            "single_thread": single,
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
