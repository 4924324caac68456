"""Consistency checks of device programs (checks.h): the host validator
kn_image_check over the images of every kind of plan and batch, the faults it
must find in images altered on the host, and the checking build of the
library (libkn_checked.so), which runs the same checks on the device before
every task."""

from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1807_02119_amd import build, gen, kn
from tests import image_model as im
from tests.test_host import gemm64_cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plans():
    out = []
    for d, q in gen.config_knots("tiny", 0)[:6]:
        out.append(("tiny", kn.Plan(kn.Tait(d.pd, d.signs if d.n == 1 else None), q)))
    work = gen.config_knots("q3_200_600", 0, count=12)
    for i, (d, q) in enumerate(work[:4]):
        out.append((f"work{i}", kn.Plan(kn.Tait(d.pd), q)))
    t = kn.Tait(work[5][0].pd)
    out.append(("fp32", kn.Plan(t, 3, precision=1)))
    out.append(("tiles", kn.Plan(t, 3, big_step_macs_log2=4, tile_outputs=8)))
    out.append(("split", kn.Plan(t, 3, big_step_macs_log2=4, tile_macs_log2=3, split_min_log2=7)))
    out.append(("sliced", kn.Plan(t, 3, slice_log2_budget=6)))
    out.append(("separator", kn.Plan(t, 3, strategy=4)))
    g = kn.Tait(gen.lattice_knot((45, 1), 60, 120).pd)
    out.append(("gradient", kn.Plan(g, 3, gradient=True, jones_only=False)))
    out.append(("recompute", kn.Plan(g, 3, gradient=True, jones_only=False,
                                     mem_budget_bytes=1, allow_budget=True)))
    for label, d, q, kw in gemm64_cases()[:3]:
        out.append((label, kn.Plan(kn.Tait(d.pd), q, **kw)))
    return out


def test_images_of_every_plan_kind_pass():
    plans = _plans()
    modes = set()
    for label, p in plans:
        raw = p.image()
        r = kn.image_check(raw)
        assert r["code"] == 0, (label, r)
        modes.update(int(x) for x in im.Image(raw).steps["mode"])
    assert modes == {0, 1, 2, 3}  # serial, tiles, 32- and 64-blocks all seen
    b = kn.Batch([p for _, p in plans if not p.stats.get("n_recompute_steps")][:8])
    assert kn.image_check(b.image())["code"] == 0


def _edit(raw, dtype, off, n):
    """A writable numpy view of n records of dtype at byte offset off."""
    return np.frombuffer(raw, dtype, n, off)


def _first(image, pred):
    return next(i for i, s in enumerate(image.steps) if pred(s))


def test_planted_faults_are_found():
    """Each kind of fault, written into a copy of a valid image on the host,
    is reported with its code, task and step."""
    d, q = gen.config_knots("q3_200_600", 0, count=12)[5]
    p = kn.Plan(kn.Tait(d.pd), 3, big_step_macs_log2=4, tile_outputs=8)
    base = p.image()
    img = im.Image(base)
    h = img.h
    tile_step = _first(img, lambda s: int(s["mode"]) != 0)
    tile_task = next(i for i, t in enumerate(img.tasks)
                     if int(t["kind"]) == 1 and int(t["first"]) == tile_step)

    def check(mutate, code, task=None, step=None, image=None):
        raw = bytearray(base if image is None else image)
        mutate(raw)
        r = kn.image_check(bytes(raw))
        assert r["code"] == code, r
        if task is not None:
            assert r["task"] == task, r
        if step is not None:
            assert r["step"] == step, r

    def steps(raw):
        return _edit(raw, im.STEP, int(h["o_steps"]), int(h["n_steps"]))

    def arena_end(raw):
        steps(raw)[tile_step]["home_c"] = int(h["arena_elems"]) - 1

    check(arena_end, 3, tile_task, tile_step)

    def tile_shape(raw):  # the tile count no longer matches the outputs
        steps(raw)[tile_step]["nm"] *= 3

    check(tile_shape, 2, tile_task, -1)

    # a serial step of the default plan with a batch or row spin in A
    base2 = kn.Plan(kn.Tait(d.pd), 3).image()
    img2 = im.Image(base2)
    h2 = img2.h
    serial_step = _first(img2, lambda s: int(s["mode"]) == 0 and
                         (int(s["ranks"]) & 255) + ((int(s["ranks"]) >> 8) & 255) > 0)

    def gather(raw):
        s = _edit(raw, im.STEP, int(h2["o_steps"]), int(h2["n_steps"]))[serial_step]
        strides = _edit(raw, "<i4", int(h2["o_strides"]), int(h2["n_strides"]))
        size_a = int(img2.tensors[int(s["a"])]["size"])
        strides[int(s["str"])] = size_a  # one digit step of A's first spin leaves A

    check(gather, 5, step=serial_step, image=base2)

    def shape(raw):
        _edit(raw, im.STEP, int(h2["o_steps"]), int(h2["n_steps"]))[serial_step]["nm"] *= 3

    check(shape, 4, step=serial_step, image=base2)

    def tile_id(raw):
        tasks = _edit(raw, im.TASK, int(h["o_tasks"]), int(h["n_tasks"]))
        tasks[tile_task]["count"] = int(img.steps[tile_step]["n_tiles"])

    check(tile_id, 2, tile_task, -1)

    def out_slot(raw):
        knots = _edit(raw, im.KNOT, int(h["o_knots"]), int(h["n_knots"]))
        knots[0]["out_slot"] = int(h["n_outputs"])

    check(out_slot, 2)

    def guard(raw):
        hdr = _edit(raw, im.HDR, 0, 1)
        hdr[0]["guard_off"] = int(h["arena_off"])  # inside the arena

    check(guard, 3)

    def section(raw):
        hdr = _edit(raw, im.HDR, 0, 1)
        hdr[0]["n_steps"] = int(h["n_steps"]) + 1_000_000  # past the image

    check(section, 2)
    # the original still passes
    assert kn.image_check(base)["code"] == 0


def _load(lib_path):
    env = dict(os.environ, KN_LIBRARY=lib_path)
    code = ("from paper_1807_02119_amd import kn; "
            "print(int(kn.device_checks()), sorted(set(kn.EXPORTED) - set(dir(kn.lib()))))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip()


def test_checking_build_loads_and_reports_itself():
    if not os.path.exists(build.CHECKED_LIB):
        pytest.skip("libkn_checked.so not built")
    assert _load(build.CHECKED_LIB).startswith("1 ")
    assert _load(build.LIB).startswith("0 ")
