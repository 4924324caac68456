"""The engine's task-queue protocol (claim a slot, wait for its task id, run,
release the next group) modelled with host threads and std::atomic in
tests/queue_model.cpp, run under ThreadSanitizer: every task runs exactly
once, after its predecessors, with their data visible, and the grid drains,
for random programs and grid sizes from one workgroup up.  The same model
with the queue's release store and acquire load made relaxed (a planted
mistake) is reported as a data race."""

from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "queue_model.cpp")


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("queue_model")
    out = {}
    for name, extra in (("model", []), ("planted", ["-DKN_MODEL_RELAXED_QUEUE"])):
        exe = str(d / name)
        r = subprocess.run([cxx, "-std=c++20", "-O1", "-g", "-fsanitize=thread", *extra, SRC,
                            "-o", exe, "-lpthread"], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("ThreadSanitizer build unavailable: " + r.stderr[-500:])
        out[name] = exe
    return out


def _run(exe, seed, grid):
    return subprocess.run([exe, str(seed), str(grid)], capture_output=True, text=True,
                          timeout=120)


def test_protocol_race_free_and_drains(builds):
    for seed in range(1, 9):
        for grid in (1, 2, 5, 16):
            r = _run(builds["model"], seed, grid)
            assert r.returncode == 0 and r.stdout.startswith("ok"), (seed, grid, r.stdout,
                                                                     r.stderr[-3000:])
            assert "ThreadSanitizer" not in r.stderr


def test_planted_relaxed_queue_is_reported(builds):
    reported = 0
    for seed in (3, 4, 5, 6):
        r = _run(builds["planted"], seed, 8)
        reported += "WARNING: ThreadSanitizer: data race" in r.stderr
    assert reported >= 2
