"""The engine's index decode (exact division by q and mixed-radix group
offsets, ``csrc/decode.h``) on the host: the header the HIP engine includes is
compiled here with g++ and checked against Python integer arithmetic over the
whole int32 range the planner admits, including the indices near q * 2^24
where a 40-bit reciprocal overflowed a 64-bit product."""

from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1807_02119_amd", "csrc")
QS = range(2, 9)
TOP = 2**31 - 1


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("decode") / "decode_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "decode_check.cpp"), "-o", exe], check=True)

    def run(lines):
        r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                           check=True)
        return [int(v) for v in r.stdout.split()]

    return run


def _division_inputs(q, rng):
    xs = {0, 1, q - 1, q, TOP, TOP - 1, TOP - q}
    for k in range(-64, 65):  # around q * 2^24 (where the old decode wrapped) and 2^25..2^30
        for base in [q * 2**24] + [2**p for p in range(24, 31)]:
            if 0 <= base + k <= TOP:
                xs.add(base + k)
    xs.update(int(v) for v in rng.integers(0, TOP, 4000, endpoint=True))
    for p in range(31):  # multiples of q and their neighbours at every scale
        m = (2**p // q) * q
        xs.update(v for v in (m - 1, m, m + 1) if 0 <= v <= TOP)
    return sorted(xs)


def test_exact_division_full_range(checker):
    rng = np.random.default_rng(20240601)
    lines, want = [], []
    for q in QS:
        for x in _division_inputs(q, rng):
            lines.append(f"d {q} {x}")
            want.append(x // q)
    got = checker(lines)
    bad = [(l, g, w) for l, g, w in zip(lines, got, want) if g != w]
    assert not bad, bad[:10]


def test_exact_division_dense_windows(checker):
    """Every x in windows of 2^20 at the bottom, around q * 2^24 and at the top
    of the int32 range (against the C++ integer divide)."""
    lines = []
    for q in QS:
        for lo in (0, q * 2**24 - 2**19, 2**30 - 2**19, TOP + 1 - 2**20):
            lines.append(f"s {q} {lo} {lo + 2**20}")
    assert checker(lines) == [0] * len(lines)


def test_group_offsets(checker):
    """Mixed-radix offsets of spin groups with arbitrary strides, up to groups of
    q^r <= 2^31 values."""
    rng = np.random.default_rng(7)
    lines, want = [], []
    for q in QS:
        rmax = 1
        while q ** (rmax + 1) <= TOP:
            rmax += 1
        for _ in range(300):
            r = int(rng.integers(1, rmax + 1))
            n = q**r
            # strides of an operand of at most 2^31 entries: a permutation of
            # q^0 .. q^(r-1), possibly scaled by the extent of spins outside the group
            perm = rng.permutation(r)
            str_ = [q ** int(perm[j]) for j in range(r)]
            scale = 1
            while scale * q * n <= TOP and rng.random() < 0.3:
                scale *= q
            str_ = [s * scale for s in str_]
            idx = int(rng.integers(0, n)) if rng.random() < 0.8 else n - 1
            lines.append(f"g {q} {idx} {r} " + " ".join(map(str, str_)))
            off, v = 0, idx
            for j in range(r - 1, -1, -1):
                off += (v % q) * str_[j]
                v //= q
            want.append(off)
    assert checker(lines) == want
