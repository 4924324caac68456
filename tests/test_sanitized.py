"""The host library built with AddressSanitizer and UndefinedBehaviorSanitizer
(``python -m paper_1807_02119_amd.build --sanitize``) under the CPU tests of the
host code: Tait graphs, planning, device programs and their CPU model,
normalisation, the index decode, and the image validator on valid and on
deliberately corrupted images.  Any invalid memory access or undefined
behaviour in the host C++ aborts the child process."""

from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    from paper_1807_02119_amd import build

    try:
        lib = build.build_sanitized()
    except RuntimeError as e:  # no sanitizer runtime in this toolchain
        pytest.skip(f"sanitized build unavailable: {e}")
    env = build.sanitizer_env()
    code = ("import sys; sys.path.insert(0, %r); from paper_1807_02119_amd import kn; kn.lib(); "
            "m = open('/proc/self/maps').read(); "
            "assert kn.LIB_PATH.endswith('libkn_san.so') and 'libkn_san.so' in m and 'libasan' in m"
            % ROOT)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_host.py"),
                        os.path.join(ROOT, "tests", "test_decode.py"),
                        os.path.join(ROOT, "tests", "test_checks.py"),
                        "-k", "not checking_build"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0 and " passed" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert os.path.exists(lib)
