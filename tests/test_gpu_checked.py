"""The checking build (libkn_checked.so) on the GPU: every task and its steps
are checked on the device before they run (checks.h) and the guard zone after
the arena is checked after each launch.  Over plans of every kind -- serial
runs, tiles, 32- and 64-blocks, split contracted ranges, slices run as
device-side loops, forked runs, the adjoint with recomputation, complex64 and
a mixed batch -- every check passes (kn_workspace_status reads 0) and the results
equal the oracle's.  The checking library runs in a child process of its own
(KN_LIBRARY selects it), printing one line per case."""

from __future__ import annotations

import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

from paper_1807_02119_amd import build

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import math
import numpy as np
import torch
from paper_1807_02119_amd import gen, kn
from tests.oracle_helpers import TOL32, TOL64, oracle_z, rel_err
from tests.test_host import gemm64_cases

assert kn.device_checks(), "not the checking build"
torch.cuda.set_device(0)


def run(label, d, q, tol=TOL64, **kw):
    p = kn.Plan(kn.Tait(d.pd, d.signs if d.n == 1 else None), q, **kw)
    ws = kn.alloc_workspace(p.workspace_bytes)
    z = kn.contract(p, workspace=ws)
    torch.cuda.synchronize()
    st = kn.workspace_status(ws)
    (m, e), = kn.scalars_from_device(z)
    tg, mo, eo = oracle_z(d, q)
    err = rel_err(m * 2.0 ** (e - eo), mo)
    print(f"{label} n={d.n} q={q}: status {st['name']}, rel err {err:.2e}", flush=True)
    assert st["code"] == 0, (label, st)
    assert err <= tol, (label, err)


work = gen.config_knots("q3_200_600", 0, count=12)
for d, q in gen.config_knots("tiny", 0)[:4]:
    run("tiny", d, q)
d5 = work[5][0]
run("default", d5, 3)
run("tiles", d5, 3, big_step_macs_log2=4, tile_outputs=8)
run("split", d5, 3, big_step_macs_log2=4, tile_macs_log2=3, split_min_log2=7)
run("complex64", d5, 3, tol=TOL32, precision=1)
run("sliced", gen.lattice_knot((82, 1), 40, 120), 3, slice_log2_budget=4)
run("separator", work[7][0], 3, strategy=4)
run("forked", d5, 3, fork_serial_log2=6)
run("forked sliced", gen.lattice_knot((82, 1), 40, 120), 3, slice_log2_budget=4, fork_serial_log2=3)
for label, d, q, kw in gemm64_cases()[:3]:
    run(label, d, q, **kw)

# a mixed batch
plans = [kn.Plan(kn.Tait(d.pd), q) for d, q in work]
b = kn.Batch(plans)
z = b.contract()
torch.cuda.synchronize()
st = kn.workspace_status(b.workspace)
worst = 0.0
for (m, e), (d, q) in zip(kn.scalars_from_device(z), work):
    tg, mo, eo = oracle_z(d, q)
    worst = max(worst, rel_err(m * 2.0 ** (e - eo), mo))
print(f"batch of {len(work)}: status {st['name']}, worst rel err {worst:.2e}", flush=True)
assert st["code"] == 0 and worst <= TOL64

# the adjoint with forward tensors recomputed (a 54-59 crossing knot at q = 8
# under half the memory its gradient plan needs unbudgeted)
from oracle import potts
dg = gen.lattice_knot((75, 0), 30, 60)
tg_ = kn.Tait(dg.pd)
full = kn.Plan(tg_, 8, gradient=True, jones_only=False)
pg = kn.Plan(tg_, 8, gradient=True, jones_only=False,
             mem_budget_bytes=full.workspace_bytes // 2, allow_budget=True)
assert pg.stats["n_recompute_steps"] > 0
ws = kn.alloc_workspace(kn.backward_workspace_bytes(pg))
rng = np.random.default_rng(5)
Jh = rng.normal(scale=0.4, size=2 * tg_.n_edges)
J = torch.tensor(Jh, dtype=torch.float64, device="cuda")
z, g = kn.contract_backward(pg, J=J, workspace=ws)
torch.cuda.synchronize()
st = kn.workspace_status(ws)
uv, _ = tg_.edges()
x = np.exp(Jh[0::2] + 1j * Jh[1::2])
go = potts.dlogz_dj(tg_.n_vertices, [tuple(a) for a in uv], x, 8)
gd = g.cpu().numpy()
gd = gd[:, 0] + 1j * gd[:, 1]
gerr = float(np.max(np.abs(gd - go) / np.abs(go)))
print(f"gradient with recompute: status {st['name']}, max rel err {gerr:.2e}", flush=True)
assert st["code"] == 0 and gerr <= TOL64
print("checked build: all cases pass", flush=True)
"""


def test_checking_build_on_the_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(build.CHECKED_LIB):
        pytest.fail("libkn_checked.so is not built (python -m paper_1807_02119_amd.build --checked)")
    env = dict(os.environ, KN_LIBRARY=build.CHECKED_LIB)
    print("checked build: starting child", flush=True)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=280)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all cases pass" in r.stdout


def test_release_build_status_is_clear():
    """kn_workspace_status on the release library after a batch launch: no
    error recorded."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_02119_amd import gen, kn
    plans = [kn.Plan(kn.Tait(d.pd), q) for d, q in gen.config_knots("tiny", 0)]
    b = kn.Batch(plans)
    b.contract()
    torch.cuda.synchronize()
    assert not kn.device_checks()
    st = kn.workspace_status(b.workspace)
    assert st["code"] == 0, st
