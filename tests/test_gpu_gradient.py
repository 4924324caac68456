"""GPU parity of the reverse pass: d log Z / d J_e from kn_contract_backward
(and its batch form and the torch.autograd wrapper) against the oracle's
gradient, against central finite differences of log Z, and against torch's
own autograd through a plain dense contraction on tiny graphs.

Tolerances: 1e-10 relative for complex128 against the oracle (the gradient
is a ratio of two exactly contracted networks, each good to ~1e-15);
finite differences with step 1e-6 are good to ~1e-7 absolute for gradients of
order one; complex64 plans are checked to TOL32 (Z, and the gradient vector
normwise).
"""

from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import jones as ojones
from oracle import potts
from paper_1807_02119_amd import gen, kn
from tests.oracle_helpers import TOL32, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kn.lib()
    yield
    torch.cuda.synchronize()


def _log(msg):
    print(msg, flush=True)


def _couplings(t, rng, scale=0.4):
    J = rng.normal(scale=scale, size=2 * t.n_edges)
    return J, torch.tensor(J, dtype=torch.float64, device="cuda")


def _gpu_grad(plan, Jd):
    z, g = kn.contract_backward(plan, Jd)
    torch.cuda.synchronize()
    (m, e), = kn.scalars_from_device(z)
    gh = g.cpu().numpy()
    return m, e, gh[:, 0] + 1j * gh[:, 1]


def _oracle(t, J, q):
    uv, eps = t.edges()
    edges = [tuple(a) for a in uv]
    x = np.exp(J[0::2] + 1j * J[1::2])
    m, e = potts.partition_function(t.n_vertices, edges, x, q)
    return m, e, potts.dlogz_dj(t.n_vertices, edges, x, q)


@pytest.mark.parametrize("q", [3, 5])
def test_gradient_parity_small(q):
    rng = np.random.default_rng(200 + q)
    cases = [gen.trefoil(), gen.figure_eight(), gen.add_kink(gen.figure_eight(), 0, True, 1)]
    cases += [gen.lattice_knot((73, k), 10, 40) for k in range(8)]
    for d in cases:
        _log(f"gradient q={q} {d.label}")
        t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
        p = kn.Plan(t, q, jones_only=False, gradient=True)
        J, Jd = _couplings(t, rng)
        m, e, g = _gpu_grad(p, Jd)
        mo, eo, go = _oracle(t, J, q)
        assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10, d.label
        assert np.max(np.abs(g - go) / np.abs(go)) <= 1e-10, d.label


def test_gradient_tiled_steps():
    """Reverse steps split across workgroups (tiles, GEMM blocks, split-K)."""
    rng = np.random.default_rng(7)
    for k in range(3):
        d = gen.lattice_knot((74, k), 60, 120)
        t = kn.Tait(d.pd)
        J, Jd = _couplings(t, rng)
        mo, eo, go = _oracle(t, J, 3)
        for kw in (dict(big_step_macs_log2=4, split_min_log2=7),
                   dict(big_step_macs_log2=6, tile_outputs=16)):
            _log(f"gradient tiled {d.label} {kw}")
            p = kn.Plan(t, 3, jones_only=False, gradient=True, **kw)
            m, e, g = _gpu_grad(p, Jd)
            assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10
            assert np.max(np.abs(g - go) / np.abs(go)) <= 1e-10, kw


def test_gradient_jones_point():
    """J = NULL: the derivative at the Jones couplings."""
    tq = ojones.t_of_q(3)
    for k in range(4):
        d = gen.lattice_knot((75, k), 20, 60)
        t = kn.Tait(d.pd)
        p = kn.Plan(t, 3, gradient=True)
        m, e, g = _gpu_grad(p, None)
        uv, eps = t.edges()
        edges = [tuple(a) for a in uv]
        x = potts.jones_weights(eps, tq)
        go = potts.dlogz_dj(t.n_vertices, edges, x, 3)
        assert np.max(np.abs(g - go) / np.abs(go)) <= 1e-10


def test_gradient_finite_differences_large():
    """150-300 crossings (the differentiation workload): the gradient of
    selected edges against central differences of log Z from kn_contract."""
    rng = np.random.default_rng(11)
    knots = gen.config_knots("grad", 0, count=3)
    for d, q in knots:
        _log(f"finite differences {d.label} n={d.n}")
        t = kn.Tait(d.pd)
        J, Jd = _couplings(t, rng, scale=0.2)
        pg = kn.Plan(t, q, jones_only=False, gradient=True)
        m, e, g = _gpu_grad(pg, Jd)
        pf = kn.Plan(t, q, jones_only=False)

        def logz(Jh):
            z = kn.contract(pf, torch.tensor(Jh, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            (mm, ee), = kn.scalars_from_device(z)
            return np.log(mm) + ee * math.log(2.0)

        h = 1e-6
        for edge in rng.choice(t.n_edges, size=6, replace=False):
            for part, unit in ((0, 1.0), (1, 1j)):
                Jp, Jm = J.copy(), J.copy()
                Jp[2 * edge + part] += h
                Jm[2 * edge + part] -= h
                fd = (logz(Jp) - logz(Jm)) / (2 * h)
                # holomorphic: d/d(Re J) = g, d/d(Im J) = i g
                assert abs(fd - unit * g[edge]) < 1e-6, (d.label, edge, part)


def test_log_z_autograd_convention():
    """kn.log_z through torch.autograd equals torch's own autograd of a plain
    dense contraction of the same network (tiny graphs, CPU complex128)."""
    rng = np.random.default_rng(5)
    for d in (gen.trefoil(), gen.figure_eight(), gen.lattice_knot((76, 0), 6, 10)):
        t = kn.Tait(d.pd, d.signs if d.n == 1 else None)
        if t.n_vertices > 8:
            continue
        p = kn.Plan(t, 3, jones_only=False, gradient=True)
        Jc = torch.tensor(rng.normal(scale=0.3, size=t.n_edges)
                          + 1j * rng.normal(scale=0.3, size=t.n_edges),
                          dtype=torch.complex128, device="cuda", requires_grad=True)
        lz = kn.log_z(Jc, p)
        (lz.real * 0.7 + lz.imag * 0.2).backward()
        # reference: dense Z(J) by summing all spin states, in torch on the CPU
        Jr = Jc.detach().cpu().clone().requires_grad_(True)
        uv, _ = t.edges()
        n = t.n_vertices
        states = torch.cartesian_prod(*[torch.arange(3)] * n) if n > 1 else torch.arange(3)[:, None]
        w = torch.ones(states.shape[0], dtype=torch.complex128)
        for k, (a, b) in enumerate(uv):
            same = (states[:, a] == states[:, b])
            w = w * torch.where(same, torch.exp(Jr[k]), torch.ones((), dtype=torch.complex128))
        lref = torch.log(w.sum())
        (lref.real * 0.7 + lref.imag * 0.2).backward()
        assert abs(complex(lz.detach().cpu()) - complex(lref.detach())) < 1e-10
        assert torch.allclose(Jc.grad.cpu(), Jr.grad, rtol=1e-10, atol=1e-12)


def test_batch_gradient_matches_single():
    rng = np.random.default_rng(9)
    knots = [gen.lattice_knot((77, k), 20, 80) for k in range(10)]
    taits = [kn.Tait(d.pd) for d in knots]
    plans = [kn.Plan(t, q, jones_only=False, gradient=True)
             for t, q in zip(taits, [3, 5, 3, 2, 6, 3, 5, 3, 3, 4])]
    Js = [rng.normal(scale=0.3, size=2 * t.n_edges) for t in taits]
    b = kn.Batch(plans)
    Jall = torch.tensor(np.concatenate(Js), dtype=torch.float64, device="cuda")
    z, g = b.contract_backward(Jall)
    torch.cuda.synchronize()
    zs = kn.scalars_from_device(z)
    gh = g.cpu().numpy()
    for i, (p, J) in enumerate(zip(plans, Js)):
        m, e, gi = _gpu_grad(p, torch.tensor(J, dtype=torch.float64, device="cuda"))
        off = b.edge_offset(i)
        gb = gh[off:off + p.tait.n_edges, 0] + 1j * gh[off:off + p.tait.n_edges, 1]
        assert zs[i][1] == e and abs(zs[i][0] - m) <= 1e-12 * abs(m)
        assert np.max(np.abs(gb - gi) / np.abs(gi)) <= 1e-12


def test_gradient_fp32():
    rng = np.random.default_rng(13)
    for k in range(4):
        d = gen.lattice_knot((78, k), 30, 90)
        t = kn.Tait(d.pd)
        J, Jd = _couplings(t, rng)
        p = kn.Plan(t, 3, jones_only=False, gradient=True, precision=1)
        m, e, g = _gpu_grad(p, Jd)
        mo, eo, go = _oracle(t, J, 3)
        ez = rel_err(m * 2.0 ** (e - eo), mo)
        # the gradient vector normwise (an edge whose derivative is small
        # next to the others carries the error of the whole contraction)
        eg = np.max(np.abs(g - go)) / np.max(np.abs(go))
        ee = np.max(np.abs(g - go) / np.abs(go))
        print(f"fp32 gradient {d.label}: Z {ez:.1e}, normwise {eg:.1e}, elementwise {ee:.1e}",
              flush=True)
        assert ez <= TOL32 and eg <= TOL32


def test_backward_api_errors():
    t = kn.Tait(gen.figure_eight().pd)
    p = kn.Plan(t, 3, jones_only=False)
    J = torch.zeros(2 * t.n_edges, dtype=torch.float64, device="cuda")
    with pytest.raises(kn.KnError) as ei:
        kn.contract_backward(p, J, workspace=kn.alloc_workspace(p.workspace_bytes))
    assert ei.value.code == -6
    b = kn.Batch([p])
    with pytest.raises(kn.KnError):
        b.contract_backward(J)


def test_gradient_recompute_under_budget():
    """Gradient plans under mem_budget_bytes: forward intermediates dropped
    after their forward use and recomputed before their reverse use.  Against
    the oracle's gradient on 54-59 crossing knots at q = 8 and 5 (intermediates
    up to 2^15 entries), and against the unbudgeted plan on a 168-crossing grid
    walk (Sec. III.A, L = 36) whose large steps run as 64 x 64 GEMM blocks."""
    rng = np.random.default_rng(31)
    for k, q in ((0, 8), (3, 5)):
        d = gen.lattice_knot((75, k), 30, 60)
        t = kn.Tait(d.pd)
        full = kn.Plan(t, q, jones_only=False, gradient=True)
        p = kn.Plan(t, q, jones_only=False, gradient=True,
                    mem_budget_bytes=full.workspace_bytes // 2, allow_budget=True)
        assert p.stats["n_recompute_steps"] > 0
        _log(f"recompute q={q} {d.label}: {p.stats['n_recompute_steps']} steps again, "
             f"workspace {p.workspace_bytes} of {full.workspace_bytes}")
        J, Jd = _couplings(t, rng)
        m, e, g = _gpu_grad(p, Jd)
        mo, eo, go = _oracle(t, J, q)
        assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10
        assert np.max(np.abs(g - go) / np.abs(go)) <= 1e-10
    d = gen.random_grid_diagram(np.random.default_rng(1), 36)
    t = kn.Tait(d.pd)
    full = kn.Plan(t, 3, jones_only=False, gradient=True)
    p = kn.Plan(t, 3, jones_only=False, gradient=True,
                mem_budget_bytes=int(0.75 * full.workspace_bytes))
    assert p.stats["n_recompute_steps"] > 0 and p.workspace_bytes <= 0.75 * full.workspace_bytes
    J, Jd = _couplings(t, rng, scale=0.3)
    m, e, g = _gpu_grad(p, Jd)
    m0, e0, g0 = _gpu_grad(full, Jd)
    assert rel_err(m * 2.0 ** (e - e0), m0) <= 1e-10
    assert np.max(np.abs(g - g0) / np.abs(g0)) <= 1e-10
    uv, eps = t.edges()
    x = np.exp(J[0::2] + 1j * J[1::2])
    mo, eo = potts.partition_function(t.n_vertices, [tuple(a) for a in uv], x, 3)
    assert rel_err(m * 2.0 ** (e - eo), mo) <= 1e-10
