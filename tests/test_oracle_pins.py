"""Pins for the CPU oracle: every oracle function checked against something
other than itself (values printed in the paper, closed forms, textbook
algorithms, exact arithmetic, invariants, brute force)."""

from __future__ import annotations

import cmath
import itertools
import math
import os

import numpy as np
import pytest

from oracle import diagram, exact, invariants, jones, kauffman, potts
from paper_1807_02119_amd import gen
from tests.oracle_helpers import oracle_tait, oracle_v, oracle_z, rel_err

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_fig1.txt")


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, re_, im_, src = line.split()
            rows.append((name, int(q), complex(float(re_), float(im_)), src))
    return rows


FIXTURE = {"trefoil": gen.trefoil, "unknot": lambda: gen.UNKNOT, "figure-eight": gen.figure_eight}


# ---------------------------------------------------------------- Eq. 1


def test_t_of_q_closed_forms():
    # Eq. 1 with principal roots
    assert abs(jones.t_of_q(2) - 1j) < 1e-15
    assert abs(jones.t_of_q(3) - cmath.exp(1j * math.pi / 3)) < 1e-15
    assert abs(jones.t_of_q(4) - 1.0) < 1e-15
    assert abs(jones.t_of_q(5) - (3 + math.sqrt(5)) / 2) < 1e-15
    assert abs(jones.t_of_q(6) - (2 + math.sqrt(3))) < 1e-14
    for q in range(2, 9):
        t = jones.t_of_q(q)
        # q = t + 2 + 1/t  (Potts-Jones correspondence)
        assert abs(t + 2 + 1 / t - q) < 1e-13


# ---------------------------------------------------------------- paper values


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}-q{r[1]}")
def test_paper_printed_values(row):
    name, q, want, src = row
    v, _ = oracle_v(FIXTURE[name](), q)
    assert abs(v - want) <= 1e-12 * max(1.0, abs(want)), (name, q, v, want, src)


def test_trefoil_closed_form_all_q():
    # right-handed trefoil: V = t + t^3 - t^4 (Fig. 1 caption form phi+phi^3-phi^4)
    for q in range(2, 9):
        t = jones.t_of_q(q)
        v, _ = oracle_v(gen.trefoil(), q)
        assert rel_err(v, t + t ** 3 - t ** 4) < 1e-12


def test_figure_eight_closed_form_all_q():
    for q in range(2, 9):
        t = jones.t_of_q(q)
        v, _ = oracle_v(gen.figure_eight(), q)
        want = t ** -2 - t ** -1 + 1 - t + t ** 2
        assert abs(v - want) < 1e-12 * max(1, abs(want))


def test_mirror_trefoil_is_conjugate_at_q3():
    v, _ = oracle_v(gen.mirror(gen.trefoil()), 3)
    assert abs(v + 1j * math.sqrt(3)) < 1e-12


def test_hand_count_trefoil_partition_function():
    # Tait graph of the trefoil fixture: 3 black regions joined in a triangle
    # (eps = +1); by hand, Z = sum over the 3 spins of prod of three q x q
    # weights = q(q-1)(q-2) + 3 q (q-1) x + q x^3 with x = -1/t.
    tg = oracle_tait(gen.trefoil())
    assert tg.n_vertices == 3 and sorted(tg.eps) == [1, 1, 1]
    assert tg.writhe == 3 and tg.tait_number == 3
    for q in range(2, 9):
        t = jones.t_of_q(q)
        x = -1 / t
        want = q * (q - 1) * (q - 2) + 3 * q * (q - 1) * x + q * x ** 3
        _, m, e = oracle_z(gen.trefoil(), q)
        assert rel_err(potts.to_complex(m, e), want) < 1e-13


# ---------------------------------------------------------------- Tait graph


def _small_diagrams(count=40, lo=3, hi=12, seed=5):
    return [gen.lattice_knot((seed, k), lo, hi) for k in range(count)]


def test_tait_graph_counts():
    # Euler: a connected 4-valent plane diagram with n crossings has n + 2
    # regions; the black ones are the Tait vertices, one edge per crossing.
    for d in _small_diagrams() + [gen.trefoil(), gen.figure_eight()]:
        face_of, nf = diagram.faces(d.pd)
        assert nf == d.n + 2
        tb = oracle_tait(d, True)
        tw = oracle_tait(d, False)   # other colour class (the dual graph)
        assert tb.n_vertices + tw.n_vertices == d.n + 2
        assert len(tb.edges) == d.n and len(tw.edges) == d.n
        assert tb.writhe == int(d.signs.sum())
        # the two colour classes see opposite Tait signs at every crossing
        assert all(a == -b for a, b in zip(tb.eps, tw.eps))


def test_crossing_signs_from_labels_match_geometry():
    for d in _small_diagrams():
        assert diagram.crossing_signs(d.pd) == [int(s) for s in d.signs]


def test_colour_convention_does_not_change_v():
    # white graph instead of black graph: same V (Sec. II convention)
    for d in _small_diagrams(12):
        for q in (2, 3, 5):
            vb, _ = oracle_v(d, q, True)
            vw, _ = oracle_v(d, q, False)
            assert rel_err(vw, vb) < 1e-10


# ---------------------------------------------------------------- Z (Eq. 2)


def _random_multigraph(rng, nv, ne):
    edges = []
    for _ in range(ne):
        u = int(rng.integers(nv))
        v = int(rng.integers(nv)) if rng.random() > 0.1 else u
        edges.append((u, v))
    x = rng.normal(size=ne) + 1j * rng.normal(size=ne)
    return edges, x


@pytest.mark.parametrize("q", [2, 3, 4, 5])
def test_elimination_matches_brute_force(q):
    rng = np.random.default_rng(q)
    for trial in range(25):
        nv = int(rng.integers(1, 9 if q <= 3 else 7))
        ne = int(rng.integers(0, 2 * nv + 3))
        edges, x = _random_multigraph(rng, nv, ne)
        m, e = potts.partition_function(nv, edges, x, q)
        bf = potts.brute_force(nv, edges, x, q)
        assert rel_err(potts.to_complex(m, e), bf) < 1e-11, (nv, edges)


def test_brute_force_special_cases():
    # no edges: q^n; a single edge: q(q-1) + q x; a loop: q x
    assert potts.brute_force(3, [], [], 3) == 27
    assert abs(potts.brute_force(2, [(0, 1)], [2.5], 4) - (4 * 3 + 4 * 2.5)) < 1e-12
    assert abs(potts.brute_force(1, [(0, 0)], [1j], 5) - 5j) < 1e-12
    # x = 1 everywhere: no interaction at all
    assert abs(potts.brute_force(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [1] * 4, 3) - 81) < 1e-9
    # x = 0: proper q-colourings of a 4-cycle: (q-1)^4 + (q-1)
    assert abs(potts.brute_force(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0] * 4, 3) - 18) < 1e-9


def test_elimination_overflow_safe():
    # 400 parallel edges of weight 8 between two spins: Z = q(q-1) + q 8^400,
    # far beyond double range; the mantissa/exponent form carries it.
    q = 3
    edges = [(0, 1)] * 400
    m, e = potts.partition_function(2, edges, [8.0] * 400, q)
    log2z = math.log2(abs(m)) + e
    assert abs(log2z - (1200 + math.log2(3))) < 1e-9


@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 7])
def test_exact_ring_matches_float_elimination(q):
    for k in range(6):
        d = gen.lattice_knot((17, k), 30, 90)
        tg = oracle_tait(d)
        ab = exact.partition_function_exact(tg.n_vertices, tg.edges, tg.eps, q)
        me, ee = exact.to_mant_exp2(ab, q)
        _, m, e = oracle_z(d, q)
        assert rel_err(m * 2.0 ** (e - ee), me) < 1e-12


def test_exact_ring_arithmetic():
    # t^2 = (q-2) t - 1 and t * t^{-1} = 1 in Z[t]
    for q in range(2, 9):
        alg = exact.ExactAlgebra(q)
        t = alg.const((0, 1))
        tinv = alg.const((q - 2, -1))
        one = alg.mul(t, tinv)
        assert (int(one.a), int(one.b)) == (1, 0)
        z = exact.to_complex((0, 1), q)
        assert abs(z - jones.t_of_q(q)) < 1e-14


# ---------------------------------------------------------------- V (Eq. 4)


@pytest.mark.parametrize("q", [2, 3, 5, 6])
def test_potts_route_matches_kauffman_state_sum(q):
    for d in _small_diagrams(30, 3, 11, seed=6):
        poly = kauffman.jones_polynomial(d.pd, int(d.signs.sum()))
        want = kauffman.evaluate(poly, jones.t_of_q(q))
        v, _ = oracle_v(d, q)
        assert abs(v - want) <= 1e-10 * max(1.0, abs(want)), (d.n, q)


def test_potts_route_matches_kauffman_on_grid_walks():
    rng = np.random.default_rng(11)
    done = 0
    while done < 12:
        d = gen.random_grid_diagram(rng, int(rng.integers(5, 9)))
        if d.n == 0 or d.n > 13:
            continue
        poly = kauffman.jones_polynomial(d.pd, int(d.signs.sum()))
        for q in (3, 5):
            want = kauffman.evaluate(poly, jones.t_of_q(q))
            v, _ = oracle_v(d, q)
            assert abs(v - want) <= 1e-10 * max(1.0, abs(want))
        done += 1


def test_kauffman_pins():
    # unknot with kinks of every kind is the unknot
    for over_first in (False, True):
        for s in (1, -1):
            k1 = gen.add_kink(gen.UNKNOT, 0, over_first, s)
            k2 = gen.add_kink(k1, 1, not over_first, -s)
            for d in (k1, k2):
                assert kauffman.jones_polynomial(d.pd, int(d.signs.sum())) == {0: 1}
    assert kauffman.jones_polynomial(gen.trefoil().pd, 3) == {1: 1, 3: 1, 4: -1}
    assert kauffman.jones_polynomial(gen.figure_eight().pd, 0) == {-2: 1, -1: -1, 0: 1, 1: -1, 2: 1}


def test_reidemeister_one_invariance():
    rng = np.random.default_rng(3)
    for d in _small_diagrams(8, 5, 40, seed=8):
        base = {q: oracle_v(d, q)[0] for q in (2, 3, 5)}
        k = d
        for _ in range(3):
            k = gen.add_kink(k, int(rng.integers(0, 2 * k.n)), bool(rng.integers(2)),
                             int(rng.choice([-1, 1])))
        for q in (2, 3, 5):
            assert rel_err(oracle_v(k, q)[0], base[q]) < 1e-10


def test_diagram_relabelling_invariance():
    rng = np.random.default_rng(4)
    for d in _small_diagrams(8, 5, 40, seed=9):
        for q in (3, 5):
            v0, _ = oracle_v(d, q)
            for d2 in (gen.reverse(d), gen.rotate_start(d, 3),
                       gen.relabel_crossings(d, rng.permutation(d.n))):
                assert rel_err(oracle_v(d2, q)[0], v0) < 1e-10


def test_mirror_inverts_t():
    # V_{mirror K}(t) = V_K(1/t): at q = 3 this is complex conjugation, at
    # real t (q >= 4) V(1/t) differs; check with the Kauffman polynomial.
    for d in _small_diagrams(8, 3, 11, seed=10):
        poly = kauffman.jones_polynomial(d.pd, int(d.signs.sum()))
        for q in (3, 5):
            t = jones.t_of_q(q)
            vm, _ = oracle_v(gen.mirror(d), q)
            assert abs(vm - kauffman.evaluate(poly, 1 / t)) < 1e-10 * max(1, abs(vm))


# ---------------------------------------------------------------- invariants


def _mid_knots(count=10, lo=60, hi=220, seed=12):
    return [gen.lattice_knot((seed, k), lo, hi) for k in range(count)]


def test_q4_identity():
    # V(1) = 1  =>  Z(4) = (-2)^{n_v+1} (-1)^w exactly
    for d in _mid_knots():
        tg, m, e = oracle_z(d, 4)
        ab = exact.partition_function_exact(tg.n_vertices, tg.edges, tg.eps, 4)
        want = (-2) ** (tg.n_vertices + 1) * (-1) ** (tg.writhe % 2)
        assert ab[0] + ab[1] == want     # t(4) = 1
        me, ee = exact.to_mant_exp2((want, 0), 4)
        assert rel_err(m * 2.0 ** (e - ee), me) < 1e-12


def test_q2_arf_invariant():
    for d in _mid_knots():
        tg = oracle_tait(d)
        v, _ = oracle_v(d, 2)
        assert abs(v - invariants.v_at_q2(tg.n_vertices, tg.edges, tg.eps)) < 1e-9


def test_q3_lickorish_millett():
    for d in _mid_knots():
        tg = oracle_tait(d)
        dd, unit = invariants.q3_class(tg.n_vertices, tg.edges, tg.eps)
        v, l2 = oracle_v(d, 3)
        assert abs(l2 - dd * math.log2(3) / 2) < 1e-9
        ratio = v / (unit * 3 ** (dd / 2))
        assert min(abs(ratio - 1), abs(ratio + 1)) < 1e-9


def test_invariant_helpers():
    assert invariants.det_int([[2, 1], [1, 2]]) == 3
    assert invariants.det_int([[0, 1], [1, 0]]) == -1
    assert invariants.corank_mod_p([[3, 0], [0, 1]], 3) == 1
    tg = oracle_tait(gen.trefoil())
    assert invariants.knot_determinant(tg.n_vertices, tg.edges, tg.eps) == 3
    tg = oracle_tait(gen.figure_eight())
    assert invariants.knot_determinant(tg.n_vertices, tg.edges, tg.eps) == 5


# ---------------------------------------------------------------- gradient


def test_gradient_matches_brute_force():
    rng = np.random.default_rng(21)
    for trial in range(10):
        nv = int(rng.integers(2, 7))
        edges, x = _random_multigraph(rng, nv, int(rng.integers(1, 10)))
        q = int(rng.choice([2, 3, 4]))
        z = potts.brute_force(nv, edges, x, q)
        dz = potts.brute_force_dz_dj(nv, edges, x, q)
        g = potts.dlogz_dj(nv, edges, x, q)
        assert np.allclose(g * z, dz, rtol=1e-10, atol=1e-12 * abs(z))


def test_gradient_closed_forms_and_fd():
    # loop: dlogZ/dJ = 1; pendant edge: x / (x + q - 1); central differences
    q = 3
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (1, 1)]
    x = np.array([0.3 + 0.2j, -0.5 + 1j, 1.5 - 0.3j, 0.7 + 0.7j, -2 + 0.1j])
    g = potts.dlogz_dj(4, edges, x, q)
    assert abs(g[4] - 1.0) < 1e-12
    assert abs(g[3] - x[3] / (x[3] + q - 1)) < 1e-12
    J = np.log(x)
    h = 1e-6
    for k in range(len(edges)):
        Jp, Jm = J.copy(), J.copy()
        Jp[k] += h
        Jm[k] -= h
        zp = potts.to_complex(*potts.partition_function(4, edges, np.exp(Jp), q))
        zm = potts.to_complex(*potts.partition_function(4, edges, np.exp(Jm), q))
        fd = (np.log(zp) - np.log(zm)) / (2 * h)
        assert abs(fd - g[k]) < 1e-7


# ---------------------------------------------------------------- planted mistakes


def test_pins_catch_planted_mistakes(monkeypatch):
    """Each plausible oracle mistake makes a pin above fail."""
    d = gen.trefoil()
    good = oracle_v(d, 3)[0]
    # (1) wrong coupling sign convention: e^{J} = -t^{+eps}
    monkeypatch.setattr(potts, "jones_weights",
                        lambda eps, t: np.array([-(complex(t) ** int(e)) for e in eps]))
    assert abs(oracle_v(d, 3)[0] - good) > 1e-3
    monkeypatch.undo()
    # (2) writhe exponent dropped from A(q)
    orig = jones.log_prefactor
    monkeypatch.setattr(jones, "log_prefactor", lambda q, n, w, tau: orig(q, n, 0, tau))
    assert abs(oracle_v(d, 3)[0] - good) > 1e-3
    monkeypatch.undo()
    # (3) n_v + 1 replaced by n_v in A(q)
    monkeypatch.setattr(jones, "log_prefactor", lambda q, n, w, tau: orig(q, n - 1, w, tau))
    assert abs(oracle_v(d, 3)[0] - good) > 1e-3
    monkeypatch.undo()
    # (4) Tait sign read on the wrong side of the over-strand
    orig_tg = diagram.tait_graph

    def flipped(pd, signs=None, outer_arc=0, outer_left=True):
        tg = orig_tg(pd, signs, outer_arc, outer_left)
        tg.eps = [-e for e in tg.eps]
        tg.tait_number = -tg.tait_number
        return tg

    monkeypatch.setattr(diagram, "tait_graph", flipped)
    assert abs(oracle_v(d, 3)[0] - good) > 1e-3
    monkeypatch.undo()
    # (5) elimination that forgets isolated spins (factor q)
    assert abs(potts.to_complex(*potts.partition_function(3, [(0, 1)], [2.0], 3))
               - potts.brute_force(3, [(0, 1)], [2.0], 3)) < 1e-12
