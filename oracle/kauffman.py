"""Jones polynomial by the Kauffman-bracket state sum (textbook definition).

Test infrastructure (see ``oracle/__init__``).

This never builds a Tait graph, never uses Potts weights and never uses the
prefactor A(q) of Eq. 4, so it checks the whole Tait-graph route (Sec. II)
independently:

    <K> = sum over states S (one of two smoothings per crossing) of
          A^{#A(S) - #B(S)} d^{loops(S) - 1},   d = -A^2 - A^{-2},
    V_K(t) = (-A^3)^{-w} <K>  at  A = t^{-1/4}.

At a crossing (a, b, c, d) (counter-clockwise from the incoming under-arc),
rotating the over-strand b-d counter-clockwise sweeps the wedges (b, c) and
(d, a): the A-smoothing opens a channel between those two wedges, which
reconnects the strands as a-b and c-d; the B-smoothing reconnects a-d and b-c.

The result is returned as an integer Laurent polynomial in t (dict
exponent -> coefficient); for a knot all A-exponents are multiples of 4.
"""

from __future__ import annotations

from collections import defaultdict
from math import comb


def _loops(n_arcs: int, pairs) -> int:
    parent = list(range(n_arcs))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in pairs:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return sum(1 for x in range(n_arcs) if find(x) == x)


def bracket(pd) -> dict:
    """<K> as a Laurent polynomial in A (dict exponent -> int)."""
    pd = [tuple(int(v) for v in row) for row in pd]
    n = len(pd)
    if n == 0:
        return {0: 1}
    n_arcs = 2 * n
    # histogram of (#A - #B, loops) over all 2^n states
    hist = defaultdict(int)
    for state in range(1 << n):
        pairs = []
        na = 0
        for i, (a, b, c, d) in enumerate(pd):
            if (state >> i) & 1:
                pairs += [(a, b), (c, d)]
                na += 1
            else:
                pairs += [(a, d), (b, c)]
        hist[(na - (n - na), _loops(n_arcs, pairs))] += 1
    poly = defaultdict(int)
    for (diff, loops), cnt in hist.items():
        # d^(loops-1) = (-1)^k sum_j C(k, j) A^{2j} A^{-2(k-j)}
        k = loops - 1
        for j in range(k + 1):
            poly[diff + 2 * j - 2 * (k - j)] += cnt * comb(k, j) * (-1) ** k
    return {e: c for e, c in poly.items() if c != 0}


def jones_polynomial(pd, writhe: int) -> dict:
    """V_K as a Laurent polynomial in t (dict exponent -> int).

    (-A^3)^{-w} = (-1)^w A^{-3w};  A^k = t^{-k/4}.
    """
    br = bracket(pd)
    out = {}
    sgn = -1 if writhe % 2 else 1
    for e, c in br.items():
        ea = e - 3 * writhe
        if ea % 4 != 0:
            raise ValueError("A-exponent not a multiple of 4: not a knot diagram")
        out[-ea // 4] = out.get(-ea // 4, 0) + sgn * c
    return {e: c for e, c in out.items() if c != 0}


def evaluate(poly: dict, t: complex) -> complex:
    return complex(sum(c * (t ** e) for e, c in poly.items()))
