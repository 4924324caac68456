"""Invariants that fix V_K(t(q)) at q = 2, 3, 4 for diagrams of any size.

Test infrastructure (see ``oracle/__init__``).  These use no partition
function at all; they pin the oracle (and the device path) where no
elimination fits in memory.

* Goeritz matrix of the checkerboard colouring: the signed Laplacian of the
  Tait graph, G_uv = -sum_{c in (u,v)} eps_c (u != v), G_uu = sum of eps_c over
  the non-loop edges at u; delete one row and column.  |det| is the knot
  determinant; its corank over GF(p) is the rank of H_1 of the double branched
  cover with Z_p coefficients.
* q = 4 (t = 1): V_K(1) = 1 for every knot.
* q = 2 (t = i): V_K(i) = (-1)^{Arf K}, and Arf K = 0 iff det = +-1 (mod 8)
  (Murasugi / Levine).
* q = 3 (t = e^{i pi/3}): V_K(e^{i pi/3}) = +-(i sqrt 3)^d with d the GF(3)
  corank above (Lickorish-Millett).  Fixes |V| and which of {+-1, +-i} times
  a positive real V is; only the overall sign is left open.
"""

from __future__ import annotations

from fractions import Fraction


def goeritz(n_vertices: int, edges, eps):
    """Reduced Goeritz matrix (list of lists of ints), vertex 0 deleted."""
    g = [[0] * n_vertices for _ in range(n_vertices)]
    for (u, v), e in zip(edges, eps):
        if u == v:
            continue
        g[u][v] -= e
        g[v][u] -= e
        g[u][u] += e
        g[v][v] += e
    return [row[1:] for row in g[1:]]


def det_int(m) -> int:
    """Exact integer determinant (fraction-free Bareiss elimination)."""
    n = len(m)
    if n == 0:
        return 1
    a = [list(r) for r in m]
    sign = 1
    prev = 1
    for k in range(n - 1):
        if a[k][k] == 0:
            piv = next((i for i in range(k + 1, n) if a[i][k] != 0), None)
            if piv is None:
                return 0
            a[k], a[piv] = a[piv], a[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                a[i][j] = (a[i][j] * a[k][k] - a[i][k] * a[k][j]) // prev
        prev = a[k][k]
    return sign * a[n - 1][n - 1]


def corank_mod_p(m, p: int) -> int:
    n = len(m)
    if n == 0:
        return 0
    a = [[x % p for x in r] for r in m]
    rank = 0
    col = 0
    rows = n
    cols = len(a[0])
    for col in range(cols):
        piv = next((i for i in range(rank, rows) if a[i][col] % p), None)
        if piv is None:
            continue
        a[rank], a[piv] = a[piv], a[rank]
        inv = pow(a[rank][col], p - 2, p)
        a[rank] = [(x * inv) % p for x in a[rank]]
        for i in range(rows):
            if i != rank and a[i][col]:
                f = a[i][col]
                a[i] = [(x - f * y) % p for x, y in zip(a[i], a[rank])]
        rank += 1
    return n - rank


def knot_determinant(n_vertices: int, edges, eps) -> int:
    return abs(det_int(goeritz(n_vertices, edges, eps)))


def v_at_q2(n_vertices: int, edges, eps) -> int:
    """V_K(i) = +1 if det = +-1 mod 8 else -1."""
    d = knot_determinant(n_vertices, edges, eps) % 8
    return 1 if d in (1, 7) else -1


def q3_class(n_vertices: int, edges, eps):
    """(d, unit) with V_K(e^{i pi/3}) = +-unit * sqrt(3)^d, unit = i^d."""
    d = corank_mod_p(goeritz(n_vertices, edges, eps), 3)
    return d, (1j) ** d
