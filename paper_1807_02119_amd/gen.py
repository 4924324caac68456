"""Seeded synthetic knot diagrams: the input side of the evaluation pipeline.

This module only draws knot diagrams and writes them down as PD codes.  It holds
none of the evaluation method's arithmetic (no Tait graph, no Potts weights, no
contraction): the device path and the CPU oracle both take its PD codes as
their input.

Diagram conventions (shared by every consumer of a PD code):

* A diagram of one closed curve with ``n`` crossings is visited ``2n`` times
  along its orientation.  Visit ``k`` is the ``k``-th time the curve passes a
  crossing; arc ``k`` runs from visit ``k`` to visit ``k+1`` (mod ``2n``).
* ``pd[i] = (a, b, c, d)``: the four arc labels around crossing ``i``, listed
  counter-clockwise starting at the incoming under-arc ``a`` (so ``c = a+1``
  is the outgoing under-arc).  For a positive crossing ``b`` is the outgoing
  over-arc (``b = d+1`` mod ``2n``), for a negative one ``d`` is.
* The crossing sign (twist sign of Sec. II) is the sign of the z-component
  of ``dir(over) x dir(under)``: the right-handed crossing is positive.

Generators:

* ``lattice``: a closed unit-step walk on the square grid (equal numbers of
  +x, -x, +y, -y steps, shuffled), every vertex jittered by U(-1/4, 1/4)^2 so
  that the polygon is generic; crossings are all proper intersections of
  non-adjacent segments; one uniform over/under bit per crossing.
* ``grid``: the random grid walk of Sec. III.A -- two random permutations
  ``x, y`` of ``range(L)``, steps ``(x_i, y_i) -> (x_i, y_{i+1}) ->
  (x_{i+1}, y_{i+1})``, vertical segments always over horizontal ones.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Diagram:
    """One oriented knot diagram.

    ``gauss``: int64[2n, 2] -- visit k passes crossing ``gauss[k,0]`` on the
    over-strand iff ``gauss[k,1] == 1``.  ``signs``: int8[n] crossing signs.
    """

    gauss: np.ndarray
    signs: np.ndarray
    label: str = ""

    @property
    def n(self) -> int:
        return int(self.signs.shape[0])

    @property
    def pd(self) -> np.ndarray:
        return gauss_to_pd(self.gauss, self.signs)


def gauss_to_pd(gauss: np.ndarray, signs: np.ndarray) -> np.ndarray:
    """PD code (int32[n, 4]) of a signed Gauss sequence (conventions above)."""
    n = int(len(signs))
    m = 2 * n
    pd = np.zeros((n, 4), dtype=np.int32)
    under = np.full(n, -1, dtype=np.int64)
    over = np.full(n, -1, dtype=np.int64)
    for k in range(m):
        c, is_over = int(gauss[k, 0]), int(gauss[k, 1])
        if is_over:
            if over[c] >= 0:
                raise ValueError("crossing visited twice on the over-strand")
            over[c] = k
        else:
            if under[c] >= 0:
                raise ValueError("crossing visited twice on the under-strand")
            under[c] = k
    if (under < 0).any() or (over < 0).any():
        raise ValueError("every crossing must be visited once over and once under")
    for c in range(n):
        ku, ko = int(under[c]), int(over[c])
        a, cc = (ku - 1) % m, ku
        o_in, o_out = (ko - 1) % m, ko
        if signs[c] > 0:
            pd[c] = (a, o_out, cc, o_in)
        else:
            pd[c] = (a, o_in, cc, o_out)
    return pd


def _cross(ax, ay, bx, by):
    return ax * by - ay * bx


def polygon_to_diagram(pts: np.ndarray, over_of, label: str = "") -> Diagram:
    """Diagram of the closed polygon ``pts[0] -> pts[1] -> ... -> pts[0]``.

    ``over_of(i, j, idx)`` returns True when segment ``i`` passes over segment
    ``j`` at the ``idx``-th crossing (crossings enumerated in (i < j) order).
    The polygon must be generic (no three segments through a point, no
    collinear overlaps of non-adjacent segments).
    """
    pts = np.asarray(pts, dtype=np.float64)
    nseg = len(pts)
    p0 = pts
    d = np.roll(pts, -1, axis=0) - pts
    # all pairs (i < j): solve p0_i + t d_i = p0_j + u d_j
    i_idx, j_idx = np.triu_indices(nseg, k=2)
    keep = ~((i_idx == 0) & (j_idx == nseg - 1))
    i_idx, j_idx = i_idx[keep], j_idx[keep]
    di, dj = d[i_idx], d[j_idx]
    w = p0[j_idx] - p0[i_idx]
    den = _cross(di[:, 0], di[:, 1], dj[:, 0], dj[:, 1])
    with np.errstate(divide="ignore", invalid="ignore"):
        t = _cross(w[:, 0], w[:, 1], dj[:, 0], dj[:, 1]) / den
        u = _cross(w[:, 0], w[:, 1], di[:, 0], di[:, 1]) / den
    hit = (den != 0) & (t > 0) & (t < 1) & (u > 0) & (u < 1)
    ci, cj, ct, cu = i_idx[hit], j_idx[hit], t[hit], u[hit]
    n = len(ci)
    if n == 0:
        return Diagram(np.zeros((0, 2), np.int64), np.zeros(0, np.int8), label)
    over_i = np.array([bool(over_of(int(ci[x]), int(cj[x]), x)) for x in range(n)])
    # visits: (segment, parameter) -> crossing id, over flag
    seg = np.concatenate([ci, cj])
    par = np.concatenate([ct, cu])
    cid = np.concatenate([np.arange(n), np.arange(n)])
    isover = np.concatenate([over_i, ~over_i]).astype(np.int64)
    order = np.lexsort((par, seg))
    gauss = np.stack([cid[order], isover[order]], axis=1).astype(np.int64)
    d_over = np.where(over_i[:, None], d[ci], d[cj])
    d_under = np.where(over_i[:, None], d[cj], d[ci])
    s = _cross(d_over[:, 0], d_over[:, 1], d_under[:, 0], d_under[:, 1])
    signs = np.where(s > 0, 1, -1).astype(np.int8)
    return Diagram(gauss, signs, label)


# --------------------------------------------------------------------------
# generators


def lattice_polygon(rng: np.random.Generator, n_steps: int) -> np.ndarray:
    """Closed unit-step walk of ``n_steps`` (multiple of 4), jittered."""
    m = n_steps // 4
    steps = np.array([(1, 0)] * m + [(-1, 0)] * m + [(0, 1)] * m + [(0, -1)] * m,
                     dtype=np.float64)
    steps = steps[rng.permutation(len(steps))]
    pts = np.concatenate([np.zeros((1, 2)), np.cumsum(steps, axis=0)[:-1]], axis=0)
    pts = pts + rng.uniform(-0.25, 0.25, size=pts.shape)
    return pts


def lattice_diagram(rng: np.random.Generator, n_steps: int, label: str = "") -> Diagram:
    pts = lattice_polygon(rng, n_steps)
    # one uniform over/under bit per crossing, drawn in (i < j) order
    bits = {}

    def over_of(i, j, idx):
        if idx not in bits:
            bits[idx] = bool(rng.integers(0, 2))
        return bits[idx]

    return polygon_to_diagram(pts, over_of, label)


def grid_polygon(x, y) -> np.ndarray:
    """Vertices of the grid walk (x_i, y_i) -> (x_i, y_{i+1}) -> (x_{i+1}, y_{i+1})."""
    x = np.asarray(x)
    y = np.asarray(y)
    L = len(x)
    pts = []
    for i in range(L):
        pts.append((x[i], y[i]))
        pts.append((x[i], y[(i + 1) % L]))
    return np.array(pts, dtype=np.float64)


def grid_diagram(x, y, label: str = "") -> Diagram:
    """Grid-walk diagram of Sec. III.A: vertical segments pass over horizontal ones."""
    pts = grid_polygon(x, y)
    d = np.roll(pts, -1, axis=0) - pts
    vertical = d[:, 0] == 0

    def over_of(i, j, idx):
        if vertical[i] == vertical[j]:
            raise ValueError("parallel grid segments cannot cross")
        return bool(vertical[i])

    return polygon_to_diagram(pts, over_of, label)


def random_grid_diagram(rng: np.random.Generator, L: int, label: str = "") -> Diagram:
    x = rng.permutation(L)
    y = rng.permutation(L)
    return grid_diagram(x, y, label)


# --------------------------------------------------------------------------
# diagram moves (used to build invariance tests)


def add_kink(diag: Diagram, pos: int, over_first: bool, sign: int) -> Diagram:
    """Insert a one-crossing curl (a Reidemeister-I kink) on arc ``pos - 1``.

    The new crossing is visited twice in a row, right before visit ``pos``.
    All four (over_first, sign) combinations are planar curls.
    """
    n = diag.n
    m = 2 * n
    pos = pos % max(m, 1)
    new = n
    v1 = (new, 1 if over_first else 0)
    v2 = (new, 0 if over_first else 1)
    g = [tuple(r) for r in diag.gauss.tolist()]
    g = g[:pos] + [v1, v2] + g[pos:]
    return Diagram(np.array(g, dtype=np.int64).reshape(-1, 2),
                   np.concatenate([diag.signs, np.array([1 if sign > 0 else -1], np.int8)]),
                   diag.label + "+kink")


def mirror(diag: Diagram) -> Diagram:
    """Mirror image: every crossing switched (over <-> under, sign negated)."""
    g = diag.gauss.copy()
    g[:, 1] = 1 - g[:, 1]
    return Diagram(g, (-diag.signs).astype(np.int8), diag.label + "+mirror")


def reverse(diag: Diagram) -> Diagram:
    """Same diagram with the orientation reversed (crossing signs unchanged)."""
    return Diagram(diag.gauss[::-1].copy(), diag.signs.copy(), diag.label + "+rev")


def rotate_start(diag: Diagram, k: int) -> Diagram:
    """Same diagram with the visit numbering started ``k`` visits later."""
    return Diagram(np.roll(diag.gauss, -k, axis=0), diag.signs.copy(), diag.label + f"+rot{k}")


def relabel_crossings(diag: Diagram, perm: np.ndarray) -> Diagram:
    """Renumber crossing ``c`` as ``perm[c]``."""
    g = diag.gauss.copy()
    g[:, 0] = perm[g[:, 0]]
    s = np.zeros_like(diag.signs)
    s[perm] = diag.signs
    return Diagram(g, s, diag.label + "+relabel")


# --------------------------------------------------------------------------
# fixtures (grid walks in the convention of Sec. III.A)

UNKNOT = Diagram(np.zeros((0, 2), np.int64), np.zeros(0, np.int8), "unknot")


def trefoil() -> Diagram:
    """Right-handed trefoil: grid walk L=5, x=[4,2,0,3,1], y=[4,1,3,0,2]."""
    return grid_diagram([4, 2, 0, 3, 1], [4, 1, 3, 0, 2], "trefoil")


def figure_eight() -> Diagram:
    """Figure-eight knot: grid walk L=6, x=[0,4,1,3,5,2], y=[2,5,3,1,4,0]."""
    return grid_diagram([0, 4, 1, 3, 5, 2], [2, 5, 3, 1, 4, 0], "figure-eight")


# --------------------------------------------------------------------------
# seeded workloads

def _steps_for(target: float) -> int:
    # mean raw crossings c of a jittered unit-step walk of N steps follow
    # c ~ 128 (N/120)^1.16 between N=24 and N=500 (calibrate_lattice, 40
    # walks per length); invert it and round to a multiple of 4.
    a = max(target, 1.0)
    n = 4 * int(round(30.0 * (a / 128.0) ** 0.863))
    return max(8, n)


def lattice_knot(seed_words, lo: int, hi: int, label: str = "", max_tries: int = 4000) -> Diagram:
    """Lattice-walk knot whose raw crossing count lies in [lo, hi]."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_words)))
    target = 0.5 * (lo + hi)
    base = _steps_for(target)
    for attempt in range(max_tries):
        jitter = int(rng.integers(-2, 3)) * 4
        ns = max(8, base + jitter)
        d = lattice_diagram(rng, ns, label)
        if lo <= d.n <= hi:
            return d
        # walk length adapts towards the window
        if d.n < lo:
            base += 4
        elif d.n > hi:
            base = max(8, base - 4)
    raise RuntimeError(f"no lattice knot with {lo}..{hi} crossings after {max_tries} tries")


def calibrate_lattice(lengths, per=200, seed=0):
    """Mean raw crossing count of lattice walks of each length (for _steps_for)."""
    rng = np.random.default_rng(seed)
    out = {}
    for n in lengths:
        out[n] = float(np.mean([lattice_diagram(rng, n).n for _ in range(per)]))
    return out


#: Named workloads.  Each entry: (config id, q values, knot count per seed,
#: crossing window or None, description).
CONFIGS = {
    "tiny": dict(cid=0, qs=(3,), count=20, window=(12, 20),
                 fixtures=True, desc="20 lattice knots, 12-20 crossings + unknot/trefoil/figure-eight, q=3"),
    "fp64": dict(cid=1, qs=(3, 5), count=64, window=(50, 200), fixtures=False,
                 desc="64 lattice knots, 50-200 crossings, q=3 and q=5"),
    "mixed": dict(cid=2, qs=(3,), count=16, window=(300, 600), fixtures=False,
                  desc="16 lattice knots, 300-600 crossings (>=4 with 560-600), q=3"),
    "batched": dict(cid=3, qs=(2, 3, 5, 6), count=512, window=None, fixtures=False,
                    desc="512 lattice knots, crossings ~U{20..250}, q ~U{2,3,5,6}"),
    "grad": dict(cid=4, qs=(3,), count=32, window=(150, 300), fixtures=False,
                 desc="32 lattice knots, 150-300 crossings, q=3"),
    "q3_200_600": dict(cid=5, qs=(3,), count=256, window=(200, 600), fixtures=False,
                       desc="lattice knots, 200-600 crossings, q=3"),
}


def config_knots(name: str, seed: int = 0, count: int | None = None):
    """List of (Diagram, q) for a named workload, fully determined by ``seed``."""
    cfg = CONFIGS[name]
    cid = cfg["cid"]
    cnt = cfg["count"] if count is None else count
    out = []
    qs = cfg["qs"]
    for k in range(cnt):
        if name == "batched":
            rng = np.random.default_rng(np.random.SeedSequence([cid, seed, k, 7]))
            target = int(rng.integers(20, 251))
            q = int(qs[int(rng.integers(0, len(qs)))])
            tol = max(2, target // 20)
            d = lattice_knot((cid, seed, k), target - tol, target + tol, f"{name}/{seed}/{k}")
            out.append((d, q))
            continue
        lo, hi = cfg["window"]
        if name == "mixed" and k < 4:
            lo = 560
        d = lattice_knot((cid, seed, k), lo, hi, f"{name}/{seed}/{k}")
        for q in qs:
            out.append((d, q))
    if cfg.get("fixtures"):
        for d in (UNKNOT, trefoil(), figure_eight()):
            for q in qs:
                out.append((d, q))
    return out
