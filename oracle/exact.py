"""Z(q) in exact arithmetic.

Test infrastructure (see ``oracle/__init__``).

By Eq. 1, t = t(q) is a root of t^2 - (q-2) t + 1 = 0 (t + 1/t = q - 2), so
t^{-1} = (q - 2) - t and every Jones coupling x_e = -t^{-eps_e} (Sec. II) lies
in the ring Z[t] = {a + b t : a, b integers} with t^2 = (q-2) t - 1.  Running
the same variable elimination as ``potts.eliminate`` over that ring (Python
integers, no rounding) gives Z(q) exactly as a + b t; converting to a complex
number at 60 significant digits (mpmath) then gives a reference that is exact
to far below double precision.
"""

from __future__ import annotations

import mpmath
import numpy as np

from . import potts


class ZtArray:
    """Array of elements a + b t of Z[t]/(t^2 - (q-2) t + 1)."""

    __slots__ = ("a", "b", "q")

    def __init__(self, a, b, q):
        self.a = a
        self.b = b
        self.q = q

    @property
    def shape(self):
        return np.shape(self.a)


class ExactAlgebra:
    exact = True

    def __init__(self, q: int):
        self.q = q

    def _arr(self, a, b):
        return ZtArray(np.asarray(a, dtype=object), np.asarray(b, dtype=object), self.q)

    def one(self):
        return self._arr(1, 0)

    def const(self, c):
        if isinstance(c, ZtArray):
            return c
        if isinstance(c, tuple):
            return self._arr(c[0], c[1])
        return self._arr(int(c), 0)

    def _eye(self, v):
        m = np.zeros((self.q, self.q), dtype=object)
        for i in range(self.q):
            m[i, i] = v
        return m

    def edge(self, x):
        xa, xb = x
        ones = np.empty((self.q, self.q), dtype=object)
        ones.fill(1)
        return self._arr(ones + self._eye(xa - 1), self._eye(xb))

    def delta(self, x):
        xa, xb = x
        return self._arr(self._eye(xa), self._eye(xb))

    def mul(self, x, y):
        # (a1 + b1 t)(a2 + b2 t) = a1 a2 - b1 b2 + (a1 b2 + a2 b1 + (q-2) b1 b2) t
        bb = x.b * y.b
        return ZtArray(x.a * y.a - bb, x.a * y.b + x.b * y.a + (self.q - 2) * bb, self.q)

    def sum_axis(self, x, ax):
        return ZtArray(x.a.sum(axis=ax), x.b.sum(axis=ax), self.q)

    def transpose(self, x, perm):
        return ZtArray(np.transpose(x.a, perm), np.transpose(x.b, perm), self.q)

    def reshape(self, x, shape):
        return ZtArray(np.reshape(x.a, shape), np.reshape(x.b, shape), self.q)


def jones_weights_exact(eps, q: int):
    """x_e = -t^{-eps}: eps=+1 -> -t^{-1} = (2-q) + t;  eps=-1 -> -t."""
    return [((2 - q), 1) if int(e) > 0 else (0, -1) for e in eps]


def partition_function_exact(n_vertices: int, edges, eps, q: int):
    """Z(q) for the Jones couplings as the exact pair (a, b): Z = a + b t(q)."""
    alg = ExactAlgebra(q)
    x = jones_weights_exact(eps, q)
    factors, const = potts.edge_factors(alg, edges, x)
    z, _ = potts.eliminate(alg, n_vertices, factors, const, edges=edges)
    return int(z.a.item()) if hasattr(z.a, "item") else int(z.a), \
        int(z.b.item()) if hasattr(z.b, "item") else int(z.b)


def t_mp(q: int, dps: int = 60):
    with mpmath.workdps(dps):
        return (mpmath.mpf(q) + mpmath.sqrt(q) * mpmath.sqrt(mpmath.mpf(q) - 4) - 2) / 2


def to_mp(ab, q: int, dps: int = 60):
    a, b = ab
    with mpmath.workdps(dps):
        return mpmath.mpf(a) + mpmath.mpf(b) * t_mp(q, dps)


def to_complex(ab, q: int) -> complex:
    """Nearest complex128 to a + b t(q) (None if out of double range)."""
    with mpmath.workdps(60):
        z = to_mp(ab, q)
        return complex(z)


def to_mant_exp2(ab, q: int):
    """(mantissa, exp2) with mantissa max(|re|,|im|) in [0.5, 1)."""
    with mpmath.workdps(60):
        z = mpmath.mpc(to_mp(ab, q))
        m = max(abs(z.real), abs(z.imag))
        if m == 0:
            return 0j, 0
        e = int(mpmath.floor(mpmath.log(m, 2))) + 1
        w = z / mpmath.mpf(2) ** e
        # guard against the floor landing one off at exact powers of two
        while max(abs(w.real), abs(w.imag)) >= 1:
            e += 1
            w = w / 2
        while max(abs(w.real), abs(w.imag)) < 0.5:
            e -= 1
            w = w * 2
        return complex(w), e
