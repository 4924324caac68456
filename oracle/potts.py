"""The PACI partition function Z(q) on a signed Tait graph (Eqs. 2-3).

Test infrastructure (see ``oracle/__init__``).

Definition (Eqs. 2-3, and its tensor-network restatement Eq. 6):

    Z(q) = sum over spin assignments sigma: V -> {0..q-1} of
           prod over edges e=(u,v) of T_e(sigma_u, sigma_v),
    T_e(a, b) = 1 if a != b,  x_e if a == b,

with x_e = e^{J_e}.  For the Jones evaluation the couplings are
e^{J_pm} = -t^{-/+1}, i.e. x_e = -t^{-eps_e} (Sec. II).  A loop edge (u, u)
always sees a == b and contributes the constant x_e.

``eliminate`` computes the sum by plain variable elimination (sum out one
spin at a time, multiplying every factor that mentions it), in min-fill order,
rescaling every new factor by a power of two so that nothing overflows.  This
is a different algorithm from the device path (no absorption into vertex
tensors, no pairwise GEMMs): only the definition above is shared.
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def jones_weights(eps, t: complex) -> np.ndarray:
    """x_e = e^{J_e} = -t^{-eps_e} (Sec. II: e^{J_pm} = -t^{-/+1})."""
    t = complex(t)
    return np.array([-(t ** (-int(e))) for e in eps], dtype=np.complex128)


def min_fill_order(n_vertices: int, edges) -> list:
    """Greedy min-fill elimination order (ties: fewest neighbours, lowest id)."""
    adj = [set() for _ in range(n_vertices)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    alive = set(range(n_vertices))

    def fill(v):
        nb = list(adj[v])
        f = 0
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                if nb[b] not in adj[nb[a]]:
                    f += 1
        return f

    cost = {v: fill(v) for v in alive}
    order = []
    while alive:
        v = min(alive, key=lambda x: (cost[x], len(adj[x]), x))
        order.append(v)
        nb = list(adj[v])
        for a in nb:
            adj[a].discard(v)
        for a in range(len(nb)):
            for b in range(a + 1, len(nb)):
                adj[nb[a]].add(nb[b])
                adj[nb[b]].add(nb[a])
        alive.remove(v)
        del cost[v]
        touched = set(nb)
        for a in nb:
            touched |= adj[a]
        for a in touched:
            if a in alive:
                cost[a] = fill(a)
    return order


class ComplexAlgebra:
    """complex128 factors, rescaled by powers of two after every product."""

    exact = False

    def __init__(self, q: int):
        self.q = q

    def one(self):
        return np.array(1.0 + 0j)

    def const(self, c):
        return np.array(complex(c))

    def edge(self, x):
        q = self.q
        return np.ones((q, q), np.complex128) + (complex(x) - 1.0) * np.eye(q, dtype=np.complex128)

    def delta(self, x):
        return complex(x) * np.eye(self.q, dtype=np.complex128)

    def mul(self, a, b):
        return a * b

    def sum_axis(self, a, ax):
        return a.sum(axis=ax)

    def transpose(self, a, perm):
        return np.transpose(a, perm)

    def reshape(self, a, shape):
        return a.reshape(shape)

    def normalise(self, a):
        m = float(np.max(np.maximum(np.abs(a.real), np.abs(a.imag)))) if a.size else 0.0
        if m == 0.0 or not math.isfinite(m):
            return a, 0
        e = math.frexp(m)[1]
        return np.ldexp(a.real, -e) + 1j * np.ldexp(a.imag, -e), e


def edge_factors(alg, edges, x, replace: int | None = None):
    """Factors of Eq. 2: one q x q matrix per non-loop edge; loops give a list
    of constants.

    With ``replace = k`` edge k's factor is dT_k/dJ_k = x_k * delta instead.
    """
    const = []
    factors = []
    for k, ((u, v), xe) in enumerate(zip(edges, x)):
        if u == v:
            const.append(alg.const(xe))
        elif k == replace:
            factors.append(((u, v), alg.delta(xe)))
        else:
            factors.append(((u, v), alg.edge(xe)))
    return factors, const


def _align(alg, arr, vars_, union):
    """View ``arr`` (axes = ``vars_``) as an array over ``union`` with size-1 axes."""
    perm = sorted(range(len(vars_)), key=lambda k: union.index(vars_[k]))
    arr = alg.transpose(arr, perm)
    present = set(vars_)
    shape = tuple(alg.q if u in present else 1 for u in union)
    return alg.reshape(arr, shape)


def eliminate(alg, n_vertices: int, factors, const, order=None, edges=None):
    """Sum out every spin of ``factors`` (variable elimination).

    Returns ``(value, exp2)``: Z = value * 2**exp2 (exp2 is 0 for exact algebras).
    """
    factors = list(factors)
    exp2 = 0
    consts = list(const) if isinstance(const, list) else [const]
    const = alg.one()
    for c in consts:
        const, exp2 = _times(alg, const, c, exp2)
    if order is None:
        order = min_fill_order(n_vertices, [vs for vs, _ in factors] if edges is None else edges)
    for var in order:
        mine = [f for f in factors if var in f[0]]
        factors = [f for f in factors if var not in f[0]]
        if not mine:
            # a spin that no factor mentions: its q values each contribute 1
            const, exp2 = _times(alg, const, alg.const(alg.q), exp2)
            continue
        union = []
        for vs, _ in mine:
            for w in vs:
                if w not in union:
                    union.append(w)
        prod = None
        for vs, arr in mine:
            a = _align(alg, arr, list(vs), union)
            prod = a if prod is None else alg.mul(prod, a)
            if not alg.exact:
                prod, e = alg.normalise(prod)
                exp2 += e
        new = alg.sum_axis(prod, union.index(var))
        rest = tuple(w for w in union if w != var)
        if not alg.exact:
            new, e = alg.normalise(new)
            exp2 += e
        if rest:
            factors.append((rest, new))
        else:
            const, exp2 = _times(alg, const, new, exp2)
    if factors:
        raise AssertionError("elimination order missed a spin")
    if not alg.exact:
        return complex(const), exp2
    return const, 0


def _times(alg, const, f, exp2):
    """const * f, renormalised to a power-of-two mantissa for complex algebras."""
    const = alg.mul(const, f)
    if not alg.exact:
        const, e = alg.normalise(const)
        exp2 += e
    return const, exp2


def partition_function(n_vertices: int, edges, x, q: int):
    """Z(q) as ``(mantissa, exp2)`` by complex128 elimination."""
    alg = ComplexAlgebra(q)
    factors, const = edge_factors(alg, edges, x)
    return eliminate(alg, n_vertices, factors, const, edges=edges)


def to_complex(m, e) -> complex:
    return complex(math.ldexp(m.real, e), math.ldexp(m.imag, e))


def brute_force(n_vertices: int, edges, x, q: int) -> complex:
    """Z as the literal spin sum of Eq. 2 (vectorised over all q^n_v states)."""
    if q ** n_vertices > 4_000_000:
        raise ValueError("brute force limited to q^n_v <= 4e6")
    if n_vertices == 0:
        states = np.zeros((1, 0), np.int8)
    else:
        states = np.array(list(itertools.product(range(q), repeat=n_vertices)), dtype=np.int8)
    w = np.ones(len(states), np.complex128)
    for (u, v), xe in zip(edges, x):
        same = states[:, u] == states[:, v]
        w = w * np.where(same, complex(xe), 1.0)
    return complex(w.sum())


def brute_force_dz_dj(n_vertices: int, edges, x, q: int) -> np.ndarray:
    """dZ/dJ_e by the spin sum: x_e * sum over states with sigma_u == sigma_v of
    the product over the other edges."""
    states = np.array(list(itertools.product(range(q), repeat=n_vertices)), dtype=np.int8)
    out = np.zeros(len(edges), np.complex128)
    for k, (uk, vk) in enumerate(edges):
        w = np.where(states[:, uk] == states[:, vk], complex(x[k]), 0.0).astype(np.complex128)
        for j, (u, v) in enumerate(edges):
            if j != k:
                w = w * np.where(states[:, u] == states[:, v], complex(x[j]), 1.0)
        out[k] = w.sum()
    return out


def dlogz_dj(n_vertices: int, edges, x, q: int) -> np.ndarray:
    """d log Z / d J_e for every edge (holomorphic derivative).

    dT_e/dJ_e = x_e * delta(a, b), so dZ/dJ_e is the same sum with T_e replaced
    by x_e times the identity: one elimination per edge.  A loop gives 1.
    """
    alg = ComplexAlgebra(q)
    m0, e0 = partition_function(n_vertices, edges, x, q)
    order = min_fill_order(n_vertices, edges)
    out = np.zeros(len(edges), np.complex128)
    for k, (u, v) in enumerate(edges):
        if u == v:
            out[k] = 1.0
            continue
        factors, const = edge_factors(alg, edges, x, replace=k)
        m, e = eliminate(alg, n_vertices, factors, const, order=order)
        out[k] = (m / m0) * 2.0 ** (e - e0)
    return out
