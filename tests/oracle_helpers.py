"""Shared test helpers: run the oracle end to end on a diagram."""

from __future__ import annotations

import numpy as np

from oracle import diagram, jones, potts


# Tolerances.  complex128: 1e-10 relative (the target for the exact method;
# measured ~1e-14).  complex64 (FP32 storage and accumulation, FP64/int64
# exponents): a few times the error of a random walk of FP32 roundings,
# u sqrt(n) with u = 2^-24 and n ~ 10^3 roundings along a knot's
# contraction chain (several per step over ~400 steps), i.e. ~2e-6; measured
# up to 2.5e-6 on 200-600 crossing knots.
TOL64 = 1e-10
TOL32 = 1e-5


def oracle_tait(d, outer_left=True):
    return diagram.tait_graph(d.pd, d.signs if d.n == 1 else None, outer_left=outer_left)


def oracle_z(d, q, outer_left=True):
    tg = oracle_tait(d, outer_left)
    x = potts.jones_weights(tg.eps, jones.t_of_q(q))
    m, e = potts.partition_function(tg.n_vertices, tg.edges, x, q)
    return tg, m, e


def oracle_v(d, q, outer_left=True):
    tg, m, e = oracle_z(d, q, outer_left)
    v, l2 = jones.jones_value(q, tg.n_vertices, tg.writhe, tg.tait_number, m, e)
    return v, l2


def rel_err(a, b):
    a, b = complex(a), complex(b)
    return abs(a - b) / max(abs(b), 1e-300)


def close_log(l2a, pha, l2b, phb, tol):
    """Relative difference of two complex numbers given as (log2|z|, phase)."""
    dr = 2.0 ** (l2a - l2b)
    return abs(dr * np.exp(1j * (pha - phb)) - 1.0) <= tol
