"""Jones variable t(q), prefactor A(q) and V_K(t(q)) = A(q) Z(q).

Test infrastructure (see ``oracle/__init__``).

* Eq. 1: t(q) = (q + sqrt(q) sqrt(q-4) - 2) / 2, principal square roots, so
  for q < 4 the value lies on the upper unit circle (t(3) = e^{i pi/3}).
* Eq. 4: V = A(q) Z(q) with
  A(q) = (-t^{1/2} - t^{-1/2})^{-n_v-1} (-t^{3/4})^{w} t^{tau/4}.
  All fractional powers are taken as integer powers of the single principal
  fourth root r = exp(Log(t)/4): t^{1/2} = r^2, t^{3/4} = r^3, t^{tau/4} = r^tau.
"""

from __future__ import annotations

import cmath
import math


def t_of_q(q: int) -> complex:
    """Eq. 1 with principal square roots."""
    q = float(q)
    return (q + cmath.sqrt(q) * cmath.sqrt(q - 4.0) - 2.0) / 2.0


def fourth_root(q: int) -> complex:
    return cmath.exp(cmath.log(t_of_q(q)) / 4.0)


def log_prefactor(q: int, n_v: int, writhe: int, tau: int) -> complex:
    """Natural log of A(q) (Eq. 4), as a complex number (imaginary part = phase).

    Integer powers of complex numbers are summed as multiples of logarithms; the
    branch of each logarithm does not matter because every exponent is an
    integer.
    """
    r = fourth_root(q)
    base1 = -(r * r) - 1.0 / (r * r)
    base2 = -(r ** 3)
    return ((-n_v - 1) * cmath.log(base1) + writhe * cmath.log(base2)
            + tau * cmath.log(r))


def jones_value(q: int, n_v: int, writhe: int, tau: int, z_mant: complex, z_exp2: int):
    """V = A(q) Z with Z = z_mant * 2**z_exp2.

    Returns ``(V, log2|V|)``; V is inf-free only when |V| fits a double.
    """
    la = log_prefactor(q, n_v, writhe, tau)
    if z_mant == 0:
        return 0j, -math.inf
    lz = cmath.log(z_mant) + z_exp2 * math.log(2.0)
    lv = la + lz
    log2_abs = lv.real / math.log(2.0)
    ph = lv.imag
    mag = math.pow(2.0, log2_abs) if log2_abs < 1023 else math.inf
    return complex(mag * math.cos(ph), mag * math.sin(ph)), log2_abs

