"""Write the stored oracle values of a named workload (tests/golden/).

Calls only the oracle (``oracle/``) and the seeded diagram generator: for
every knot of the workload, Z(q) of Eqs. 2-3 by the oracle's variable
elimination (complex128 with power-of-two rescaling) and V = A(q) Z of
Eq. 4, stored as mantissa/exponent pairs so that no value overflows.

    python tests/golden/make_oracle_values.py mixed 0
"""

from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import diagram, jones, potts  # noqa: E402
from paper_1807_02119_amd import gen  # noqa: E402


def path_of(workload: str, seed: int) -> str:
    return os.path.join(HERE, f"oracle_{workload}_seed{seed}.json")


def main():
    workload = sys.argv[1] if len(sys.argv) > 1 else "mixed"
    seed = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    rows = []
    t0 = time.perf_counter()
    for i, (d, q) in enumerate(gen.config_knots(workload, seed)):
        tg = diagram.tait_graph(d.pd, d.signs if d.n == 1 else None)
        x = potts.jones_weights(tg.eps, jones.t_of_q(q))
        m, e = potts.partition_function(tg.n_vertices, tg.edges, x, q)
        v, l2 = jones.jones_value(q, tg.n_vertices, tg.writhe, tg.tait_number, m, e)
        rows.append({"index": i, "label": d.label, "crossings": d.n, "q": q,
                     "z_re": m.real, "z_im": m.imag, "z_exp2": int(e),
                     "v_log2_abs": l2, "v_arg": math.atan2(v.imag, v.real) if v != 0 else 0.0})
        print(f"{d.label} n={d.n} q={q} log2|Z|={math.log2(abs(m)) + e:.3f}", flush=True)
    out = {"workload": workload, "seed": seed,
           "source": "oracle/potts.py partition_function (Eqs. 2-3), oracle/jones.py jones_value "
                     "(Eq. 4), written by tests/golden/make_oracle_values.py",
           "seconds": time.perf_counter() - t0, "knots": rows}
    with open(path_of(workload, seed), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path_of(workload, seed)}")


if __name__ == "__main__":
    main()
