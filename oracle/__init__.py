"""CPU oracle for the Jones-polynomial evaluation of Meichanetzidis & Kourtis
(arXiv:1807.02119).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or runs
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_1807_02119_amd``); both read the same PD codes produced by the
seeded input generator ``paper_1807_02119_amd.gen``, which holds none of the
method's arithmetic.

Modules (each function cites the passage it follows):

* ``diagram``   -- PD code -> bicoloured regions -> signed Tait graph, twist
                   signs, writhe, Tait number (Sec. II).
* ``potts``     -- the PACI partition function Z(q) (Eqs. 2-3): complex128
                   variable elimination with power-of-two rescaling, a
                   brute-force spin sum, and the edge-coupling gradient.
* ``exact``     -- Z(q) by the same elimination in the ring Z[t]/(t^2-(q-2)t+1),
                   exact in Python integers.
* ``jones``     -- t(q) (Eq. 1), the prefactor A(q) and V = A Z (Eq. 4).
* ``kauffman``  -- an independent Kauffman-bracket state sum that never builds
                   a Tait graph (textbook definition of V_K).
* ``invariants``-- Goeritz-matrix invariants that fix V at q = 2, 3, 4 for
                   diagrams of any size.

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself (see ``tests/test_oracle_*.py``).
"""
