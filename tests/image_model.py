"""CPU model of the device program that libkn's planner writes.

Test infrastructure: it reads a plan's image bytes (kn_plan_image) and
executes the task list in order with numpy, following the semantics the HIP
engine implements (setup -> gather-GEMM steps with power-of-two exponents ->
final product).  It checks the host-side planner and image builder (tables,
dependencies, arena layout) on the CPU; the device engine itself is checked
against the oracle by the GPU parity tests.
"""

from __future__ import annotations

import math

import numpy as np

HDR = np.dtype([
    ("magic", "<i4"), ("precision", "<i4"), ("n_tasks", "<i4"), ("n_knots", "<i4"),
    ("n_tensors", "<i4"), ("n_steps", "<i4"), ("n_vtx", "<i4"), ("n_medges", "<i4"),
    ("n_members", "<i4"), ("n_factors", "<i4"), ("n_tables", "<i4"), ("n_deps", "<i4"),
    ("n_edges", "<i4"), ("tile", "<i4"),
    ("o_tasks", "<i8"), ("o_deps", "<i8"), ("o_knots", "<i8"), ("o_tensors", "<i8"),
    ("o_steps", "<i8"), ("o_vtx", "<i8"), ("o_vslot", "<i8"), ("o_medges", "<i8"),
    ("o_members", "<i8"), ("o_factors", "<i8"), ("o_tables", "<i8"), ("o_eps", "<i8"),
    ("o_comps", "<i8"), ("image_bytes", "<i8"), ("state_off", "<i8"), ("state_bytes", "<i8"),
    ("o_tstate", "<i8"), ("o_weights", "<i8"), ("arena_off", "<i8"), ("arena_elems", "<i8"),
    ("workspace_bytes", "<i8")], align=True)
TASK = np.dtype([(f, "<i4") for f in ("kind", "knot", "first", "count", "flags", "dep_off",
                                      "n_deps", "sig_off", "n_sig")], align=True)
KNOT = np.dtype([("t_re", "<f8"), ("t_im", "<f8")] + [(f, "<i4") for f in (
    "q", "edge_off", "n_edges", "medge_off", "n_medges", "vtx_off", "n_vtx", "factor_off",
    "n_factors", "comp_off", "n_comps", "n_iso", "out_slot", "step_off", "n_steps")], align=True)
TENSOR = np.dtype([("off", "<i8"), ("size", "<i4"), ("target", "<i4")], align=True)
STEP = np.dtype([(f, "<i4") for f in ("a", "b", "c", "nb", "nm", "nn", "nk", "tab", "n_tiles",
                                      "tile")], align=True)
VTX = np.dtype([(f, "<i4") for f in ("tensor", "n_slots", "slot_off", "keep_center")], align=True)
PAIR = np.dtype([("x", "<i4"), ("y", "<i4")], align=True)


class Image:
    def __init__(self, raw: bytes):
        self.raw = raw
        self.h = np.frombuffer(raw, HDR, 1)[0]
        h = self.h
        assert h["magic"] == 0x4B4E4731

        def arr(dt, off, n):
            return np.frombuffer(raw, dt, int(n), int(off))

        self.tasks = arr(TASK, h["o_tasks"], h["n_tasks"])
        self.deps = arr("<i4", h["o_deps"], h["n_deps"])
        self.knots = arr(KNOT, h["o_knots"], h["n_knots"])
        self.tensors = arr(TENSOR, h["o_tensors"], h["n_tensors"])
        self.steps = arr(STEP, h["o_steps"], h["n_steps"])
        self.vtx = arr(VTX, h["o_vtx"], h["n_vtx"])
        n_vslot = int(sum(int(v["n_slots"]) for v in self.vtx))
        self.vslot = arr("<i4", h["o_vslot"], n_vslot)
        self.medges = arr(PAIR, h["o_medges"], h["n_medges"])
        self.members = arr("<i4", h["o_members"], h["n_members"])
        self.factors = arr(PAIR, h["o_factors"], h["n_factors"])
        self.tables = arr("<i4", h["o_tables"], h["n_tables"])
        self.eps = arr("<i1", h["o_eps"], h["n_edges"])
        n_comps = int(sum(int(k["n_comps"]) for k in self.knots))
        self.comps = arr("<i4", h["o_comps"], n_comps)


def run(raw: bytes, J=None):
    """Execute the image; returns a list of (mantissa, exp2) per knot."""
    im = Image(raw)
    h = im.h
    arena = np.zeros(int(h["arena_elems"]), np.complex128)
    nt = int(h["n_tensors"])
    shift = [None] * nt
    exp2 = [0] * nt
    done = np.zeros(nt, np.int64)
    weights = np.zeros(int(h["n_edges"]) + int(h["n_medges"]), np.complex128)
    out = [None] * int(h["n_knots"])
    # arena regions in use: check that no live tensor is overwritten
    live = {}

    for t in range(nt):
        assert 0 <= int(im.tensors[t]["off"]) and \
            int(im.tensors[t]["off"]) + int(im.tensors[t]["size"]) <= int(h["arena_elems"])
    assert int(h["arena_off"]) + int(h["arena_elems"]) * (8 if h["precision"] else 16) \
        <= int(h["workspace_bytes"])
    assert int(h["state_off"]) + int(h["state_bytes"]) <= int(h["arena_off"])
    assert int(h["image_bytes"]) == len(raw)

    def write_tensor(t, data):
        off, size = int(im.tensors[t]["off"]), int(im.tensors[t]["size"])
        for u, (o2, s2) in list(live.items()):
            if u != t and o2 < off + size and off < o2 + s2:
                raise AssertionError(f"tensor {t} overwrites live tensor {u}")
        arena[off:off + size] = data
        live[t] = (off, size)

    def read(t):
        off, size = int(im.tensors[t]["off"]), int(im.tensors[t]["size"])
        return arena[off:off + size]

    def sh(t):
        return 0 if shift[t] is None else shift[t]

    local = set()  # tensors produced by the running task (visible to it at once)

    def step(si):
        s = im.steps[si]
        nb, nm, nn, nk = (int(s[f]) for f in ("nb", "nm", "nn", "nk"))
        tab = int(s["tab"])
        tAb = im.tables[tab:tab + nb]
        tAm = im.tables[tab + nb:tab + nb + nm]
        tAk = im.tables[tab + nb + nm:tab + nb + nm + nk]
        tBb = im.tables[tab + nb + nm + nk:tab + 2 * nb + nm + nk]
        tBk = im.tables[tab + 2 * nb + nm + nk:tab + 2 * nb + nm + 2 * nk]
        tBn = im.tables[tab + 2 * nb + nm + 2 * nk:tab + 2 * nb + nm + 2 * nk + nn]
        a, b, c = int(s["a"]), int(s["b"]), int(s["c"])
        for t in (a, b):
            assert t in local or done[t] >= im.tensors[t]["target"], \
                f"step {si} reads unfinished tensor {t}"
        A = read(a)
        B = read(b)
        # every gather stays inside its operand
        assert int(tAb.max()) + int(tAm.max()) + int(tAk.max()) < A.size
        assert int(tBb.max()) + int(tBk.max()) + int(tBn.max()) < B.size
        assert min(int(tAb.min()), int(tAm.min()), int(tAk.min()), int(tBb.min()),
                   int(tBk.min()), int(tBn.min())) >= 0
        assert nb * nm * nn == int(im.tensors[c]["size"])
        if int(s["n_tiles"]):
            assert int(s["n_tiles"]) * int(s["tile"]) >= nb * nm * nn
            assert int(s["n_tiles"]) == int(im.tensors[c]["target"])
        Am = A[tAb[:, None, None] + tAm[None, :, None] + tAk[None, None, :]]
        Bm = B[tBb[:, None, None] + tBk[None, :, None] + tBn[None, None, :]]
        C = np.matmul(Am, Bm).reshape(-1) * math.ldexp(1.0, -(sh(a) + sh(b)))
        write_tensor(c, C)
        m = float(np.max(np.maximum(np.abs(C.real), np.abs(C.imag)))) if C.size else 0.0
        shift[c] = math.frexp(m)[1] if m > 0 else None
        exp2[c] = exp2[a] + exp2[b] + sh(a) + sh(b)
        # operands are consumed exactly once
        live.pop(a, None)
        live.pop(b, None)

    for ti, task in enumerate(im.tasks):
        local.clear()
        for d in im.deps[task["dep_off"]:task["dep_off"] + task["n_deps"]]:
            assert done[d] >= im.tensors[d]["target"], f"task {ti} waits on unfinished tensor {d}"
        k = im.knots[task["knot"]]
        q = int(k["q"])
        if task["kind"] == 0:
            if task["flags"] & 1:
                t = complex(k["t_re"], k["t_im"])
                eo, mo = int(k["edge_off"]), int(k["medge_off"])
                for e in range(int(k["n_edges"])):
                    if J is not None:
                        x = np.exp(complex(J[2 * (eo + e)], J[2 * (eo + e) + 1]))
                    else:
                        x = -(t ** (-int(im.eps[eo + e])))
                    weights[eo + e] = x
                for m in range(int(k["n_medges"])):
                    me = im.medges[mo + m]
                    x = 1.0 + 0j
                    for i in range(int(me["y"])):
                        x *= weights[eo + int(im.members[int(me["x"]) + i])]
                    weights[int(h["n_edges"]) + mo + m] = x
                for v in range(int(k["n_vtx"])):
                    vd = im.vtx[int(k["vtx_off"]) + v]
                    ns = int(vd["n_slots"])
                    xs = [weights[int(h["n_edges"]) + mo + int(im.vslot[int(vd["slot_off"]) + j])]
                          for j in range(ns)]
                    size = int(im.tensors[vd["tensor"]]["size"])
                    data = np.zeros(size, np.complex128)
                    for i in range(size):
                        rem = i
                        dig = [0] * ns
                        for j in range(ns - 1, -1, -1):
                            dig[j] = rem % q
                            rem //= q
                        centres = [rem] if vd["keep_center"] else range(q)
                        acc = 0j
                        for aa in centres:
                            p = 1 + 0j
                            for j in range(ns):
                                if dig[j] == aa:
                                    p *= xs[j]
                            acc += p
                        data[i] = acc
                    write_tensor(int(vd["tensor"]), data)
                    shift[int(vd["tensor"])] = 0
                    exp2[int(vd["tensor"])] = 0
                    local.add(int(vd["tensor"]))
            for si in range(int(task["first"]), int(task["first"]) + int(task["count"])):
                step(si)
                local.add(int(im.steps[si]["c"]))
            if task["flags"] & 2:
                z, e = 1 + 0j, 0

                def mul(z, e, f):
                    z = z * f
                    m = max(abs(z.real), abs(z.imag))
                    if m == 0 or not math.isfinite(m):
                        return z, e
                    s = math.frexp(m)[1]
                    return complex(math.ldexp(z.real, -s), math.ldexp(z.imag, -s)), e + s

                for i in range(int(k["n_comps"])):
                    t = int(im.comps[int(k["comp_off"]) + i])
                    assert t in local or done[t] >= im.tensors[t]["target"]
                    e += exp2[t]
                    z, e = mul(z, e, read(t)[0])
                eo, mo = int(k["edge_off"]), int(k["medge_off"])
                for i in range(int(k["n_factors"])):
                    f = im.factors[int(k["factor_off"]) + i]
                    if f["x"] == 0:
                        x = weights[eo + int(f["y"])]
                    else:
                        x = weights[int(h["n_edges"]) + mo + int(f["y"])] + (q - 1)
                    z, e = mul(z, e, x)
                for i in range(int(k["n_iso"])):
                    z, e = mul(z, e, q)
                out[int(k["out_slot"])] = (z, e)
        else:
            si = int(task["first"])
            s = im.steps[si]
            if task["count"] == 0:
                step(si)
        # publish: every signalled tensor's counter goes up by one
        sig = im.deps[task["sig_off"]:task["sig_off"] + task["n_sig"]]
        for t in sig:
            done[t] += 1
            assert done[t] <= im.tensors[t]["target"]
    return out
