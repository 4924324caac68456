"""CPU model of the device program that libkn's planner writes.

Test infrastructure: it reads a program image (kn_plan_image /
kn_batch_image) and executes it with numpy, following the semantics the HIP
engine implements: a FIFO ready queue seeded with the knots' first groups,
group chains, setup -> gather-GEMM steps with power-of-two exponents ->
final product, and tensors homed in a per-task LDS arena or the global arena.
It checks the host-side planner and image builder (tables, group order,
arena and LDS layout, bounds) on the CPU; the device engine itself is checked
against the oracle by the GPU parity tests.
"""

from __future__ import annotations

import math
from collections import deque

import numpy as np

HDR = np.dtype([
    ("magic", "<i4"), ("precision", "<i4"), ("n_tasks", "<i4"), ("n_knots", "<i4"),
    ("n_tensors", "<i4"), ("n_steps", "<i4"), ("n_vtx", "<i4"), ("n_medges", "<i4"),
    ("n_members", "<i4"), ("n_factors", "<i4"), ("n_strides", "<i4"), ("n_groups", "<i4"),
    ("n_edges", "<i4"), ("n_roots", "<i4"), ("lds_bytes", "<i4"), ("n_pins", "<i4"),
    ("n_wslots", "<i4"), ("n_outputs", "<i4"), ("sliced", "<i4"), ("n_consts", "<i4"),
    ("n_queue", "<i4"), ("n_zslice", "<i4"),
    ("o_tasks", "<i8"), ("o_groups", "<i8"), ("o_roots", "<i8"), ("o_knots", "<i8"),
    ("o_tensors", "<i8"), ("o_steps", "<i8"), ("o_vtx", "<i8"), ("o_vslot", "<i8"),
    ("o_medges", "<i8"), ("o_members", "<i8"), ("o_factors", "<i8"), ("o_strides", "<i8"),
    ("o_eps", "<i8"), ("o_comps", "<i8"), ("o_pins", "<i8"), ("o_consts", "<i8"),
    ("image_bytes", "<i8"),
    ("state_off", "<i8"),
    ("state_bytes", "<i8"), ("o_queue", "<i8"), ("o_pending", "<i8"), ("o_tstate", "<i8"),
    ("o_weights", "<i8"), ("o_mgrad", "<i8"), ("o_zslice", "<i8"), ("o_uslice", "<i8"),
    ("arena_off", "<i8"),
    ("arena_elems", "<i8"),
    ("workspace_bytes", "<i8"), ("guard_off", "<i8")], align=True)
TASK = np.dtype([(f, "<i4") for f in ("kind", "knot", "group", "first", "count", "flags",
                                      "state_lo", "state_len")], align=True)
GROUP = np.dtype([(f, "<i4") for f in ("knot", "first_task", "n_tasks", "next", "n_pred")],
                 align=True)
KNOT = np.dtype([("t_re", "<f8"), ("t_im", "<f8")] + [(f, "<i4") for f in (
    "q", "edge_off", "n_edges", "medge_off", "n_medges", "vtx_off", "n_vtx", "factor_off",
    "n_factors", "comp_off", "n_comps", "n_iso", "out_slot", "step_off", "n_steps", "grad",
    "slice", "n_slices", "n_slice_spins", "plan_slot", "slice_step", "group_off", "n_groups",
    "tensor_off", "n_tensors", "w_off", "const_off", "pad")], align=True)
TENSOR = np.dtype([("off", "<i8"), ("size", "<i4"), ("lds_off", "<i4")], align=True)
STEP = np.dtype([(f, "<i4") for f in ("a", "b", "c", "nb", "nm", "nn", "nk", "str", "ranks",
                                      "n_tiles", "tile", "home_a", "home_b", "home_c", "mode",
                                      "n_mb", "n_nb", "n_ks", "kseg", "partial", "lvl")],
                align=True)
VTX = np.dtype([(f, "<i4") for f in ("tensor", "n_slots", "slot_off", "keep_center", "adjoint",
                                    "comp", "adj_str", "pin_off", "n_pins")], align=True)
PAIR = np.dtype([("x", "<i4"), ("y", "<i4")], align=True)
FACTOR = np.dtype([("x", "<i4"), ("y", "<i4"), ("a", "<i4"), ("b", "<i4")], align=True)
TAB_CAP = 3072
STEP_SERIAL, STEP_TILES, STEP_GEMM, STEP_GEMM64 = 0, 1, 2, 3
GEMM_BLOCK = {STEP_GEMM: 32, STEP_GEMM64: 64}
GEMM_CHUNK = 16
# byte offset of the LDS tensor arena (program.h): gather tables (3072 int32),
# 64 step descriptors, 768 int32 shifts, 768 int64 exponents, 128 operand
# states of 16 bytes
LDS_ARENA = (((3072 * 4 + 64 * STEP.itemsize + 768 * 4 + 7) // 8 * 8 + 768 * 8 + 15) // 16 * 16
             + 128 * 16)
REDUCE_CHUNK = 8192
TASK_SERIAL, TASK_TILE, TASK_REDUCE = 0, 1, 2


class Image:
    def __init__(self, raw: bytes):
        self.raw = raw
        self.h = np.frombuffer(raw, HDR, 1)[0]
        h = self.h
        assert h["magic"] == 0x4B4E4732

        def arr(dt, off, n):
            if int(n) == 0:
                return np.zeros(0, dt)
            assert int(off) + int(n) * np.dtype(dt).itemsize <= len(raw), "array past the image"
            return np.frombuffer(raw, dt, int(n), int(off))

        self.tasks = arr(TASK, h["o_tasks"], h["n_tasks"])
        self.groups = arr(GROUP, h["o_groups"], h["n_groups"])
        self.roots = arr("<i4", h["o_roots"], h["n_roots"])
        self.knots = arr(KNOT, h["o_knots"], h["n_knots"])
        self.tensors = arr(TENSOR, h["o_tensors"], h["n_tensors"])
        self.steps = arr(STEP, h["o_steps"], h["n_steps"])
        self.vtx = arr(VTX, h["o_vtx"], h["n_vtx"])
        # slot lists are shared by the slices of a plan: the furthest slot used
        n_vslot = max([int(v["slot_off"]) + int(v["n_slots"]) for v in self.vtx] + [0])
        self.vslot = arr("<i4", h["o_vslot"], n_vslot)
        self.medges = arr(PAIR, h["o_medges"], h["n_medges"])
        self.members = arr("<i4", h["o_members"], h["n_members"])
        self.factors = arr(FACTOR, h["o_factors"], h["n_factors"])
        self.pins = arr(PAIR, h["o_pins"], h["n_pins"])
        self.strides = arr("<i4", h["o_strides"], h["n_strides"])
        self.eps = arr("<i1", h["o_eps"], h["n_edges"])
        c = arr("<f8", h["o_consts"], 2 * int(h["n_consts"]))
        self.consts = c[0::2] + 1j * c[1::2]
        n_comps = int(sum(int(k["n_comps"]) for k in self.knots))
        self.comps = arr("<i4", h["o_comps"], n_comps)


def run(raw: bytes, J=None, want_grad=False):
    """Execute the image; returns a list of (mantissa, exp2) per knot, and with
    want_grad also d log Z / d J per original edge (knot-global edge order)
    for the knots of gradient plans."""
    im = Image(raw)
    h = im.h
    es = 8 if h["precision"] else 16
    lds_cap = int(h["lds_bytes"]) // es
    arena = np.zeros(int(h["arena_elems"]), np.complex128)
    nt = int(h["n_tensors"])
    shift = [None] * nt
    exp2 = [0] * nt
    finished = np.zeros(nt, bool)   # producer finished (visible to later groups)
    weights = np.zeros(int(h["n_wslots"]), np.complex128)
    out = [None] * int(h["n_outputs"])
    zslice = {}
    grads = np.full(int(h["n_edges"]), np.nan, np.complex128)
    # a tensor dies after the last step that reads it (its consumer; in a
    # gradient plan forward tensors are read again by the reverse steps); the
    # component scalars of gradient plans and the adjoints of vertex tensors
    # are read after the last step and never die
    last_use = {}
    for si in range(int(h["n_steps"])):
        for op in (int(im.steps[si]["a"]), int(im.steps[si]["b"])):
            last_use[op] = si
    forever = set()
    for k in im.knots:
        if int(k["grad"]):
            forever.update(int(im.comps[int(k["comp_off"]) + i]) for i in range(int(k["n_comps"])))
    for v in im.vtx:
        if int(v["adjoint"]) >= 0:
            forever.add(int(v["adjoint"]))

    def dies_at(op, si):
        return op not in forever and last_use.get(op) == si

    # layout checks
    assert int(h["image_bytes"]) == len(raw)
    assert int(h["state_off"]) + int(h["state_bytes"]) <= int(h["arena_off"])
    assert int(h["arena_off"]) + int(h["arena_elems"]) * es <= int(h["workspace_bytes"])
    for t in range(nt):
        off, size = int(im.tensors[t]["off"]), int(im.tensors[t]["size"])
        lo = int(im.tensors[t]["lds_off"])
        assert 0 <= off and off + size <= int(h["arena_elems"])
        if lo >= 0:
            assert lo + size <= lds_cap, "LDS tensor beyond the LDS arena"
    for g in im.groups:
        assert 0 <= g["first_task"] and g["first_task"] + g["n_tasks"] <= h["n_tasks"]
        for t in range(int(g["first_task"]), int(g["first_task"] + g["n_tasks"])):
            assert im.tasks[t]["knot"] == g["knot"]

    # the LDS arena exists only while one serial task runs
    live_g, live_l = {}, {}
    split_pending = {}
    state = {"lds": None}

    def home(t):
        return int(im.tensors[t]["lds_off"])

    # the serial tasks of one group run at once on different workgroups: every
    # global-arena range each of them reads or writes, checked against the
    # others' when the group completes, and their outputs visible to other
    # tasks only after the whole group
    group_acc = {}
    group_made = {}

    def concurrent_group():
        g = int(im.tasks[cur_task[0]]["group"])
        multi = (int(im.tasks[cur_task[0]]["kind"]) == TASK_SERIAL
                 and int(im.groups[g]["n_tasks"]) > 1)
        return g if multi else None

    def record(write, off, size):
        g = concurrent_group()
        if g is not None:
            group_acc.setdefault(g, []).append((cur_task[0], write, off, size))

    def write_tensor(t, data, task_local):
        size = int(im.tensors[t]["size"])
        assert data.size == size
        lo = home(t)
        if lo >= 0:
            assert task_local, f"tensor {t} homed in LDS but written by a tile task"
            for u, (o2, s2) in list(live_l.items()):
                if u != t and o2 < lo + size and lo < o2 + s2:
                    raise AssertionError(f"LDS tensor {t} overwrites live LDS tensor {u}")
            state["lds"][lo:lo + size] = data
            live_l[t] = (lo, size)
        else:
            off = int(im.tensors[t]["off"])
            for u, (o2, s2) in list(live_g.items()):
                if u != t and o2 < off + size and off < o2 + s2:
                    raise AssertionError(f"tensor {t} overwrites live tensor {u}")
            arena[off:off + size] = data
            live_g[t] = (off, size)
            record(True, off, size)

    def read(t, local):
        size = int(im.tensors[t]["size"])
        lo = home(t)
        if lo >= 0:
            assert t in local, f"LDS tensor {t} read outside the task that made it"
            return state["lds"][lo:lo + size]
        assert t in local or finished[t], f"tensor {t} read before its producer finished"
        off = int(im.tensors[t]["off"])
        record(False, off, size)
        return arena[off:off + size]

    def sh(t):
        return 0 if shift[t] is None else shift[t]

    def table(strides, n, q):
        """Offsets of the n = q^r values of a spin group (first spin most significant)."""
        r = len(strides)
        assert q ** r == n
        idx = np.arange(n, dtype=np.int64)
        off = np.zeros(n, np.int64)
        for j in range(r - 1, -1, -1):
            off += (idx % q) * int(strides[j])
            idx //= q
        return off

    def step(si, local):
        s = im.steps[si]
        nb, nm, nn, nk = (int(s[f]) for f in ("nb", "nm", "nn", "nk"))
        q = int(im.knots[int(im.tasks[cur_task[0]]["knot"])]["q"])
        if not int(s["n_tiles"]):
            assert 2 * nb + nm + 2 * nk + nn <= TAB_CAP, "serial step tables exceed LDS staging"
        rk = [(int(s["ranks"]) >> sh) & 255 for sh in (0, 8, 16, 24)]
        rb, rm, rkk, rn = rk
        st0 = int(s["str"])
        sp = im.strides[st0:st0 + 2 * rb + rm + 2 * rkk + rn]
        tAb = table(sp[:rb], nb, q)
        tAm = table(sp[rb:rb + rm], nm, q)
        tAk = table(sp[rb + rm:rb + rm + rkk], nk, q)
        tBb = table(sp[rb + rm + rkk:2 * rb + rm + rkk], nb, q)
        tBk = table(sp[2 * rb + rm + rkk:2 * rb + rm + 2 * rkk], nk, q)
        tBn = table(sp[2 * rb + rm + 2 * rkk:], nn, q)
        a, b, c = int(s["a"]), int(s["b"]), int(s["c"])
        for t, hm in ((a, "home_a"), (b, "home_b"), (c, "home_c")):
            lo = home(t)
            want = -1 - lo if lo >= 0 else int(im.tensors[t]["off"])
            assert int(s[hm]) == want, "step descriptor home differs from the tensor's"
        A = read(a, local)
        B = read(b, local)
        assert int(tAb.max()) + int(tAm.max()) + int(tAk.max()) < A.size
        assert int(tBb.max()) + int(tBk.max()) + int(tBn.max()) < B.size
        assert min(int(x.min()) for x in (tAb, tAm, tAk, tBb, tBk, tBn)) >= 0
        outs = nb * nm * nn
        assert outs == int(im.tensors[c]["size"])
        mode, n_tiles, n_ks, kseg = (int(s[f]) for f in ("mode", "n_tiles", "n_ks", "kseg"))
        assert (mode == STEP_SERIAL) == (n_tiles == 0)
        if mode != STEP_SERIAL:
            assert n_ks >= 1 and kseg >= 1
            assert n_ks * kseg >= nk and (n_ks - 1) * kseg < nk, "split does not cover k"
            assert n_tiles % n_ks == 0
            base = n_tiles // n_ks
            if mode == STEP_TILES:
                tile = int(s["tile"])
                assert base * tile >= outs and (base - 1) * tile < outs
            else:
                assert mode in GEMM_BLOCK
                bm = GEMM_BLOCK[mode]
                # both staged operand chunks fit in the launch's LDS
                assert 2 * GEMM_CHUNK * (bm + 1) * es <= LDS_ARENA + int(h["lds_bytes"])
                n_mb, n_nb, per = int(s["n_mb"]), int(s["n_nb"]), int(s["tile"])
                assert per >= 1 and base == -(-nb * n_mb * n_nb // per)
                assert n_mb * bm >= nm and (n_mb - 1) * bm < nm
                assert n_nb * bm >= nn and (n_nb - 1) * bm < nn
        Am = A[tAb[:, None, None] + tAm[None, :, None] + tAk[None, None, :]]
        Bm = B[tBb[:, None, None] + tBk[None, :, None] + tBn[None, None, :]]
        scale = math.ldexp(1.0, -(sh(a) + sh(b)))
        if mode != STEP_SERIAL and n_ks > 1:
            # partial sums of each contracted range go to the partial buffer,
            # which must not touch a live tensor (operands, C or any other)
            off = int(s["partial"])
            assert off >= 0 and off + n_ks * outs <= int(h["arena_elems"])
            reserved = dict(live_g)
            reserved[c] = (int(im.tensors[c]["off"]), outs)
            for u, (o2, s2) in reserved.items():
                assert not (o2 < off + n_ks * outs and off < o2 + s2), \
                    f"partial buffer of step {si} overlaps live tensor {u}"
            parts = [np.matmul(Am[:, :, j * kseg:(j + 1) * kseg],
                               Bm[:, j * kseg:(j + 1) * kseg, :]).reshape(-1) * scale
                     for j in range(n_ks)]
            arena[off:off + n_ks * outs] = np.concatenate(parts)
            split_pending[si] = (off, n_ks, outs)
            return
        C = np.matmul(Am, Bm).reshape(-1) * scale
        if mode == STEP_SERIAL:
            return C  # the caller commits the level's results together
        finish_step(si, C, local, task_local=False)

    def commit_step(si, C, local, task_local=True):
        s = im.steps[si]
        a, b, c = int(s["a"]), int(s["b"]), int(s["c"])
        write_tensor(c, C, task_local=task_local)
        m = float(np.max(np.maximum(np.abs(C.real), np.abs(C.imag)))) if C.size else 0.0
        shift[c] = math.frexp(m)[1] if m > 0 else None
        exp2[c] = exp2[a] + exp2[b] + sh(a) + sh(b)
        local.add(c)

    def finish_step(si, C, local, task_local):
        commit_step(si, C, local, task_local)
        s = im.steps[si]
        for op in (int(s["a"]), int(s["b"])):
            if dies_at(op, si):
                live_g.pop(op, None)
            live_l.pop(op, None)

    def reduce(si, local):
        off, n_ks, outs = split_pending.pop(si)
        P = arena[off:off + n_ks * outs].reshape(n_ks, outs).copy()
        C = P[0].copy()
        for j in range(1, n_ks):
            C = C + P[j]
        finish_step(si, C, local, task_local=False)

    def mul(z, e, f):
        z = z * f
        m = max(abs(z.real), abs(z.imag))
        if m == 0 or not math.isfinite(m):
            return z, e
        s = math.frexp(m)[1]
        return complex(math.ldexp(z.real, -s), math.ldexp(z.imag, -s)), e + s

    def knot_gradient(k, local):
        """d log Z / d J per original edge, as the device computes it: for the
        merged edge in slot j of vertex tensor F_v, x_m * sum_i dS/dF_v[i]
        dF_v/dx_m[i] / S with S the component's scalar; spikes x/(x+q-1),
        loops 1."""
        q = int(k["q"])
        eo, mo = int(k["edge_off"]), int(k["medge_off"])
        ne, nm = int(h["n_edges"]), int(k["n_medges"])
        mg = np.full(nm, np.nan, np.complex128)
        for v in range(int(k["n_vtx"])):
            vd = im.vtx[int(k["vtx_off"]) + v]
            ns = int(vd["n_slots"])
            if int(vd["keep_center"]) < 0 or int(vd["adjoint"]) < 0 or ns == 0:
                continue
            adj_t = int(vd["adjoint"])
            fb = read(adj_t, local)
            root = int(im.comps[int(k["comp_off"]) + int(vd["comp"])])
            r = complex(read(root, local)[0])
            slots = [int(im.vslot[int(vd["slot_off"]) + j]) for j in range(ns)]
            xs = [weights[int(k["w_off"]) + int(k["n_edges"]) + m] for m in slots]
            qn = q ** ns
            kc = 1 if int(vd["keep_center"]) else 0
            astr = [int(x) for x in im.strides[int(vd["adj_str"]):int(vd["adj_str"]) + kc + ns]]
            assert sorted(astr) == [q ** r for r in range(kc + ns)], "adjoint strides"
            for j in range(ns):
                acc = 0j
                for i in range(fb.size):
                    rem = i
                    dig = [0] * ns
                    for l in range(ns - 1, -1, -1):
                        dig[l] = rem % q
                        rem //= q
                    off = sum(dig[l] * astr[kc + l] for l in range(ns)) + (rem * astr[0] if kc else 0)
                    a = rem if kc else dig[j]
                    if dig[j] != a:
                        continue
                    p = complex(fb[off])
                    for l in range(ns):
                        if l != j and dig[l] == a:
                            p *= xs[l]
                    acc += p
                assert math.isnan(mg[slots[j]].real), "merged edge absorbed twice"
                mg[slots[j]] = xs[j] * acc / r * 2.0 ** (exp2[adj_t] - exp2[root])
            assert fb.size == qn * (q if int(vd["keep_center"]) else 1)
        for i in range(int(k["n_factors"])):
            f = im.factors[int(k["factor_off"]) + i]
            if f["x"] == 1:
                x = weights[int(k["w_off"]) + int(k["n_edges"]) + int(f["y"])]
                mg[int(f["y"])] = x / (x + q - 1)
        for m in range(nm):
            me = im.medges[mo + m]
            for i in range(int(me["y"])):
                grads[eo + int(im.members[int(me["x"]) + i])] = mg[m]
        for i in range(int(k["n_factors"])):
            f = im.factors[int(k["factor_off"]) + i]
            if f["x"] == 0:
                grads[eo + int(f["y"])] = 1.0

    queue = deque(int(r) for r in im.roots)
    pending = {gi: int(g["n_pred"]) for gi, g in enumerate(im.groups)}
    # the slice each knot descriptor (a chain of slices) is running
    uslice = [int(k["slice"]) for k in im.knots]
    assert len(queue) == len(im.knots), "one root group per knot descriptor"
    assert all(im.groups[im.tasks[r]["group"]]["n_pred"] == 0 for r in queue)
    done_in_group = {}
    executed = 0
    cur_task = [0]
    while queue:
        ti = queue.popleft()
        cur_task[0] = ti
        task = im.tasks[ti]
        executed += 1
        k = im.knots[task["knot"]]
        q = int(k["q"])
        local = set()
        if task["kind"] == 0:
            # the task's state range covers exactly the tensors it produces
            lo, ln = int(task["state_lo"]), int(task["state_len"])
            made = set(range(lo, lo + ln))
            state["lds"] = np.zeros(max(lds_cap, 1), np.complex128)
            live_l.clear()
            if task["flags"] & 1:
                t = complex(k["t_re"], k["t_im"])
                eo, mo = int(k["edge_off"]), int(k["medge_off"])
                wo, wm = int(k["w_off"]), int(k["w_off"]) + int(k["n_edges"])
                for e in range(int(k["n_edges"])):
                    if J is not None:
                        x = np.exp(complex(J[2 * (eo + e)], J[2 * (eo + e) + 1]))
                    else:
                        x = -(t ** (-int(im.eps[eo + e])))
                    weights[wo + e] = x
                for m in range(int(k["n_medges"])):
                    me = im.medges[mo + m]
                    x = 1.0 + 0j
                    if int(me["y"]) < 0:  # derived edge: a constant of the plan
                        assert int(me["y"]) == -1
                        x = im.consts[int(k["const_off"]) + int(me["x"])]
                    for i in range(int(me["y"])):
                        x *= weights[wo + int(im.members[int(me["x"]) + i])]
                    weights[wm + m] = x
                sigma = [(uslice[int(task["knot"])] // q ** j) % q
                         for j in range(int(k["n_slice_spins"]))]
                for v in range(int(k["n_vtx"])):
                    vd = im.vtx[int(k["vtx_off"]) + v]
                    ns = int(vd["n_slots"])
                    assert ns <= 8
                    xs = [weights[wm + int(im.vslot[int(vd["slot_off"]) + j])] for j in range(ns)]
                    pins = [(int(im.pins[int(vd["pin_off"]) + j]["x"]),
                             int(im.pins[int(vd["pin_off"]) + j]["y"])) for j in range(int(vd["n_pins"]))]
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
                            for m, sj in pins:  # edges to fixed spins
                                if sigma[sj] == aa:
                                    p *= weights[wm + m]
                            acc += p
                        data[i] = acc
                    write_tensor(int(vd["tensor"]), data, task_local=True)
                    shift[int(vd["tensor"])] = 0
                    exp2[int(vd["tensor"])] = 0
                    local.add(int(vd["tensor"]))
            # adjacent steps of equal level run concurrently on the device:
            # every output is computed from operands that are all still live,
            # outputs must not overlap them, and operands die after the level
            first, count = int(task["first"]), int(task["count"])
            i = first
            while i < first + count:
                j = i + 1
                while j < first + count and int(im.steps[j]["lvl"]) == int(im.steps[i]["lvl"]):
                    j += 1
                assert all(int(im.steps[u]["lvl"]) >= 1 for u in range(i, j))
                made_here = {int(im.steps[u]["c"]) for u in range(i, j)}
                for u in range(i, j):
                    assert int(im.steps[u]["a"]) not in made_here, "step reads its own level"
                    assert int(im.steps[u]["b"]) not in made_here, "step reads its own level"
                results = [step(u, local) for u in range(i, j)]
                for u, C in zip(range(i, j), results):
                    commit_step(u, C, local)
                for u in range(i, j):
                    for op in (int(im.steps[u]["a"]), int(im.steps[u]["b"])):
                        if dies_at(op, u):
                            live_g.pop(op, None)
                        live_l.pop(op, None)
                i = j
            if task["flags"] & 2:
                z, e = 1 + 0j, 0
                for i in range(int(k["n_comps"])):
                    t = int(im.comps[int(k["comp_off"]) + i])
                    e += exp2[t]
                    z, e = mul(z, e, read(t, local)[0])
                    live_l.pop(t, None)
                    if t not in forever:
                        live_g.pop(t, None)
                wo, wm = int(k["w_off"]), int(k["w_off"]) + int(k["n_edges"])
                sigma = [(uslice[int(task["knot"])] // q ** j) % q
                         for j in range(int(k["n_slice_spins"]))]
                for i in range(int(k["n_factors"])):
                    f = im.factors[int(k["factor_off"]) + i]
                    if f["x"] == 0:
                        x = weights[wo + int(f["y"])]
                    elif f["x"] == 1:
                        x = weights[wm + int(f["y"])] + (q - 1)
                    elif f["x"] == 3:  # constant of the plan (series reduction)
                        x = im.consts[int(k["const_off"]) + int(f["y"])]
                    else:  # edge between two fixed spins
                        x = weights[wm + int(f["y"])] if sigma[int(f["a"])] == sigma[int(f["b"])] else 1.0
                    z, e = mul(z, e, x)
                for i in range(int(k["n_iso"])):
                    z, e = mul(z, e, q)
                if int(k["n_slices"]) > 1:
                    s_ = uslice[int(task["knot"])]
                    assert int(k["out_slot"]) + s_ not in zslice, "slice computed twice"
                    zslice[int(k["out_slot"]) + s_] = (z, e, int(k["plan_slot"]))
                else:
                    out[int(k["out_slot"])] = (z, e)
                if int(k["grad"]):
                    knot_gradient(k, local)
            assert local == made, "state range differs from the tensors the task produced"
            # LDS contents die with the task: nothing homed there may outlive it
            assert not live_l, f"LDS tensors {list(live_l)} still live when their task ends"
            g_ = concurrent_group()
            for t in local:
                if home(t) < 0:
                    if g_ is None:
                        finished[t] = True
                    else:
                        group_made.setdefault(g_, []).append(t)
        elif task["kind"] == TASK_TILE:
            sd = im.steps[int(task["first"])]
            assert int(sd["mode"]) in (STEP_TILES, STEP_GEMM, STEP_GEMM64)
            assert 0 <= int(task["count"]) < int(sd["n_tiles"])
            if task["count"] == 0:
                step(int(task["first"]), local)  # the model computes the whole step once
        else:
            assert task["kind"] == TASK_REDUCE
            si = int(task["first"])
            sd = im.steps[si]
            outs = int(sd["nb"]) * int(sd["nm"]) * int(sd["nn"])
            assert int(sd["n_ks"]) > 1
            assert int(im.groups[int(task["group"])]["n_tasks"]) == -(-outs // REDUCE_CHUNK)
            if task["count"] == 0:
                assert si in split_pending, "reduce before the step's tiles"
                reduce(si, local)
        # the final task of a slice whose chain has more: reset the unit and
        # start its next slice
        ki = int(task["knot"])
        if (task["kind"] == TASK_SERIAL and task["flags"] & 2 and int(k["n_slices"]) > 1
                and uslice[ki] + int(k["slice_step"]) < int(k["n_slices"])):
            uslice[ki] += int(k["slice_step"])
            g0, ng = int(k["group_off"]), int(k["n_groups"])
            assert int(im.groups[g0 + ng - 1]["next"]) == -1
            for gi in range(g0, g0 + ng):
                pending[gi] = int(im.groups[gi]["n_pred"])
                done_in_group.pop(gi, None)
            t0, nt_ = int(k["tensor_off"]), int(k["n_tensors"])
            for t in range(t0, t0 + nt_):
                assert t not in live_g, f"tensor {t} still live at the end of a slice"
                finished[t] = False
                shift[t] = None
                exp2[t] = 0
            G = im.groups[g0]
            queue.extend(range(int(G["first_task"]), int(G["first_task"] + G["n_tasks"])))
            continue
        # group completion -> enqueue the next group
        g = int(task["group"])
        done_in_group[g] = done_in_group.get(g, 0) + 1
        if done_in_group[g] == int(im.groups[g]["n_tasks"]):
            acc = group_acc.pop(g, [])
            for x in range(len(acc)):
                for y in range(x + 1, len(acc)):
                    (t1, w1, o1, s1), (t2, w2, o2, s2) = acc[x], acc[y]
                    if t1 != t2 and (w1 or w2) and o1 < o2 + s2 and o2 < o1 + s1:
                        raise AssertionError(f"concurrent tasks {t1} and {t2} of group {g} "
                                             "touch overlapping arena ranges")
            for t in group_made.pop(g, []):
                finished[t] = True
            if task["kind"] != TASK_SERIAL:
                sd = im.steps[int(task["first"])]
                if task["kind"] == TASK_REDUCE or int(sd["n_ks"]) == 1:
                    finished[int(sd["c"])] = True
                else:
                    nxt_g = im.groups[int(im.groups[g]["next"])]
                    assert im.tasks[int(nxt_g["first_task"])]["kind"] == TASK_REDUCE
            nxt = int(im.groups[g]["next"])
            if nxt >= 0:
                pending[nxt] -= int(im.groups[g]["n_tasks"])
                assert pending[nxt] == 0
                G = im.groups[nxt]
                queue.extend(range(int(G["first_task"]), int(G["first_task"] + G["n_tasks"])))
    assert executed == int(h["n_queue"]), "some tasks were never enqueued"
    assert all(int(h["n_queue"]) >= 0 for _ in [0])
    for k in im.knots:  # every slice of every sliced plan computed once
        if int(k["n_slices"]) > 1 and int(k["slice"]) == 0:
            for s_ in range(int(k["n_slices"])):
                assert int(k["out_slot"]) + s_ in zslice, "slice never computed"
    # sliced plans: Z is the sum over slices (exact complex sum, aligned exponents)
    acc = {}
    for z, e, slot in zslice.values():
        acc.setdefault(slot, []).append((z, e))
    for slot, terms in acc.items():
        emax = max(e for z, e in terms if z != 0) if any(z != 0 for z, e in terms) else 0
        tot = sum(z * 2.0 ** (e - emax) for z, e in terms)
        m = max(abs(tot.real), abs(tot.imag))
        sh = math.frexp(m)[1] if m > 0 else 0
        out[slot] = (complex(math.ldexp(tot.real, -sh), math.ldexp(tot.imag, -sh)), emax + sh)
    if want_grad:
        return out, grads
    return out
