"""Python binding of libkn (ctypes).  Argument marshalling only: every step of
the evaluation runs in the C++ planner and the HIP kernels of libkn.so.

PyTorch supplies device memory (workspaces, outputs, couplings) and streams.
The names mirror the C ABI in ``include/kn.h``.
"""

from __future__ import annotations

import cmath
import ctypes
import math
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# KN_LIBRARY selects another build of the same library (the sanitized one
# that the CPU tests can be run against, see build.py)
LIB_PATH = os.environ.get("KN_LIBRARY") or os.path.join(_HERE, "libkn.so")

KN_OK = 0
STATUS = {0: "KN_OK", -1: "KN_E_INVALID", -2: "KN_E_NOMEM", -3: "KN_E_BUDGET",
          -4: "KN_E_DEVICE", -5: "KN_E_NUMERIC", -6: "KN_E_UNSUPPORTED"}


class KnError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


N_BUCKETS = 5  # KN_N_BUCKETS: intermediate sizes <= 2^8, 2^12, 2^16, 2^20, larger
BUCKET_KNOBS = ("tile_macs_log2", "tile_outs_log2", "gemm64_pct", "gemm_tasks_log2")


class BucketOpts(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in BUCKET_KNOBS]


class PlanOpts(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("simplify", ctypes.c_int32), ("jones_only", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_uint64), ("tile_outputs", ctypes.c_int32),
                ("big_step_macs_log2", ctypes.c_int32), ("paper_stats", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("gradient", ctypes.c_int32),
                ("tile_macs_log2", ctypes.c_int32), ("slice_log2_budget", ctypes.c_int32),
                ("split_serial_log2", ctypes.c_int32), ("gemm_tasks_log2", ctypes.c_int32),
                ("gemm64_pct", ctypes.c_int32), ("big_step_outs_log2", ctypes.c_int32),
                ("tile_outs_log2", ctypes.c_int32), ("bucket", BucketOpts * N_BUCKETS),
                ("order_trials", ctypes.c_int32), ("fork_serial_log2", ctypes.c_int32),
                ("split_min_log2", ctypes.c_int32)]


def plan_opts(strategy=3, precision=0, simplify=None, jones_only=True, mem_budget_bytes=0,
              tile_outputs=0, big_step_macs_log2=0, paper_stats=False, lds_bytes=0,
              gradient=False, tile_macs_log2=0, slice_log2_budget=0, split_serial_log2=0,
              gemm_tasks_log2=0, gemm64_pct=0, big_step_outs_log2=0, tile_outs_log2=0,
              buckets=None, order_trials=0, fork_serial_log2=0, split_min_log2=0):
    """kn_plan_opts from keyword arguments (0 = the library default).
    ``buckets``: {bucket index: {knob: value}} overrides of the tile-shape knobs
    (BUCKET_KNOBS) per intermediate-size bucket (keys may be strings)."""
    if simplify is None:
        simplify = 1 if (gradient or not jones_only) else 3
    o = PlanOpts()
    for name, v in (("strategy", strategy), ("precision", precision), ("simplify", simplify),
                    ("jones_only", 1 if jones_only else 0), ("mem_budget_bytes", mem_budget_bytes),
                    ("tile_outputs", tile_outputs), ("big_step_macs_log2", big_step_macs_log2),
                    ("paper_stats", 1 if paper_stats else 0), ("lds_bytes", lds_bytes),
                    ("gradient", 1 if gradient else 0), ("tile_macs_log2", tile_macs_log2),
                    ("slice_log2_budget", slice_log2_budget),
                    ("split_serial_log2", split_serial_log2), ("gemm_tasks_log2", gemm_tasks_log2),
                    ("gemm64_pct", gemm64_pct), ("big_step_outs_log2", big_step_outs_log2),
                    ("tile_outs_log2", tile_outs_log2), ("order_trials", order_trials),
                    ("fork_serial_log2", fork_serial_log2), ("split_min_log2", split_min_log2)):
        setattr(o, name, int(v))
    for b, knobs in (buckets or {}).items():
        for name, v in knobs.items():
            if name not in BUCKET_KNOBS:
                raise ValueError(f"unknown bucket knob {name}")
            setattr(o.bucket[int(b)], name, int(v))
    return o


class PlanStats(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("n_vertex_tensors", ctypes.c_int32),
                ("log2_max_entries", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64),
                ("image_bytes", ctypes.c_uint64), ("delta_h_paper", ctypes.c_int32),
                ("n_edges_simplified", ctypes.c_int32), ("n_vertices_simplified", ctypes.c_int32),
                ("n_tasks", ctypes.c_int32), ("n_components", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("slice_chains", ctypes.c_int32), ("n_recompute_steps", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("image_bytes", ctypes.c_uint64),
                ("n_tasks", ctypes.c_int32), ("n_knots", ctypes.c_int32),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("total_edges", ctypes.c_int64), ("grid", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Scalar(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double), ("exp2", ctypes.c_int64)]


_lib = None
_lock = threading.Lock()

P = ctypes.c_void_p
I32 = ctypes.c_int32
PI32 = ctypes.POINTER(ctypes.c_int32)
PI8 = ctypes.POINTER(ctypes.c_int8)
PD = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "kn_build_tait": (I32, [I32, PI32, PI8, I32, I32, ctypes.POINTER(P)]),
    "kn_tait_info": (I32, [P, PI32, PI32, PI32, PI32]),
    "kn_tait_edges": (I32, [P, PI32, PI8]),
    "kn_tait_free": (None, [P]),
    "kn_plan_create": (I32, [P, I32, ctypes.POINTER(PlanOpts), ctypes.POINTER(P)]),
    "kn_plan_info": (I32, [P, ctypes.POINTER(PlanStats)]),
    "kn_plan_steps": (I32, [P, PI32]),
    "kn_plan_image": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]),
    "kn_plan_free": (None, [P]),
    "kn_contract": (I32, [P, P, P, ctypes.c_size_t, P, P]),
    "kn_contract_noalloc": (I32, [P, P, P, P]),
    "kn_backward_workspace": (I32, [P, ctypes.POINTER(ctypes.c_uint64)]),
    "kn_contract_backward": (I32, [P, P, P, ctypes.c_size_t, P, P, P]),
    "kn_jones": (I32, [I32, P, ctypes.POINTER(Scalar), PD, PD, PD, PD]),
    "kn_jones_variable": (I32, [I32, PD, PD]),
    "kn_batch_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(P)]),
    "kn_free_many": (None, [I32, ctypes.POINTER(P), ctypes.POINTER(P)]),
    "kn_batch_info": (I32, [P, ctypes.POINTER(BatchStats)]),
    "kn_batch_edge_offset": (I32, [P, I32, ctypes.POINTER(ctypes.c_int64)]),
    "kn_batch_upload": (I32, [P, P, ctypes.c_size_t, P]),
    "kn_batch_contract": (I32, [P, P, P, ctypes.c_size_t, P, P]),
    "kn_batch_contract_backward": (I32, [P, P, P, ctypes.c_size_t, P, P, P]),
    "kn_batch_set_grid": (I32, [P, I32]),
    "kn_batch_image": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]),
    "kn_batch_set_trace": (I32, [P, P, ctypes.c_size_t]),
    "kn_batch_free": (None, [P]),
    "kn_plan_many": (I32, [I32, PI32, PI32, PI8, PI32, ctypes.POINTER(PlanOpts), I32,
                           ctypes.POINTER(P), ctypes.POINTER(P), PI32]),
    "kn_jones_many": (I32, [I32, PI32, ctypes.POINTER(P), ctypes.POINTER(Scalar), PD, PD, PD]),
    "kn_workspace_status": (I32, [P, P, PI32]),
    "kn_device_checks": (I32, []),
    "kn_image_check": (I32, [P, ctypes.c_size_t, PI32]),
    "kn_status_string": (ctypes.c_char_p, [I32]),
    "kn_version": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libkn.so (building it first if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build
                build.build()
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _check(code, where):
    if code != KN_OK:
        raise KnError(code, where)


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(PI32)


class Tait:
    """Signed Tait graph of a PD code (kn_build_tait)."""

    def __init__(self, pd, signs=None, outer_arc: int = -1, outer_side: int = 0):
        L = lib()
        pd = np.ascontiguousarray(np.asarray(pd, dtype=np.int32).reshape(-1))
        n = pd.size // 4
        sg = None
        if signs is not None:
            sg = np.ascontiguousarray(np.asarray(signs, dtype=np.int8))
        h = P()
        rc = L.kn_build_tait(n, pd.ctypes.data_as(PI32) if n else None,
                             sg.ctypes.data_as(PI8) if sg is not None else None,
                             outer_arc, outer_side, ctypes.byref(h))
        _check(rc, "kn_build_tait")
        self._h = h
        self._info = None

    def _get_info(self):
        if self._info is None:
            nv, ne, w, t = I32(), I32(), I32(), I32()
            _check(lib().kn_tait_info(self._h, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(w),
                                      ctypes.byref(t)), "kn_tait_info")
            self._info = (nv.value, ne.value, w.value, t.value)
        return self._info

    # graph facts are read from the library on first use (kn_tait_info)
    n_vertices = property(lambda self: self._get_info()[0])
    n_edges = property(lambda self: self._get_info()[1])
    writhe = property(lambda self: self._get_info()[2])
    tait_number = property(lambda self: self._get_info()[3])

    def edges(self):
        uv = np.zeros(2 * self.n_edges, np.int32)
        eps = np.zeros(self.n_edges, np.int8)
        _check(lib().kn_tait_edges(self._h, uv.ctypes.data_as(PI32), eps.ctypes.data_as(PI8)),
               "kn_tait_edges")
        return uv.reshape(-1, 2), eps

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and getattr(self, "_owner", None) is None:
            _lib.kn_tait_free(h)
        self._h = None


class Plan:
    """Contraction plan for one knot at one q (kn_plan_create)."""

    def __init__(self, tait: Tait, q: int, allow_budget=False, **opts):
        """``opts``: the keyword arguments of plan_opts (kn_plan_opts fields)."""
        L = lib()
        o = plan_opts(**opts)
        gradient = bool(o.gradient)
        precision = o.precision
        jones_only = bool(o.jones_only)
        h = P()
        rc = L.kn_plan_create(tait._h, q, ctypes.byref(o), ctypes.byref(h))
        self._h = h if h.value else None
        self.status = rc
        if rc != KN_OK and not (allow_budget and rc == -3 and h.value):
            if h.value:
                L.kn_plan_free(h)
                self._h = None
            raise KnError(rc, "kn_plan_create")
        self.tait = tait
        self.q = q
        self.precision = precision
        self.jones_only = jones_only
        self.gradient = bool(gradient)
        self._stats = None

    @property
    def stats(self):
        """kn_plan_info as a dict (read on first use)."""
        if self._stats is None:
            st = PlanStats()
            _check(lib().kn_plan_info(self._h, ctypes.byref(st)), "kn_plan_info")
            self._stats = st.as_dict()
        return self._stats

    @property
    def workspace_bytes(self):
        return int(self.stats["workspace_bytes"])

    def steps(self):
        n = self.stats["n_steps"]
        ab = np.zeros(2 * max(n, 1), np.int32)
        _check(lib().kn_plan_steps(self._h, ab.ctypes.data_as(PI32)), "kn_plan_steps")
        return ab[:2 * n].reshape(-1, 2)

    def image(self) -> bytes:
        """Copy of the plan's device image (kn_plan_image)."""
        d, n = P(), ctypes.c_size_t()
        _check(lib().kn_plan_image(self._h, ctypes.byref(d), ctypes.byref(n)), "kn_plan_image")
        return ctypes.string_at(d, n.value) if n.value else b""

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and getattr(self, "_owner", None) is None:
            _lib.kn_plan_free(h)
        self._h = None


def _wrap_tait(h):
    t = Tait.__new__(Tait)
    t._h = h
    t._info = None
    return t


def _wrap_plan(h, tait, q, opts):
    p = Plan.__new__(Plan)
    p._h = h
    p.status = 0
    p.tait = tait
    p.q = q
    p.precision = opts.precision
    p.jones_only = bool(opts.jones_only)
    p.gradient = bool(opts.gradient)
    p._stats = None
    return p


class PlanSet:
    """Tait graphs and plans of many knots kept as two handle arrays (one
    Python object for the whole set, freed with one kn_free_many call).  For
    pipelines that plan thousands of knots per second; ``plan(i)`` and
    ``tait(i)`` give views of single members."""

    def __init__(self, taits, plans, qs, opts):
        self.n = len(plans)
        self._th = taits
        self._ph = plans
        self.q = qs
        self._opts = opts

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        return self.plan(i)

    def tait(self, i):
        t = _wrap_tait(P(self._th[i]))
        t._owner = self  # a view: the set frees it
        return t

    def plan(self, i):
        p = _wrap_plan(P(self._ph[i]), self.tait(i), int(self.q[i]), self._opts)
        p._owner = self
        return p

    def __del__(self):
        if getattr(self, "_ph", None) is not None and _lib is not None:
            _lib.kn_free_many(self.n, self._th, self._ph)
            self._ph = self._th = None


def plan_set(n_crossings, flat_pd, qs, n_threads=0, **opts):
    """kn_plan_many over knots given as one int32 crossing-count array and
    their PD codes concatenated in one flat int32 array (``opts``: the keyword
    arguments of plan_opts).  Returns a PlanSet."""
    L = lib()
    ncr = np.ascontiguousarray(n_crossings, np.int32)
    n = len(ncr)
    flat = np.ascontiguousarray(flat_pd, np.int32)
    if flat.size == 0:
        flat = np.zeros(4, np.int32)
    qa = np.ascontiguousarray(np.broadcast_to(np.asarray(qs, np.int32), (n,)))
    o = plan_opts(**opts)
    th = (P * n)()
    ph = (P * n)()
    stv = np.zeros(n, np.int32)
    rc = L.kn_plan_many(n, ncr.ctypes.data_as(PI32), flat.ctypes.data_as(PI32), None,
                        qa.ctypes.data_as(PI32), ctypes.byref(o), n_threads, th, ph,
                        stv.ctypes.data_as(PI32))
    ps = PlanSet(th, ph, qa, o)
    if rc != KN_OK:
        del ps
        raise KnError(rc, "kn_plan_many")
    return ps


def plan_many(pds, qs, n_threads=0, **opts):
    """Tait graphs and plans for many knots on the library's host thread pool
    (kn_plan_many).  ``pds``: list of int32 arrays (n_i, 4); ``opts``: the
    keyword arguments of plan_opts.  Returns (taits, plans)."""
    L = lib()
    n = len(pds)
    ncr = np.array([np.asarray(p).reshape(-1, 4).shape[0] for p in pds], np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(p, np.int32).reshape(-1) for p in pds])
                                if ncr.sum() else np.zeros(4, np.int32))
    qa = np.ascontiguousarray(np.broadcast_to(np.asarray(qs, np.int32), (n,)))
    o = plan_opts(**opts)
    th = (P * n)()
    ph = (P * n)()
    stv = np.zeros(n, np.int32)
    rc = L.kn_plan_many(n, ncr.ctypes.data_as(PI32), flat.ctypes.data_as(PI32), None,
                        qa.ctypes.data_as(PI32), ctypes.byref(o), n_threads, th, ph,
                        stv.ctypes.data_as(PI32))
    taits = [_wrap_tait(P(h)) if h else None for h in th]
    if rc != KN_OK:
        for h in ph:
            if h:
                L.kn_plan_free(P(h))
        raise KnError(rc, "kn_plan_many")
    plans = [_wrap_plan(P(h), t, int(q), o) for h, t, q in zip(ph, taits, qa)]
    return taits, plans


def jones_many(qs, taits, z):
    """kn_jones for many knots; z: (n, 3) float64 host array of kn_scalar;
    taits: a list of Tait objects or a PlanSet.  Returns (v complex array,
    log2|v|, arg v)."""
    n = len(taits)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(n, 3)
    qa = np.ascontiguousarray(np.broadcast_to(np.asarray(qs, np.int32), (n,)))
    th = taits._th if isinstance(taits, PlanSet) else (P * n)(*[t._h for t in taits])
    v = np.zeros(2 * n)
    l2 = np.zeros(n)
    ar = np.zeros(n)
    _check(lib().kn_jones_many(n, qa.ctypes.data_as(PI32), th,
                               z.ctypes.data_as(ctypes.POINTER(Scalar)),
                               v.ctypes.data_as(PD), l2.ctypes.data_as(PD), ar.ctypes.data_as(PD)),
           "kn_jones_many")
    return v[0::2] + 1j * v[1::2], l2, ar


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def scalars_from_device(z):
    """(n, 3) float64 device tensor of kn_scalar -> list of (complex mantissa, exp2)."""
    a = z.detach().cpu().numpy().reshape(-1, 3)
    ex = a.view(np.int64)[:, 2]
    return [(complex(a[i, 0], a[i, 1]), int(ex[i])) for i in range(a.shape[0])]


def alloc_scalars(n, device="cuda"):
    torch = _torch()
    return torch.empty((n, 3), dtype=torch.float64, device=device)


def alloc_workspace(nbytes, device="cuda"):
    torch = _torch()
    return torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)


def _aligned_ptr(ws):
    p = ws.data_ptr()
    return (p + 255) & ~255, ws.numel() - ((p + 255 & ~255) - p)


def _device_f64(t, n, what):
    """Pointer of a contiguous float64 GPU tensor of exactly n entries (a
    complex128 one counts as two float64 per entry); anything else raises
    ValueError before a pointer reaches the kernels."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what} must be a torch tensor, not {type(t).__name__}")
    if t.dtype == torch.complex128:
        t = torch.view_as_real(t)
    if t.dtype != torch.float64:
        raise ValueError(f"{what} must be float64 (or complex128), not {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{what} must be in GPU memory, not on {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what} must hold {n} float64 values, not {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _couplings(J, n_edges):
    """Device pointer of the couplings J (2 float64 per original edge), or None
    for the Jones couplings."""
    return None if J is None else _device_f64(J, 2 * n_edges, "J")


def _scalars(z, n):
    return _device_f64(z, 3 * n, "z")


def _workspace(ws):
    """Aligned pointer and usable bytes of a workspace tensor (the library
    itself rejects one that is too small, with KN_E_BUDGET)."""
    torch = _torch()
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous torch tensor in GPU memory")
    return _aligned_ptr(ws)


def contract(plan: Plan, J=None, workspace=None, stream=None, z=None):
    """Z of the plan's knot on the GPU (kn_contract).  Returns the (1, 3)
    float64 device tensor holding the kn_scalar; see scalars_from_device."""
    if workspace is None:
        workspace = alloc_workspace(plan.workspace_bytes)
    if z is None:
        z = alloc_scalars(1)
    ptr, nbytes = _workspace(workspace)
    jp = _couplings(J, plan.tait.n_edges)
    _scalars(z, 1)
    rc = lib().kn_contract(plan._h, jp, ctypes.c_void_p(ptr), nbytes, _stream_ptr(stream),
                           ctypes.c_void_p(z.data_ptr()))
    _check(rc, "kn_contract")
    return z


def contract_noalloc(plan: Plan, J=None, stream=None, z=None):
    """Z of the plan's knot with the library's own fixed device array as the
    workspace (kn_contract_noalloc): the call allocates no device memory.
    Calls that overlap on one device race.  Returns z."""
    if z is None:
        z = alloc_scalars(1)
    jp = _couplings(J, plan.tait.n_edges)
    rc = lib().kn_contract_noalloc(plan._h, jp, _stream_ptr(stream), _scalars(z, 1))
    _check(rc, "kn_contract_noalloc")
    return z


CHECK_CODES = {0: "ok", 1: "queue wait time limit", 2: "task record", 3: "tensor extent",
               4: "group shape", 5: "gather bound", 6: "table buffer", 7: "guard zone"}


def workspace_status(workspace, stream=None):
    """Error words of the last launch in a workspace tensor
    (kn_workspace_status): dict(code, name, task, step, info); code 0 = none."""
    ptr, _ = _workspace(workspace)
    st = (ctypes.c_int32 * 4)()
    _check(lib().kn_workspace_status(ctypes.c_void_p(ptr), _stream_ptr(stream), st),
           "kn_workspace_status")
    return dict(code=st[0], name=CHECK_CODES.get(st[0], str(st[0])), task=st[1], step=st[2],
                info=st[3])


def device_checks() -> bool:
    """True when the loaded library is the checking build."""
    return bool(lib().kn_device_checks())


def image_check(image: bytes):
    """Host validation of a device image (kn_image_check): the same dict as
    workspace_status (code 0 = the image passes)."""
    buf = np.frombuffer(image, dtype=np.uint8)
    al = np.empty((len(buf) + 15) // 8, dtype=np.int64)  # 8-byte aligned copy
    al.view(np.uint8)[:len(buf)] = buf
    st = (ctypes.c_int32 * 4)()
    _check(lib().kn_image_check(ctypes.c_void_p(al.ctypes.data), len(buf), st), "kn_image_check")
    return dict(code=st[0], name=CHECK_CODES.get(st[0], str(st[0])), task=st[1], step=st[2],
                info=st[3])


def backward_workspace_bytes(plan: Plan) -> int:
    v = ctypes.c_uint64()
    _check(lib().kn_backward_workspace(plan._h, ctypes.byref(v)), "kn_backward_workspace")
    return int(v.value)


def contract_backward(plan: Plan, J=None, workspace=None, stream=None, z=None, grad=None):
    """d log Z / d J_e for every original edge (kn_contract_backward).
    Returns (z, grad) device tensors; grad is (n_edges, 2) float64."""
    torch = _torch()
    if workspace is None:
        workspace = alloc_workspace(backward_workspace_bytes(plan))
    if z is None:
        z = alloc_scalars(1)
    if grad is None:
        grad = torch.empty((plan.tait.n_edges, 2), dtype=torch.float64, device="cuda")
    ptr, nbytes = _workspace(workspace)
    ne = plan.tait.n_edges
    jp = _couplings(J, ne)
    rc = lib().kn_contract_backward(plan._h, jp, ctypes.c_void_p(ptr), nbytes,
                                    _stream_ptr(stream), _scalars(z, 1),
                                    _device_f64(grad, 2 * ne, "grad"))
    _check(rc, "kn_contract_backward")
    return z, grad


def jones(q: int, tait: Tait, z_mant: complex, z_exp2: int):
    """V = A(q) Z (kn_jones).  Returns (V, log2|V|, arg V)."""
    s = Scalar(z_mant.real, z_mant.imag, z_exp2)
    vr, vi, l2, ar = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().kn_jones(q, tait._h, ctypes.byref(s), ctypes.byref(vr), ctypes.byref(vi),
                          ctypes.byref(l2), ctypes.byref(ar)), "kn_jones")
    return complex(vr.value, vi.value), l2.value, ar.value


def jones_variable(q: int) -> complex:
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().kn_jones_variable(q, ctypes.byref(a), ctypes.byref(b)), "kn_jones_variable")
    return complex(a.value, b.value)


class Batch:
    """Many plans contracted in one persistent launch (kn_batch_*)."""

    def __init__(self, plans):
        L = lib()
        if isinstance(plans, PlanSet):
            self.plans = plans  # kept alive with the batch
            arr, n = plans._ph, plans.n
        else:
            self.plans = list(plans)
            n = len(self.plans)
            arr = (P * n)(*[p._h for p in self.plans])
        h = P()
        _check(L.kn_batch_create(arr, n, ctypes.byref(h)), "kn_batch_create")
        self._h = h
        st = BatchStats()
        _check(L.kn_batch_info(h, ctypes.byref(st)), "kn_batch_info")
        self.stats = st.as_dict()
        self.workspace = None

    @property
    def workspace_bytes(self):
        return int(self.stats["workspace_bytes"])

    def edge_offset(self, i):
        v = ctypes.c_int64()
        _check(lib().kn_batch_edge_offset(self._h, i, ctypes.byref(v)), "kn_batch_edge_offset")
        return int(v.value)

    def image(self) -> bytes:
        d, n = P(), ctypes.c_size_t()
        _check(lib().kn_batch_image(self._h, ctypes.byref(d), ctypes.byref(n)), "kn_batch_image")
        return ctypes.string_at(d, n.value)

    def set_trace(self, trace=None):
        """Record per-task timing into ``trace`` (a uint8 device tensor of at
        least 64 * n_tasks bytes) on later launches; None switches it off."""
        if trace is None:
            _check(lib().kn_batch_set_trace(self._h, None, 0), "kn_batch_set_trace")
        else:
            _check(lib().kn_batch_set_trace(self._h, ctypes.c_void_p(trace.data_ptr()),
                                            trace.numel() * trace.element_size()),
                   "kn_batch_set_trace")
        self._trace = trace

    @staticmethod
    def decode_trace(raw: bytes):
        dt = np.dtype([("t_claim", "<i8"), ("t_start", "<i8"), ("t_end", "<i8"),
                       ("task", "<i4"), ("wg", "<i4"), ("ph", "<i8", (4,))])
        return np.frombuffer(raw, dt)

    def set_grid(self, grid: int):
        _check(lib().kn_batch_set_grid(self._h, grid), "kn_batch_set_grid")

    def upload(self, workspace=None, stream=None):
        if workspace is None:
            workspace = alloc_workspace(self.workspace_bytes)
        ptr, nbytes = _workspace(workspace)
        _check(lib().kn_batch_upload(self._h, ctypes.c_void_p(ptr), nbytes, _stream_ptr(stream)),
               "kn_batch_upload")
        self.workspace = workspace
        return workspace

    def contract(self, J=None, stream=None, z=None):
        if self.workspace is None:
            self.upload(stream=stream)
        if z is None:
            z = alloc_scalars(len(self.plans))
        ptr, nbytes = _workspace(self.workspace)
        jp = _couplings(J, int(self.stats["total_edges"]))
        _check(lib().kn_batch_contract(self._h, jp, ctypes.c_void_p(ptr), nbytes,
                                       _stream_ptr(stream), _scalars(z, len(self.plans))),
               "kn_batch_contract")
        return z

    def graph(self, z, J=None, grad=None):
        """Capture one launch of the batch (its clear kernel and persistent
        kernel; with ``grad`` also the gradient kernel) in a hipGraph through
        torch.cuda.CUDAGraph; ``g.replay()`` then re-runs the contraction into
        the same ``z`` (and ``grad``).  The batch must have been uploaded and
        launched once eagerly (kernel attributes are set on the first launch)."""
        torch = _torch()
        if self.workspace is None:
            raise RuntimeError("upload and run the batch once before capturing it")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s = torch.cuda.current_stream()
            if grad is None:
                self.contract(J, stream=s, z=z)
            else:
                self.contract_backward(J, stream=s, z=z, grad=grad)
        return g

    def contract_backward(self, J=None, stream=None, z=None, grad=None):
        """Z and d log Z / d J of every knot (kn_batch_contract_backward);
        grad: (total_edges, 2) float64, knot i's edges from edge_offset(i)."""
        torch = _torch()
        if self.workspace is None:
            self.upload(stream=stream)
        if z is None:
            z = alloc_scalars(len(self.plans))
        if grad is None:
            grad = torch.empty((max(1, int(self.stats["total_edges"])), 2), dtype=torch.float64,
                               device="cuda")
        ptr, nbytes = _workspace(self.workspace)
        ne = int(self.stats["total_edges"])
        jp = _couplings(J, ne)
        _check(lib().kn_batch_contract_backward(self._h, jp, ctypes.c_void_p(ptr), nbytes,
                                                _stream_ptr(stream), _scalars(z, len(self.plans)),
                                                _device_f64(grad, 2 * max(1, ne), "grad")),
               "kn_batch_contract_backward")
        return z, grad

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.kn_batch_free(h)
            self._h = None


def status_string(code: int) -> str:
    return lib().kn_status_string(code).decode()


def version() -> str:
    return lib().kn_version().decode()


def z_to_log(z_mant: complex, z_exp2: int):
    """(log2|Z|, arg Z) of a mantissa/exponent pair."""
    if z_mant == 0:
        return -math.inf, 0.0
    return math.log2(abs(z_mant)) + z_exp2, math.atan2(z_mant.imag, z_mant.real)


def _make_logz():
    torch = _torch()

    class LogZ(torch.autograd.Function):
        """log Z of one knot as a differentiable function of its complex edge
        couplings J (complex128, n_edges, on the GPU).  The forward launch runs
        the forward and reverse sweeps together (kn_contract_backward) and
        keeps d log Z / d J for the backward call."""

        @staticmethod
        def forward(ctx, J, plan):
            if J.dtype != torch.complex128:
                raise ValueError(f"J must be complex128, not {J.dtype}")
            Jr = torch.view_as_real(J.detach().contiguous()).reshape(-1)
            z, g = contract_backward(plan, Jr)
            (m, e), = scalars_from_device(z)
            ctx.save_for_backward(torch.view_as_complex(g))
            logz = cmath.log(m) + e * math.log(2.0)
            return torch.tensor(logz, dtype=torch.complex128, device=J.device)

        @staticmethod
        def backward(ctx, gout):
            dlogz, = ctx.saved_tensors
            # holomorphic function: vector-Jacobian product with conj(f')
            return gout * dlogz.conj(), None

    return LogZ


_LOGZ = None


def log_z(J, plan: Plan):
    """Differentiable log Z(J) for a gradient plan (torch.autograd)."""
    global _LOGZ
    if _LOGZ is None:
        _LOGZ = _make_logz()
    return _LOGZ.apply(J, plan)
