"""ctypes binding of libtmfg (argument marshalling only; every step runs in the HIP kernels).

Tensors passed in must be CUDA (ROCm) tensors on the plan's device, contiguous, of the
dtype named in the C header include/tmfg.h. PyTorch is used for device memory and
streams only. If libtmfg.so has not been built the first call raises at once: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtmfg.so")

STATUS = {
    0: "TMFG_OK", 1: "TMFG_E_INVALID", 2: "TMFG_E_SIZE", 3: "TMFG_E_NONFINITE",
    4: "TMFG_E_ASYMMETRIC", 5: "TMFG_E_DEGENERATE", 6: "TMFG_E_NOMEM", 7: "TMFG_E_HIP",
    8: "TMFG_E_INTERNAL", 9: "TMFG_PENDING",
}
PENDING = 9
NO_VALIDATE = 1 << 0
TIMING = 1 << 1
BATCH_NO_GRAPH = 1 << 2
BATCH_AUTOTUNE = 1 << 3
IDX32 = 1 << 4               # declared by the C header; not provided (TMFG_E_INVALID)
STATS = 1 << 5               # plans: record the insertion loop's counters (Plan.stats)
RULE_PAPER = 1 << 8
RULE_CORR = 1 << 9
PREFIX_SHIFT = 16


def rule_corr_prefix(p: int) -> int:
    """Plan/batch flags for corr-tmfg (Algorithm 1) with prefix size p (1..16)."""
    return RULE_CORR | (int(p) << PREFIX_SHIFT)


SERVER_FIFO = 1 << 0
SERVER_RULE_PAPER = 1 << 1

# Every symbol the header declares, with its ctypes signature.
_P = ctypes.c_void_p
_I = ctypes.c_int32
SIGNATURES = {
    "tmfg_plan_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, ctypes.c_uint32]),
    "tmfg_plan_destroy": (_I, [_P]),
    "tmfg_footprint_bytes": (ctypes.c_size_t, [_I, _I, ctypes.c_uint32]),
    "tmfg_build": (_I, [_P, _P, _P]),
    "tmfg_build_noalloc": (_I, [_P, ctypes.c_uint32, _P]),
    "tmfg_plan_phase_ms": (_I, [_P, ctypes.POINTER(ctypes.c_float)]),
    "tmfg_plan_stats": (_I, [_P, ctypes.POINTER(_I)]),
    "tmfg_correlation": (_I, [_P, _P, _I, _I, _P, _P, _P]),
    "tmfg_sort_rows": (_I, [_P, _P, _I, _P, _P, ctypes.c_int64, _P]),
    "tmfg_seed": (_I, [_P, _P, _I, _P, _P, _P]),
    "tmfg_face_sweep": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _P]),
    "tmfg_batch_create": (_I, [ctypes.POINTER(_P), _P, _I, ctypes.c_uint32]),
    "tmfg_batch_run": (_I, [_P, _P]),
    "tmfg_batch_destroy": (_I, [_P]),
    "tmfg_batch_footprint_bytes": (ctypes.c_size_t, [_P, _I, ctypes.c_uint32]),
    "tmfg_batch_config": (_I, [_P, ctypes.POINTER(_I)]),
    "tmfg_batch_set_config": (_I, [_P, ctypes.POINTER(_I)]),
    "tmfg_build_batch": (_I, [_P, _P, _I, _P]),
    "tmfg_server_create": (_I, [ctypes.POINTER(_P), _P]),
    "tmfg_server_submit": (_I, [_P, _P, _I, _I, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "tmfg_server_poll": (_I, [_P, ctypes.c_int64, _I, _P]),
    "tmfg_server_stats": (_I, [_P, _P, _I]),
    "tmfg_server_destroy": (_I, [_P]),
    "tmfg_server_now_ns": (ctypes.c_int64, []),
    "tmfg_dbht": (_I, [_I, _P, _P, _P, _P, _I, _I, _P, _P, _P, _P]),
    "tmfg_status_string": (ctypes.c_char_p, [_I]),
    "tmfg_last_hip_error": (ctypes.c_int, []),
    "tmfg_probe_load_latency": (_I, [ctypes.c_int64, _I, _I, ctypes.POINTER(ctypes.c_double)]),
}


class TmfgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = int(code)
        name = STATUS.get(self.code, str(code))
        msg = f"{where}: {name}"
        if self.code == 7:
            msg += f" (hipError {_lib().tmfg_last_hip_error()})"
        super().__init__(msg)


class Job(ctypes.Structure):
    _fields_ = [
        ("n", _I), ("L", _I), ("X", _P), ("W", _P), ("W_out", _P), ("order", _P),
        ("edges", _P), ("steps", _P), ("step_gain", _P), ("faces", _P), ("status", _P),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("host_budget", ctypes.c_size_t), ("max_batch", _I),
                ("n_streams", _I), ("n_max", _I), ("L_max", _I), ("flags", ctypes.c_uint32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("order", _P), ("edges", _P), ("steps", _P), ("step_gain", _P), ("faces", _P),
                ("n", _I), ("status", _I), ("arrival_ns", ctypes.c_int64), ("dispatch_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64)]


class ServerReport(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("dispatches", ctypes.c_int64),
                ("waiting", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("builds_per_s", ctypes.c_double),
                ("mean_batch", ctypes.c_double)]


_LIB: Optional[ctypes.CDLL] = None


def _lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2408_09399_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def lib() -> ctypes.CDLL:
    return _lib()


def _check(code: int, where: str) -> None:
    if code != 0:
        raise TmfgError(code, where)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _need(t, dtype, name: str):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _shape(t, name: str, ndim: int, cols: Optional[int] = None, square: bool = False):
    """Host-side shape check, made before anything reaches the device: the kernels read
    exactly the extents the header states, so a tensor of another shape is refused here."""
    if t is None:
        return
    shape = tuple(t.shape)
    if len(shape) != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions, got shape {shape}")
    if square and shape[0] != shape[1]:
        raise ValueError(f"{name} must be square, got shape {shape}")
    if cols is not None and shape[1] != cols:
        raise ValueError(f"{name} must have {cols} columns, got shape {shape}")


def footprint_bytes(n_max: int, L_max: int, flags: int = 0) -> int:
    return int(_lib().tmfg_footprint_bytes(n_max, L_max, flags))


class Plan:
    """A plan owns the scratch for builds with n <= n_max and L <= L_max; tmfg_build_batch on
    it accepts up to max_jobs jobs."""

    def __init__(self, n_max: int, L_max: int = 2, flags: int = 0, max_jobs: int = 4096):
        h = ctypes.c_void_p()
        _check(_lib().tmfg_plan_create(ctypes.byref(h), n_max, L_max, max_jobs, flags), "tmfg_plan_create")
        self._h = h
        self.n_max, self.L_max, self.flags, self.max_jobs = n_max, L_max, flags, max_jobs

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib().tmfg_plan_destroy(self._h), "tmfg_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def phase_ms(self) -> Tuple[float, ...]:
        out = (ctypes.c_float * 5)()
        _check(_lib().tmfg_plan_phase_ms(self.handle, out), "tmfg_plan_phase_ms")
        return tuple(float(x) for x in out)

    def stats(self) -> Tuple[int, ...]:
        """The insertion loop's counters of the last build (tmfg_plan_stats); the plan must have
        been made with STATS, else TmfgError (TMFG_E_INVALID)."""
        out = (ctypes.c_int32 * 32)()
        _check(_lib().tmfg_plan_stats(self.handle, out), "tmfg_plan_stats")
        return tuple(int(x) for x in out)


@dataclasses.dataclass
class Result:
    order: "object"
    edges: "object"
    steps: "object"
    step_gain: "object"
    faces: "object"
    status: "object"
    W: "object" = None

    def to_numpy(self) -> dict:
        d = {k: getattr(self, k).cpu().numpy() for k in ("order", "edges", "steps", "step_gain", "faces")}
        d["status"] = int(self.status.item())
        if self.W is not None:
            d["W"] = self.W.cpu().numpy()
        return d


def alloc_result(n: int, device, keep_w: bool = False) -> Result:
    import torch
    i32 = dict(dtype=torch.int32, device=device)
    return Result(
        order=torch.empty(n, **i32),
        edges=torch.empty((3 * n - 6, 2), **i32),
        steps=torch.empty((max(n - 4, 0), 4), **i32),
        step_gain=torch.empty(max(n - 4, 0), dtype=torch.float32, device=device),
        faces=torch.empty((2 * n - 4, 3), **i32),
        status=torch.full((1,), -1, **i32),
        W=torch.empty((n, n), dtype=torch.float32, device=device) if keep_w else None,
    )


def make_job(n: int, L: int, X, W, res: Result) -> Job:
    j = Job()
    j.n, j.L = n, L
    j.X, j.W = _ptr(X), _ptr(W)
    j.W_out = _ptr(res.W)
    j.order, j.edges = _ptr(res.order), _ptr(res.edges)
    j.steps = _ptr(res.steps) if n > 4 else None
    j.step_gain = _ptr(res.step_gain) if n > 4 else None
    j.faces, j.status = _ptr(res.faces), _ptr(res.status)
    return j


def build(X=None, W=None, plan: Optional[Plan] = None, stream=None, keep_w: bool = False,
          out: Optional[Result] = None, flags: int = 0) -> Result:
    """Enqueue one TMFG build (from series X (n, L) or similarity W (n, n), float32).
    `flags` are the plan flags (e.g. RULE_PAPER) of the plan made when none is given."""
    import torch
    if (X is None) == (W is None):
        raise ValueError("give exactly one of X and W")
    _shape(X, "X", 2)
    _shape(W, "W", 2, square=True)
    src = _need(X if X is not None else W, torch.float32, "X" if X is not None else "W")
    n = src.shape[0]
    L = src.shape[1] if X is not None else 0
    if plan is None:
        plan = Plan(n, max(L, 2), flags)
    if out is not None and (out.order.numel() != n or (keep_w and out.W is None)):
        raise ValueError(f"out was allocated for n = {out.order.numel()}, not {n}")
    res = out if out is not None else alloc_result(n, src.device, keep_w)
    job = make_job(n, L, X, W, res)
    _check(_lib().tmfg_build(plan.handle, ctypes.byref(job), _stream(stream)), "tmfg_build")
    res._plan = plan          # keep the scratch alive until the caller drops the result
    return res


def correlation(X, plan: Optional[Plan] = None, stream=None):
    """Pearson similarity (float32, MFMA). Returns (W, status tensor)."""
    import torch
    _shape(X, "X", 2)
    X = _need(X, torch.float32, "X")
    n, L = X.shape
    if plan is None:
        plan = Plan(n, L)
    W = torch.empty((n, n), dtype=torch.float32, device=X.device)
    status = torch.full((1,), -1, dtype=torch.int32, device=X.device)
    _check(_lib().tmfg_correlation(plan.handle, _ptr(X), n, L, _ptr(W), _ptr(status), _stream(stream)),
           "tmfg_correlation")
    return W, status


def sort_stride(n: int) -> int:
    return (max(n - 1, 1) + 7) // 8 * 8


def sort_rows(W, plan: Optional[Plan] = None, stream=None, with_values: bool = False):
    """Per-vertex order as an (n, ld) int16 tensor holding uint16 ids (first n-1 valid),
    plus the (n, ld) float32 similarities in that order when with_values is set."""
    import torch
    _shape(W, "W", 2, square=True)
    W = _need(W, torch.float32, "W")
    n = W.shape[0]
    if plan is None:
        plan = Plan(n, 2)
    ld = sort_stride(n)
    idx = torch.empty((n, ld), dtype=torch.int16, device=W.device)
    vals = torch.empty((n, ld), dtype=torch.float32, device=W.device) if with_values else None
    _check(_lib().tmfg_sort_rows(plan.handle, _ptr(W), n, _ptr(idx), _ptr(vals), ld, _stream(stream)),
           "tmfg_sort_rows")
    return (idx, vals) if with_values else idx


def seed(W, plan: Optional[Plan] = None, stream=None):
    """Seed scores (float64) and the four seed vertices."""
    import torch
    _shape(W, "W", 2, square=True)
    W = _need(W, torch.float32, "W")
    n = W.shape[0]
    if plan is None:
        plan = Plan(n, 2)
    scores = torch.empty(n, dtype=torch.float64, device=W.device)
    s4 = torch.empty(4, dtype=torch.int32, device=W.device)
    _check(_lib().tmfg_seed(plan.handle, _ptr(W), n, _ptr(scores), _ptr(s4), _stream(stream)), "tmfg_seed")
    return scores, s4


def face_sweep(W, faces, inserted_words, plan: Optional[Plan] = None, stream=None):
    """Exact best vertex per face by a full sweep. faces: (F, 3) int32; inserted: int32 words."""
    import torch
    _shape(W, "W", 2, square=True)
    _shape(faces, "faces", 2, cols=3)
    n = W.shape[0]
    if inserted_words is None or inserted_words.dim() != 1 or inserted_words.numel() < (n + 31) // 32:
        raise ValueError(f"inserted must be a 1-D tensor of at least {(n + 31) // 32} words")
    W = _need(W, torch.float32, "W")
    faces = _need(faces, torch.int32, "faces")
    inserted_words = _need(inserted_words, torch.int32, "inserted")
    if plan is None:
        plan = Plan(n, 2)
    F = faces.shape[0]
    bu = torch.empty(F, dtype=torch.int32, device=W.device)
    bg = torch.empty(F, dtype=torch.float32, device=W.device)
    _check(_lib().tmfg_face_sweep(plan.handle, _ptr(W), n, _ptr(faces), F, _ptr(inserted_words),
                                  _ptr(bu), _ptr(bg), _stream(stream)), "tmfg_face_sweep")
    return bu, bg


class Batch:
    """Many independent builds prepared once and replayed as one graph.

    `inputs` is a list of (kind, tensor) with kind "X" (series, (n, L)) or "W"
    (similarity, (n, n)), float32 device tensors that stay alive with the batch; their
    contents may change between runs. Results are allocated here, one Result per input.
    """

    def __init__(self, inputs, keep_w: bool = False, flags: int = 0):
        import torch
        self.inputs = list(inputs)
        self.results = []
        jobs = (Job * len(self.inputs))()
        for i, (kind, t) in enumerate(self.inputs):
            if kind not in ("X", "W"):
                raise ValueError(f"input {i}: kind must be 'X' or 'W', got {kind!r}")
            _shape(t, f"input {i} ({kind})", 2, square=kind == "W")
            t = _need(t, torch.float32, kind)
            n = t.shape[0]
            res = alloc_result(n, t.device, keep_w)
            self.results.append(res)
            X, W = (t, None) if kind == "X" else (None, t)
            jobs[i] = make_job(n, t.shape[1] if kind == "X" else 0, X, W, res)
        self._jobs = jobs
        h = ctypes.c_void_p()
        _check(_lib().tmfg_batch_create(ctypes.byref(h), ctypes.cast(jobs, ctypes.c_void_p), len(self.inputs),
                                        flags), "tmfg_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(_lib().tmfg_batch_run(self._h, _stream(stream)), "tmfg_batch_run")
        return self.results

    def config(self) -> dict:
        """The launch configuration in use (see tmfg_batch_config)."""
        out = (_I * 16)()
        _check(_lib().tmfg_batch_config(self._h, out), "tmfg_batch_config")
        v = list(out)
        return {"sort_config": v[0:8], "sort_rows_per_wg": v[8], "loop_workgroups": v[9],
                "tune_trials": v[10], "tune_ms": v[11], "walk_rounds": v[12],
                "gemm_tile": v[13:15], "from_cache": bool(v[15])}

    def set_config(self, cfg: dict) -> None:
        """Apply a launch configuration given as config() returns it (tmfg_batch_set_config);
        raises on a value out of range."""
        v = [0] * 16
        v[0:8] = cfg["sort_config"]
        v[8] = cfg["sort_rows_per_wg"]
        v[9] = cfg["loop_workgroups"]
        v[12] = cfg["walk_rounds"]
        v[13:15] = cfg["gemm_tile"]
        _check(_lib().tmfg_batch_set_config(self._h, (_I * 16)(*v)), "tmfg_batch_set_config")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib().tmfg_batch_destroy(self._h), "tmfg_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request server over host memory (tmfg_server_*): submit numpy series, poll results.

    The scheduler runs in the library's own thread on the device current at creation.
    """

    def __init__(self, hbm_budget: int, host_budget: int, max_batch: int = 512, n_streams: int = 2,
                 n_max: int = 8192, L_max: int = 1024, flags: int = 0):
        cfg = ServerConfig(hbm_budget, host_budget, max_batch, n_streams, n_max, L_max, flags)
        h = ctypes.c_void_p()
        self._sizes = {}
        _check(_lib().tmfg_server_create(ctypes.byref(h), ctypes.cast(ctypes.pointer(cfg), ctypes.c_void_p)),
               "tmfg_server_create")
        self._h = h

    @staticmethod
    def now_ns() -> int:
        return int(_lib().tmfg_server_now_ns())

    def submit(self, X, arrival_ns: int = 0) -> int:
        """Queue a build of the (n, L) float32 series X (host memory, copied at once)."""
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float32)
        _shape(X, "X", 2)
        n, L = X.shape
        t = ctypes.c_int64()
        _check(_lib().tmfg_server_submit(self._h, X.ctypes.data, n, L, int(arrival_ns), ctypes.byref(t)),
               "tmfg_server_submit")
        self._sizes[t.value] = n
        return t.value

    def poll(self, ticket: int, wait_ms: int = -1):
        """None while the request is pending; else its outputs, build status and times."""
        import numpy as np
        n = self._sizes[ticket]
        out = {"order": np.empty(n, np.int32), "edges": np.empty((3 * n - 6, 2), np.int32),
               "steps": np.empty((max(n - 4, 0), 4), np.int32), "step_gain": np.empty(max(n - 4, 0), np.float32),
               "faces": np.empty((2 * n - 4, 3), np.int32)}
        r = ServerResult(*(out[k].ctypes.data if out[k].size else None
                           for k in ("order", "edges", "steps", "step_gain", "faces")))
        code = _lib().tmfg_server_poll(self._h, int(ticket), int(wait_ms), ctypes.byref(r))
        if code == PENDING:
            return None
        _check(code, "tmfg_server_poll")
        del self._sizes[ticket]
        out.update(n=r.n, status=r.status, arrival_ns=r.arrival_ns, dispatch_ns=r.dispatch_ns, done_ns=r.done_ns)
        return out

    def stats(self, reset: bool = False) -> dict:
        rep = ServerReport()
        _check(_lib().tmfg_server_stats(self._h, ctypes.byref(rep), int(reset)), "tmfg_server_stats")
        return {k: getattr(rep, k) for k, _ in ServerReport._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib().tmfg_server_destroy(self._h), "tmfg_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dbht(W, order, edges, steps, k: int, n_threads: int = 0) -> dict:
    """DBHT clustering of a finished TMFG on the host (tmfg_dbht). Inputs are numpy arrays
    or tensors (copied to host memory); returns labels, linkage, group and bubble."""
    import numpy as np

    def host(a, dtype):
        if hasattr(a, "detach"):
            a = a.detach().cpu().numpy()
        return np.ascontiguousarray(np.asarray(a), dtype=dtype)

    Wh = host(W, np.float32)
    _shape(Wh, "W", 2, square=True)
    n = Wh.shape[0]
    order_h, edges_h = host(order, np.int32).ravel(), host(edges, np.int32).reshape(-1, 2)
    steps_h = host(steps, np.int32).reshape(-1, 4) if n > 4 else np.zeros((0, 4), np.int32)
    # the C call reads exactly these extents
    for name, a, rows in (("order", order_h, n), ("edges", edges_h, 3 * n - 6), ("steps", steps_h, max(n - 4, 0))):
        if a.shape[0] != rows:
            raise ValueError(f"{name} must have {rows} rows for n = {n}, got {a.shape[0]}")
    labels = np.empty(n, np.int32)
    linkage = np.empty((max(n - 1, 0), 4), np.float64)
    group = np.empty(n, np.int32)
    bubble = np.empty(n, np.int32)
    p = lambda a: a.ctypes.data if a.size else None
    _check(_lib().tmfg_dbht(n, p(Wh), p(order_h), p(edges_h), p(steps_h), int(k), int(n_threads), p(labels),
                            p(linkage), p(group), p(bubble)), "tmfg_dbht")
    return {"labels": labels, "linkage": linkage, "group": group, "bubble": bubble}


def load_latency_ns(bytes_: int, lanes: int = 64, steps: int = 20000) -> float:
    """Nanoseconds per dependent trip to memory from one wave (tmfg_probe_load_latency)."""
    out = ctypes.c_double()
    _check(_lib().tmfg_probe_load_latency(int(bytes_), int(lanes), int(steps), ctypes.byref(out)),
           "tmfg_probe_load_latency")
    return float(out.value)
