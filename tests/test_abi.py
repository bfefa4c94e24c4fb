"""The C ABI library loads without a GPU, exports every declared symbol, and rejects bad
arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2408_09399_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmfg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(tmfg_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_what_binding_wraps():
    assert declared_functions() == sorted(binding.SIGNATURES)


def test_library_exports_every_symbol():
    lib = binding.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = binding.lib()
    for code in range(10):
        assert b"unknown" not in lib.tmfg_status_string(code)
    assert b"unknown" in lib.tmfg_status_string(10)


def test_host_side_argument_errors():
    lib = binding.lib()
    h = ctypes.c_void_p()
    assert lib.tmfg_plan_create(None, 100, 10, 1, 0) == 1
    assert lib.tmfg_plan_create(ctypes.byref(h), 3, 10, 1, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 32769, 10, 1, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 1, 1, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, -1, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, 1, 1 << 10) == 1
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, 1, binding.IDX32) == 1     # declared, not provided
    # corr-tmfg keeps a 16-bit vertex per face in LDS: up to n = 20480
    assert lib.tmfg_plan_create(ctypes.byref(h), 20481, 10, 1, binding.rule_corr_prefix(4)) == 2
    # face-rule flags: corr-tmfg needs a prefix in [1, 16], and excludes the paper's heap rule
    # (a well-formed job with placeholder pointers: a bad rule is rejected before any HIP call,
    # a good one gets as far as the HIP runtime, which has no device here)
    jobs = (binding.Job * 1)()
    j = jobs[0]
    j.n, j.L = 10, 8
    j.X = j.order = j.edges = j.steps = j.step_gain = j.faces = j.status = 256
    pj = ctypes.cast(jobs, ctypes.c_void_p)
    for bad in (binding.RULE_CORR, binding.rule_corr_prefix(17), binding.rule_corr_prefix(255),
                binding.rule_corr_prefix(2) | binding.RULE_PAPER, 3 << binding.PREFIX_SHIFT):
        assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, 1, bad) == 1, hex(bad)
        assert lib.tmfg_batch_create(ctypes.byref(h), pj, 1, bad) == 1, hex(bad)
    import torch
    if torch.cuda.device_count() == 0:       # with a device this would build a real batch
        for good in (binding.rule_corr_prefix(1), binding.rule_corr_prefix(16), binding.RULE_PAPER):
            assert lib.tmfg_batch_create(ctypes.byref(h), pj, 1, good) != 1, hex(good)
    assert lib.tmfg_build(None, None, None) == 1
    assert lib.tmfg_correlation(None, None, 10, 10, None, None, None) == 1
    assert lib.tmfg_sort_rows(None, None, 10, None, None, 16, None) == 1
    assert lib.tmfg_seed(None, None, 10, None, None, None) == 1
    assert lib.tmfg_face_sweep(None, None, 10, None, 1, None, None, None, None) == 1
    assert lib.tmfg_plan_destroy(None) == 0
    assert lib.tmfg_plan_phase_ms(None, None) == 1
    assert lib.tmfg_plan_stats(None, None) == 1


def test_footprint_grows_quadratically():
    f1 = binding.footprint_bytes(5000, 512)
    f2 = binding.footprint_bytes(10000, 512)
    assert 3.5 < f2 / f1 < 4.5
    assert binding.footprint_bytes(3, 10) == 0


def test_server_host_side_argument_errors():
    lib = binding.lib()
    h = ctypes.c_void_p()
    cfg = binding.ServerConfig(1 << 20, 1 << 20, 16, 2, 100, 64)
    pc = ctypes.cast(ctypes.pointer(cfg), ctypes.c_void_p)
    assert lib.tmfg_server_create(None, pc) == 1
    assert lib.tmfg_server_create(ctypes.byref(h), None) == 1
    for field, bad, code in [("hbm_budget", 0, 1), ("host_budget", 0, 1), ("max_batch", 0, 1),
                             ("max_batch", 4097, 1), ("n_streams", 0, 1), ("n_streams", 9, 1),
                             ("n_max", 3, 2), ("n_max", 20481, 2), ("L_max", 1, 2), ("flags", 4, 1),
                             ("flags", binding.RULE_CORR, 1), ("flags", binding.rule_corr_prefix(20), 1),
                             ("flags", binding.SERVER_RULE_PAPER | binding.rule_corr_prefix(2), 1)]:
        c = binding.ServerConfig(1 << 20, 1 << 20, 16, 2, 100, 64)
        setattr(c, field, bad)
        assert lib.tmfg_server_create(ctypes.byref(h), ctypes.cast(ctypes.pointer(c), ctypes.c_void_p)) == code, field
    t = ctypes.c_int64()
    assert lib.tmfg_server_submit(None, None, 10, 10, 0, ctypes.byref(t)) == 1
    assert lib.tmfg_server_poll(None, 1, 0, None) == 1
    assert lib.tmfg_server_stats(None, None, 0) == 1
    assert lib.tmfg_server_destroy(None) == 0
    a = lib.tmfg_server_now_ns()
    b = lib.tmfg_server_now_ns()
    assert 0 < a <= b


def test_binding_refuses_wrong_shapes_before_the_device():
    """The Python layer checks every extent the C calls read, before any device work: the
    tensors here are host tensors, so a check made after the device check would fail with
    another message."""
    import numpy as np
    import torch
    import paper_2408_09399_amd as tm
    with pytest.raises(ValueError, match="square"):
        tm.build(W=torch.zeros(6, 7))
    with pytest.raises(ValueError, match="2 dimensions"):
        tm.build(X=torch.zeros(24))
    with pytest.raises(ValueError, match="square"):
        tm.sort_rows(torch.zeros(6, 5))
    with pytest.raises(ValueError, match="square"):
        tm.seed(torch.zeros(5, 6))
    with pytest.raises(ValueError, match="3 columns"):
        tm.face_sweep(torch.zeros(40, 40), torch.zeros(5, 2, dtype=torch.int32), torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError, match="at least 2 words"):
        tm.face_sweep(torch.zeros(40, 40), torch.zeros(5, 3, dtype=torch.int32), torch.zeros(1, dtype=torch.int32))
    with pytest.raises(ValueError, match="kind"):
        tm.Batch([("Y", torch.zeros(8, 8))])
    with pytest.raises(ValueError, match="square"):
        tm.Batch([("W", torch.zeros(8, 9))])
    n = 8
    W = np.eye(n, dtype=np.float32)
    order = np.arange(n, dtype=np.int32)
    edges = np.zeros((3 * n - 6, 2), np.int32)
    steps = np.zeros((n - 4, 4), np.int32)
    with pytest.raises(ValueError, match="order must have 8 rows"):
        tm.dbht(W, order[:-1], edges, steps, 2)
    with pytest.raises(ValueError, match="edges must have 18 rows"):
        tm.dbht(W, order, edges[:-1], steps, 2)
    with pytest.raises(ValueError, match="steps must have 4 rows"):
        tm.dbht(W, order, edges, steps[:-1], 2)
    with pytest.raises(ValueError, match="square"):
        tm.dbht(W[:, :-1], order, edges, steps, 2)


def test_missing_library_raises(monkeypatch):
    """Without libtmfg.so the binding raises at the first call: there is no CPU fallback."""
    import torch
    import paper_2408_09399_amd as tm
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libtmfg.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.lib()
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        tm.footprint_bytes(100, 16)


def test_batch_footprint_host_side():
    """tmfg_batch_footprint_bytes checks every job and sizes its scratch on the host (no
    device call): the pointers below are placeholders it only tests for NULL."""
    lib = binding.lib()
    P = 0x1000

    def job(n, L=0, X=False, W_out=False, steps=True):
        j = binding.Job()
        j.n, j.L = n, L
        j.X, j.W = (P, None) if X else (None, P)
        j.W_out = P if W_out else None
        j.order = j.edges = j.faces = j.status = P
        j.steps = j.step_gain = P if steps else None
        return j

    def fp(*jobs):
        arr = (binding.Job * len(jobs))(*jobs)
        return lib.tmfg_batch_footprint_bytes(ctypes.cast(arr, ctypes.c_void_p), len(jobs), 0)

    assert fp(job(3)) == 0 and fp(job(20481)) == 0          # n outside [4, 20480] (batches)
    assert fp(job(20480)) > 0
    assert fp(job(100, steps=False)) == 0                   # steps needed from n = 5
    assert fp(job(4, steps=False)) > 0
    neither = job(100)
    neither.W = None
    assert fp(neither) == 0                                 # exactly one of X and W
    assert fp(job(100, L=1, X=True)) == 0                   # L < 2
    assert fp(job(100), neither) == 0                       # one bad job spoils the batch
    n, L = 1000, 256
    ldi = (n - 1 + 7) // 8 * 8
    w = fp(job(n))
    x = fp(job(n, L, X=True))
    xo = fp(job(n, L, X=True, W_out=True))
    assert w >= 6 * n * ldi                                 # sorted ids and values
    assert x - xo >= 4 * n * n                              # its own W without a W_out
    assert xo - w >= n * L * 4                              # the standardised series
    two = fp(job(n), job(500))
    assert two - w >= 6 * 500 * ((499 + 7) // 8 * 8)


def test_noalloc_build_host_side_checks():
    """tmfg_build_noalloc refuses, before any device call, bad flags (TMFG_TIMING among them)
    and jobs whose scratch would not fit its fixed array; the limit is the plan footprint."""
    lib = binding.lib()
    P = 0x1000
    cap = 64 << 20

    def job(n, L=0, X=False):
        j = binding.Job()
        j.n, j.L = n, L
        j.X, j.W = (P, None) if X else (None, P)
        j.order = j.edges = j.faces = j.status = j.steps = j.step_gain = P
        return j

    def call(j, flags=0):
        return lib.tmfg_build_noalloc(ctypes.byref(j), flags, None)

    assert lib.tmfg_build_noalloc(None, 0, None) == 1
    assert call(job(100), binding.TIMING) == 1
    assert call(job(100), binding.STATS) == 1                   # plans only
    assert call(job(100), binding.RULE_CORR) == 1               # corr-tmfg needs a prefix
    assert call(job(3)) == 2
    assert call(job(100, L=1, X=True)) == 2
    # the largest n that fits at L = 256, and the next one, which must be refused
    fits = [n for n in range(2400, 2700) if binding.footprint_bytes(n, 256) <= cap]
    n_top = max(fits)
    assert n_top >= 2530 and binding.footprint_bytes(2048, 2048) <= cap
    assert call(job(n_top + 1, L=256, X=True)) == 2
    assert call(job(20000, L=1024, X=True)) == 2
    # a W job is sized as L = 2
    fits_w = max(n for n in range(2400, 2800) if binding.footprint_bytes(n, 2) <= cap)
    assert call(job(fits_w + 1)) == 2
