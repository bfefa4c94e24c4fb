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
    assert lib.tmfg_plan_create(None, 100, 10, 0) == 1
    assert lib.tmfg_plan_create(ctypes.byref(h), 3, 10, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 20481, 10, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 1, 0) == 2
    assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, 1 << 10) == 1
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
        assert lib.tmfg_plan_create(ctypes.byref(h), 100, 10, bad) == 1, hex(bad)
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
                             ("max_batch", 4097, 1), ("n_streams", 0, 1), ("n_streams", 5, 1),
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
