"""MI355X-native construction of the triangular maximally filtered graph (TMFG).

The compute path is libtmfg.so (hand-written HIP for gfx950 behind the C ABI in
include/tmfg.h); this package holds its ctypes binding and the seeded synthetic input
generators. The library is loaded on first use, and a missing build raises.
"""
from .binding import (Plan, Result, Batch, Server, TmfgError, build, correlation, sort_rows, seed, face_sweep, dbht,
                      footprint_bytes, alloc_result, load_latency_ns, STATUS, NO_VALIDATE, TIMING, STATS, BATCH_NO_GRAPH, BATCH_AUTOTUNE,
                      RULE_PAPER, RULE_CORR, rule_corr_prefix, SERVER_FIFO, SERVER_RULE_PAPER, PENDING)

__all__ = ["Plan", "Result", "Batch", "Server", "TmfgError", "build", "correlation", "sort_rows", "seed",
           "face_sweep", "dbht", "footprint_bytes", "alloc_result", "load_latency_ns", "STATUS", "NO_VALIDATE", "TIMING", "STATS",
           "BATCH_NO_GRAPH", "BATCH_AUTOTUNE", "RULE_PAPER", "RULE_CORR", "rule_corr_prefix", "SERVER_FIFO", "SERVER_RULE_PAPER", "PENDING"]
