"""Request server (continuous batching from host memory): every request's result is bitwise
that of its own single build, under a roomy budget and under one that admits a single
request at a time; a bad request fails alone; tickets are collected once."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import binding, synth
from gpu_util import to_dev, same_tmfg

pytestmark = pytest.mark.gpu


def _requests(count, seed, n_hi=1500):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = [4, 5, 6][i] if i < 3 else int(round(np.exp(rng.uniform(np.log(7), np.log(n_hi)))))
        L = int(rng.integers(2, 260))
        k = int(rng.integers(1, min(n, 8) + 1))
        sizes = synth.dirichlet_sizes(rng, n, k)
        out.append(synth.planted_clusters(n, L, sizes, (0.3, 1.0), seed=seed * 1000 + i).X)
    return out


def _solo(X):
    res = tm.build(X=to_dev(X), keep_w=True)
    torch.cuda.synchronize()
    return res.to_numpy()


def _serve(server, reqs):
    tickets = [server.submit(X) for X in reqs]
    return [server.poll(t, wait_ms=-1) for t in tickets]


@pytest.mark.parametrize("flags", [0, binding.SERVER_FIFO])
def test_server_equals_solo_builds(flags):
    reqs = _requests(40, 3)
    srv = tm.Server(hbm_budget=2 << 30, host_budget=256 << 20, max_batch=16, n_streams=2, n_max=2048, L_max=512,
                    flags=flags)
    got = _serve(srv, reqs)
    for X, g in zip(reqs, got):
        assert g["status"] == 0
        solo = _solo(X)
        same_tmfg(g, solo)
        assert g["arrival_ns"] <= g["dispatch_ns"] <= g["done_ns"]
        if X.shape[0] <= 300:
            same_tmfg(g, oracle.tmfg_lazy(solo["W"]))
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["submitted"] == len(reqs) and st["waiting"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["dispatches"] >= 3 and st["mean_batch"] <= 16
    srv.close()


def test_server_tight_budget_serialises():
    reqs = _requests(10, 4, n_hi=600)
    probe = tm.Server(hbm_budget=1 << 30, host_budget=64 << 20, max_batch=8, n_streams=1, n_max=1024, L_max=512)
    probe.close()
    # room for the largest request only: every dispatch holds one request
    big = max(X.shape[0] for X in reqs)
    Lmax = max(X.shape[1] for X in reqs)
    budget = 2 * tm.footprint_bytes(big, Lmax)
    srv = tm.Server(hbm_budget=budget, host_budget=64 << 20, max_batch=8, n_streams=2, n_max=1024, L_max=512)
    got = _serve(srv, reqs)
    for X, g in zip(reqs, got):
        assert g["status"] == 0
        same_tmfg(g, _solo(X))
    assert srv.stats()["completed"] == len(reqs)
    srv.close()


def test_server_bad_request_fails_alone_and_tickets_are_single_use():
    reqs = _requests(6, 5, n_hi=400)
    bad = reqs[2].copy()
    bad[3, :] = 1.25                                  # a constant series: no correlation
    reqs[2] = bad
    srv = tm.Server(hbm_budget=1 << 30, host_budget=64 << 20, max_batch=8, n_streams=1, n_max=1024, L_max=512)
    tickets = [srv.submit(X) for X in reqs]
    got = [srv.poll(t) for t in tickets]
    for i, (X, g) in enumerate(zip(reqs, got)):
        if i == 2:
            assert tm.STATUS[g["status"]] == "TMFG_E_DEGENERATE"
        else:
            assert g["status"] == 0
            same_tmfg(g, _solo(X))
    r = binding.ServerResult()
    assert binding.lib().tmfg_server_poll(srv._h, tickets[0], 0, ctypes.byref(r)) == 1
    with pytest.raises(tm.TmfgError):
        srv.submit(np.zeros((2000, 8), np.float32))   # n above the server's n_max
    srv.close()
