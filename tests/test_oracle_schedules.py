"""Brute force over every face/vertex pair == cached eager == lazy heap, plus invariants.

The cached and lazy schedules rely on one fact: taking vertices out of the candidate
set never raises a face's best gain, so a cached pair whose vertex is still uninserted
stays exact and one whose vertex was inserted is an upper bound. Agreement with brute
force on hundreds of inputs, tie-heavy ones included, pins that reasoning.
"""
import numpy as np
import pytest

import oracle
from paper_2408_09399_amd import synth


def _same(a, b):
    for k in ("order", "edges", "steps", "faces"):
        assert np.array_equal(a[k], b[k]), k
    assert a["step_gain"].tobytes() == b["step_gain"].tobytes()


@pytest.mark.parametrize("block", range(10))
def test_random_continuous(block):
    for seed in range(block * 20, block * 20 + 20):
        n = 4 + seed % 40
        W = synth.random_symmetric(n, seed)
        b = oracle.tmfg_bruteforce(W)
        _same(oracle.tmfg_exact(W), b)
        _same(oracle.tmfg_lazy(W), b)
        oracle.check_tmfg(W, b, planarity=(seed % 5 == 0))


@pytest.mark.parametrize("block", range(10))
def test_tie_heavy_grid(block):
    for seed in range(block * 20, block * 20 + 20):
        n = 4 + (seed * 7) % 50
        levels = [2, 4, 8][seed % 3]
        W = synth.grid_symmetric(n, 1000 + seed, levels=levels)
        b = oracle.tmfg_bruteforce(W)
        _same(oracle.tmfg_exact(W), b)
        _same(oracle.tmfg_lazy(W), b)
        oracle.check_tmfg(W, b, planarity=(seed % 5 == 0))


def test_all_equal_weights():
    W = np.full((12, 12), 0.5, dtype=np.float32)
    np.fill_diagonal(W, 1.0)
    b = oracle.tmfg_bruteforce(W)
    _same(oracle.tmfg_exact(W), b)
    _same(oracle.tmfg_lazy(W), b)
    assert b["order"].tolist() == list(range(12))
    assert (b["steps"][:, 0] == 0).all()     # every gain ties: always face 0, lowest vertex


def test_planted_pearson():
    s = synth.planted_clusters(120, 64, [30, 30, 30, 30], 0.5, seed=9)
    W = oracle.pearson64(s.X).astype(np.float32)
    b = oracle.tmfg_bruteforce(W)
    _same(oracle.tmfg_exact(W), b)
    _same(oracle.tmfg_lazy(W), b)
    oracle.check_tmfg(W, b)


def test_invariant_checker_catches_mistakes():
    # A planted mistake in an oracle result must be caught by the checker.
    W = synth.random_symmetric(15, 2)
    r = oracle.tmfg_exact(W)
    bad = {k: v.copy() for k, v in r.items()}
    bad["step_gain"][3] = np.float32(bad["step_gain"][3] + 1e-3)
    with pytest.raises(AssertionError):
        oracle.check_tmfg(W, bad)
    bad = {k: v.copy() for k, v in r.items()}
    bad["faces"][[2, 5]] = bad["faces"][[5, 2]]
    with pytest.raises(AssertionError):
        oracle.check_tmfg(W, bad)
    bad = {k: v.copy() for k, v in r.items()}
    bad["edges"][10] = bad["edges"][10][::-1]
    with pytest.raises(AssertionError):
        oracle.check_tmfg(W, bad)


def test_wrong_addition_order_would_fail_golden():
    # Summing the gain as a + (b + c) changes the result on the addition-order fixture,
    # so the fixture really pins the order.
    import json, os
    case = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "tmfg_n6_addition_order.json")))
    W = np.asarray(case["W"], dtype=np.float32)
    a, b, c = 0, 1, 2
    right = (W[a, 5] + W[b, 5]) + W[c, 5]
    wrong = W[a, 5] + (W[b, 5] + W[c, 5])
    assert right == np.float32(1.0) and wrong > np.float32(1.0)


def test_signed_zero_gain_recorded_positive():
    # A face whose best gain is exactly zero from -0.0 entries: -0 == +0 in every
    # comparison, and the recorded gain is +0.0.
    W = np.full((5, 5), 0.5, dtype=np.float32)
    np.fill_diagonal(W, 1.0)
    W[4, :4] = W[:4, 4] = np.float32(-0.0)
    for fn in (oracle.tmfg_exact, oracle.tmfg_lazy, oracle.tmfg_bruteforce):
        r = fn(W)
        assert r["step_gain"].view(np.uint32).tolist() == [0]
        oracle.check_tmfg(W, r)


def test_lazy_prefix_is_the_full_schedules_prefix():
    """tmfg_lazy(W, max_steps=k) stops after k insertions of the same schedule (the CPU
    baseline times such a prefix): its order, steps and gains are the full run's first k."""
    from paper_2408_09399_amd import synth
    W = synth.random_symmetric(120, 9)
    full = oracle.tmfg_lazy(W)
    for k in (0, 1, 37, 116):
        r = oracle.tmfg_lazy(W, max_steps=k)
        assert np.array_equal(r["order"], full["order"][:4 + k])
        assert np.array_equal(r["steps"], full["steps"][:k])
        assert r["step_gain"].tobytes() == full["step_gain"][:k].tobytes()
        assert r["faces"].shape == (4 + 2 * k, 3)
    assert all(np.array_equal(oracle.tmfg_lazy(W, max_steps=116)[key], full[key]) for key in full)
