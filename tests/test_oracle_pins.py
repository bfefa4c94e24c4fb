"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Hand-derived golden cases (tests/golden/*.json, each citing the passage it follows),
independent library routines (numpy.corrcoef, numpy.argsort), closed forms, a plain
Python loop, and invariances.
"""
import glob
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2408_09399_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


TMFG_CASES = sorted(os.path.basename(p) for p in glob.glob(os.path.join(GOLDEN, "tmfg_*.json")))


@pytest.mark.parametrize("name", TMFG_CASES)
@pytest.mark.parametrize("schedule", ["exact", "lazy", "bruteforce"])
def test_tmfg_golden(name, schedule):
    case = _load(name)
    W = np.asarray(case["W"], dtype=np.float32)
    res = getattr(oracle, "tmfg_" + schedule)(W)
    assert res["order"].tolist() == case["order"]
    assert res["edges"].tolist() == case["edges"]
    assert res["steps"].reshape(-1, 4).tolist() == case["steps"]
    assert res["step_gain"].tolist() == case["step_gain"]
    assert res["faces"].tolist() == case["faces"]
    oracle.check_tmfg(W, res)


def test_pearson_golden():
    case = _load("pearson_tiny.json")
    R = oracle.pearson64(np.asarray(case["X"], dtype=np.float32))
    np.testing.assert_allclose(R, np.asarray(case["R"]), rtol=0, atol=1e-15)


def test_sort_golden():
    case = _load("sort_row_tiny.json")
    row = np.asarray(case["row"], dtype=np.float32)
    W = np.tile(row, (len(row), 1))
    assert oracle.sorted_row(W, case["v"]).tolist() == case["sorted_ids"]


@pytest.mark.parametrize("seed", range(5))
def test_pearson_vs_corrcoef(seed):
    rng = np.random.default_rng(seed)
    X = np.cumsum(rng.standard_normal((40, 64)), axis=1).astype(np.float32)
    R = oracle.pearson64(X)
    np.testing.assert_allclose(R, np.corrcoef(X.astype(np.float64)), rtol=0, atol=1e-12)
    assert np.array_equal(R, R.T)
    assert (np.diag(R) == 1.0).all()


def test_pearson_textbook_loop():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, 9)).astype(np.float32)
    R = oracle.pearson64(X)
    for i in range(5):
        for j in range(5):
            xi = [float(v) for v in X[i]]
            xj = [float(v) for v in X[j]]
            mi, mj = sum(xi) / 9, sum(xj) / 9
            num = sum((a - mi) * (b - mj) for a, b in zip(xi, xj))
            den = math.sqrt(sum((a - mi) ** 2 for a in xi) * sum((b - mj) ** 2 for b in xj))
            assert abs(R[i, j] - num / den) < 1e-13


def test_pearson_closed_form_L2():
    X = np.array([[0.0, 1.0], [5.0, 3.0], [-2.0, 7.5]], dtype=np.float32)
    R = oracle.pearson64(X)
    expect = np.array([[1, -1, 1], [-1, 1, -1], [1, -1, 1]], dtype=np.float64)
    np.testing.assert_allclose(R, expect, atol=1e-15)


def test_pearson_affine_invariance():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((12, 30))
    Y = 2.5 * X + 4.0
    np.testing.assert_allclose(oracle.pearson64(X.astype(np.float32)),
                               oracle.pearson64(Y.astype(np.float32)), atol=1e-6)


def test_pearson_errors():
    X = np.ones((3, 5), dtype=np.float32)
    X[0] = [1, 2, 3, 4, 5]
    X[2] = [1, 2, 3, 4, 5]
    with pytest.raises(oracle.DegenerateSeries):
        oracle.pearson64(X)
    X[1, 0] = np.nan
    with pytest.raises(oracle.NonFinite):
        oracle.pearson64(X)


@pytest.mark.parametrize("seed", range(4))
def test_sort_vs_argsort(seed):
    W = synth.grid_symmetric(50, seed, levels=4)   # many ties
    W[0, 1] = W[1, 0] = np.float32(-0.0)
    W[0, 2] = W[2, 0] = np.float32(0.0)
    S = oracle.sorted_rows(W)
    for v in range(50):
        row = W[v].copy()
        ids = np.argsort(-row, kind="stable")
        ids = ids[ids != v]
        assert S[v].tolist() == ids.tolist()


def test_seed_scores_vs_python_loop():
    W = synth.random_symmetric(37, 11)
    s = oracle.seed_scores(W)
    for v in range(37):
        acc = 0.0
        for u in range(37):
            if u != v:
                acc += float(W[v, u])
        assert s[v] == acc     # same sequential float64 order: bit-equal


def test_seed_scores_exact_on_grid():
    # Grid entries (multiples of 1/8) make every float64 partial sum exact, so the scores
    # must equal the exact rational row sums whatever the order.
    from fractions import Fraction
    W = synth.grid_symmetric(41, 5, levels=16)
    s = oracle.seed_scores(W)
    for v in range(41):
        exact = sum(Fraction(float(W[v, u])) for u in range(41) if u != v)
        assert Fraction(s[v]) == exact


def test_seed_tie_lowest_id():
    n = 8
    W = np.full((n, n), 0.25, dtype=np.float32)
    np.fill_diagonal(W, 1.0)
    assert oracle.seed_vertices(W) == [0, 1, 2, 3]
    W[7, :6] = W[:6, 7] = 0.5
    W[5, 6] = W[6, 5] = 0.5
    # row sums: 7 -> 6*0.5+0.25 = 3.25; 5 -> 5*0.25+0.5+0.5 = 2.25; rows 0..4 and 6 -> 2.0
    # (a six-way tie, resolved to the lowest ids 0 and 1)
    assert oracle.seed_vertices(W) == [7, 5, 0, 1]


def test_errors():
    with pytest.raises(oracle.SizeError):
        oracle.tmfg_exact(np.eye(3, dtype=np.float32))
    W = synth.random_symmetric(6, 0)
    W[1, 2] = np.inf
    with pytest.raises(oracle.NonFinite):
        oracle.tmfg_exact(W)
