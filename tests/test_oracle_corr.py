"""corr-tmfg with a prefix size (Algorithm 1) in the oracle: hand-derived cases for a
two-vertex round, a prefix conflict and the eager update, the candidate property of every
step, the structural invariants, and a second formulation (MaxCorrs evaluated on use)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import check_tmfg, tmfg_exact
from oracle import corr_rule
from oracle.corr_rule import tmfg_corr, tmfg_corr_lazyrows
from oracle.paper_rule import check_paper_steps, tmfg_paper
from paper_2408_09399_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = ["corr_rule_n7_prefix.json", "corr_rule_n7_eager.json"]


def _same(a, b):
    for k in ("order", "edges", "steps", "faces"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert np.asarray(a["step_gain"], np.float32).tobytes() == np.asarray(b["step_gain"], np.float32).tobytes()


@pytest.mark.parametrize("name", CASES)
def test_golden(name):
    fx = json.load(open(os.path.join(GOLDEN, name)))
    W = np.asarray(fx["W"], dtype=np.float32)
    for p, exp in fx["expected"].items():
        want = {k: np.asarray(v) for k, v in exp.items()}
        for fn in (tmfg_corr, tmfg_corr_lazyrows):
            got = fn(W, int(p))
            _same(got, want)
            check_tmfg(W, got)
            check_paper_steps(W, got)


def test_eager_departs_from_heap():
    """The eager update (Algorithm 1) and the heap (Algorithm 2) take different faces for the
    second vertex on the same matrix."""
    fx = json.load(open(os.path.join(GOLDEN, "corr_rule_n7_eager.json")))
    W = np.asarray(fx["W"], dtype=np.float32)
    assert tmfg_corr(W, 1)["steps"][1].tolist() == [1, 0, 1, 3]
    assert tmfg_paper(W)["steps"][1].tolist() == [2, 0, 2, 3]


@pytest.mark.parametrize("seed", range(30))
def test_formulations_agree(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(4, 70))
    W = synth.random_symmetric(n, 300 + seed) if seed % 2 else \
        synth.grid_symmetric(n, 300 + seed, levels=[2, 3, 5, 8][seed % 4])
    for p in (1, 2, 3, 8):
        a, b = tmfg_corr(W, p), tmfg_corr_lazyrows(W, p)
        _same(a, b)
        check_tmfg(W, a, planarity=(seed % 5 == 0))
        check_paper_steps(W, a)


def test_prefix_covers_everything():
    """With a prefix as large as the number of faces every round inserts one vertex per
    distinct pair vertex; the result is still a valid TMFG whose steps are all candidates."""
    W = synth.random_symmetric(40, 7)
    a = tmfg_corr(W, 10_000)
    check_tmfg(W, a)
    check_paper_steps(W, a)
    _same(a, tmfg_corr_lazyrows(W, 10_000))


def test_planted_clusters_c1_edge_sum():
    s = synth.config_c1()
    W = oracle.pearson64(s.X).astype(np.float32)
    ee = float(np.asarray(tmfg_exact(W)["step_gain"], np.float64).sum())
    for p in (1, 4):
        a = tmfg_corr(W, p)
        check_tmfg(W, a)
        ea = float(np.asarray(a["step_gain"], np.float64).sum())
        assert ea <= ee + 1e-6 and abs(ea - ee) / abs(ee) < 0.05


def test_bad_prefix():
    W = synth.random_symmetric(6, 1)
    with pytest.raises(ValueError):
        tmfg_corr(W, 0)
    with pytest.raises(ValueError):
        tmfg_corr_lazyrows(W, 0)


def test_planted_mistake_in_conflict_rule(monkeypatch):
    """A planted mistake: a prefix that keeps every pair, even two with the same vertex,
    inserts vertex 2 twice on the hand-derived case, and the invariants reject it."""
    fx = json.load(open(os.path.join(GOLDEN, "corr_rule_n7_prefix.json")))
    W = np.asarray(fx["W"], dtype=np.float32)

    def no_conflicts(pu, pg, p):
        live = [f for f in range(len(pu)) if pu[f] >= 0]
        return sorted(live, key=lambda f: corr_rule._key(pg[f], f), reverse=True)[:p]

    monkeypatch.setattr(corr_rule, "_prefix", no_conflicts)
    got = tmfg_corr(W, 2)
    assert got["order"].tolist().count(2) == 2
    with pytest.raises(AssertionError):
        check_tmfg(W, got)
