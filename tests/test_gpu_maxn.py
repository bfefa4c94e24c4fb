"""Builds at the largest size a plan accepts, n = 20480: every structure the insertion loop
keeps in LDS is at its largest there (640 chunk maxima of 64 faces each, the n-bit inserted
set, n row positions), face ids reach 2n - 5 in the 16-bit field of the face record, and a
single build passes all six row-compaction checkpoints. The exact rule, the paper's heap
rule and corr-tmfg with p = 16, bit for bit against their oracles on one random
similarity matrix; and the same matrix as the largest instance of a batch, whose loop runs
without compaction, beside small instances."""
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev, same_tmfg

pytestmark = pytest.mark.gpu

N = 20480
CHECKPOINTS = 6            # n - n/d for d = 4, 8, ..., 128 (n/d >= 128)


@pytest.fixture(scope="module")
def W():
    return synth.random_symmetric(N, 2048)


_refs = {}


def reference(W, rule):
    """The oracle's TMFG of W under `rule`, computed once per module."""
    if rule not in _refs:
        _refs[rule] = {"exact": lambda: oracle.tmfg_lazy(W), "paper": lambda: oracle.tmfg_paper(W),
                       "corr16": lambda: oracle.tmfg_corr_lazyrows(W, 16)}[rule]()
    return _refs[rule]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("rule", ["exact", "paper", "corr16"])
def test_max_n(W, rule):
    flags = {"exact": 0, "paper": tm.RULE_PAPER, "corr16": tm.rule_corr_prefix(16)}[rule]
    plan = tm.Plan(N, 2, flags | tm.STATS)
    print(f"n={N} {rule}: GPU build", flush=True)
    res = tm.build(W=to_dev(W), plan=plan)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0, tm.STATUS.get(got["status"])
    assert plan.stats()[24] == CHECKPOINTS
    print(f"n={N} {rule}: running the oracle", flush=True)
    same_tmfg(got, reference(W, rule))


@pytest.mark.timeout(600)
def test_max_n_in_a_batch(W):
    small = [synth.random_symmetric(n, 300 + n) for n in (5, 97, 640)]
    b = tm.Batch([("W", to_dev(W))] + [("W", to_dev(a)) for a in small])
    print(f"batch with n={N}: GPU run", flush=True)
    results = [r.to_numpy() for r in b.run()]
    torch.cuda.synchronize()
    assert [r["status"] for r in results] == [0] * 4
    print(f"batch with n={N}: comparing", flush=True)
    same_tmfg(results[0], reference(W, "exact"))
    for a, got in zip(small, results[1:]):
        same_tmfg(got, oracle.tmfg_lazy(a))
    b.close()
