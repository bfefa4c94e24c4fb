"""The insertion loop's counters are recorded only for plans made with TMFG_STATS, and the
two kinds of plan give the same bits (the counters are compiled out of the other one)."""
import numpy as np
import pytest
import torch

import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

RULES = {"exact": 0, "paper": tm.RULE_PAPER, "corr4": tm.rule_corr_prefix(4)}


@pytest.mark.parametrize("rule", sorted(RULES))
def test_stats_plan_gives_the_same_bits(rule):
    n, L = 1500, 128                     # past the first row compactions (n - n/4, n - n/8)
    s = synth.planted_clusters(n, L, [500, 400, 300], (0.4, 1.0), n_noise=n - 1200, seed=31)
    X = to_dev(s.X)
    outs = []
    for extra in (0, tm.STATS):
        plan = tm.Plan(n, L, RULES[rule] | extra)
        res = tm.build(X=X, plan=plan, keep_w=True)
        torch.cuda.synchronize()
        got = res.to_numpy()
        assert got["status"] == 0
        if extra:
            st = plan.stats()
            assert st[3] > 0 and st[10] > 0          # phases (rounds) and loop microseconds
            assert st[24] == 2                        # compactions at n - n/4 and n - n/8
        else:
            with pytest.raises(tm.TmfgError):
                plan.stats()
        plan.close()
        outs.append(got)
    a, b = outs
    for k in ("order", "edges", "steps", "faces"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["step_gain"].view(np.int32), b["step_gain"].view(np.int32))
    assert np.array_equal(a["W"].view(np.int32), b["W"].view(np.int32))
