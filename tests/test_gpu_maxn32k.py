"""Single builds above the in-LDS row sort, up to n = 32768, the most vertices whose 2n - 4
face ids fit the face record's 16-bit field. Rows of more than 20480 entries are sorted as
two halves of their columns and merged; the sorted rows are compared with the oracle's
order on sampled rows (a tie-heavy matrix just above the threshold, where equal values
straddle the two halves, and n = 32768), and the whole TMFG at n = 32768 bit for bit with
the oracle under the exact rule and the paper's rule. Batches, servers and corr-tmfg stop
at n = 20480 and refuse larger sizes."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev, same_tmfg, uint16_rows

pytestmark = pytest.mark.gpu

N = 32768


def _sample_rows(n, extra=()):
    rng = np.random.default_rng(n)
    h = n // 2
    rows = {0, 1, h - 1, h, h + 1, n - 2, n - 1, *extra}
    rows.update(int(x) for x in rng.integers(0, n, 24))
    return sorted(r for r in rows if 0 <= r < n)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n", [20482, 20483])
def test_two_run_sort_ties_across_halves(n):
    """Grid values: every row has long runs of equal similarities on both sides of n/2."""
    W = synth.grid_symmetric(n, 77 + n, levels=4)
    plan = tm.Plan(n, 2)
    idx, vals = tm.sort_rows(to_dev(W), plan=plan, with_values=True)
    torch.cuda.synchronize()
    got = uint16_rows(idx, n)
    gv = vals.cpu().numpy()
    for v in _sample_rows(n):
        want = oracle.sorted_row(W, v)
        assert np.array_equal(got[v], want), f"row {v}"
        assert np.array_equal(gv[v, : n - 1], W[v, want] + np.float32(0.0)), f"row {v} values"
        assert (idx[v, n - 1:].cpu().numpy().view(np.uint16) == 0xffff).all()
        assert np.isneginf(gv[v, n - 1:]).all()


@pytest.fixture(scope="module")
def big():
    rng = np.random.default_rng(3276)
    s = synth.planted_clusters(N, 64, synth.dirichlet_sizes(rng, N - 2048, 40), (0.3, 1.0), n_noise=2048, seed=3276)
    return s.X


_refs = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("rule", ["exact", "paper"])
def test_n32768_build(big, rule):
    flags = tm.RULE_PAPER if rule == "paper" else 0
    plan = tm.Plan(N, 64, flags | tm.STATS)
    print(f"n={N} {rule}: GPU build", flush=True)
    res = tm.build(X=to_dev(big), plan=plan, keep_w=True)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0, tm.STATUS.get(got["status"])
    assert plan.stats()[24] == 7                     # n - n/d for d = 4, ..., 256 (n/d >= 128)
    W = got["W"]
    if rule == "exact":
        # the sorted rows themselves, on a sample
        idx = tm.sort_rows(res.W, plan=plan)
        torch.cuda.synchronize()
        rows = uint16_rows(idx, N)
        for v in _sample_rows(N, extra=(int(got["order"][0]), int(got["order"][-1]))):
            assert np.array_equal(rows[v], oracle.sorted_row(W, v)), f"row {v}"
        del idx, rows
    print(f"n={N} {rule}: running the oracle", flush=True)
    ref = oracle.tmfg_lazy(W) if rule == "exact" else oracle.tmfg_paper(W)
    same_tmfg(got, ref)
    if rule == "exact":
        oracle.check_tmfg(W, got, planarity=False)


def test_limits_above_20480_for_batches_servers_and_corr():
    with pytest.raises(tm.TmfgError, match="SIZE"):
        tm.Plan(20481, 2, tm.rule_corr_prefix(4))
    with pytest.raises(tm.TmfgError, match="SIZE"):
        tm.Server(hbm_budget=1 << 30, host_budget=1 << 20, n_max=20481)
    W = torch.zeros((20481, 20481), dtype=torch.float32, device="cuda:0")
    with pytest.raises(tm.TmfgError, match="SIZE"):
        tm.Batch([("W", W)])
    del W
    with pytest.raises(tm.TmfgError, match="SIZE"):
        tm.Plan(N + 1, 2)
    with pytest.raises(tm.TmfgError, match="INVALID"):
        tm.Plan(100, 2, tm.binding.IDX32)
