"""tmfg_build_noalloc (the build whose scratch is the library's fixed device array) against
tmfg_build on a plan: two calls in a row on one stream, the second with a smaller input,
each bitwise equal to the plan build of the same job."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2408_09399_amd as tm
from paper_2408_09399_amd import binding, synth
from gpu_util import DEV, to_dev, same_tmfg

pytestmark = pytest.mark.gpu


def _noalloc(n, L, X, W, keep_w, flags=0):
    res = binding.alloc_result(n, DEV, keep_w)
    job = binding.make_job(n, L, X, W, res)
    code = binding.lib().tmfg_build_noalloc(ctypes.byref(job), flags, torch.cuda.current_stream().cuda_stream)
    assert code == 0, tm.STATUS.get(code)
    res._job = job
    return res


def test_noalloc_equals_plan_build_two_calls():
    rng = np.random.default_rng(21)
    n1, L1 = 2000, 256                    # series in; n >= 512, so the loop compacts its rows
    X1 = to_dev(synth.planted_clusters(n1, L1, synth.dirichlet_sizes(rng, n1, 12), (0.3, 1.0), seed=21).X)
    n2 = 300                              # a tie-heavy similarity in, smaller than the first
    W2 = to_dev(synth.grid_symmetric(n2, 22, levels=4))
    print(f"noalloc: n={n1} L={L1} from series, then n={n2} from W", flush=True)
    r1 = _noalloc(n1, L1, X1, None, keep_w=True)
    r2 = _noalloc(n2, 0, None, W2, keep_w=False)
    torch.cuda.synchronize()
    ref1 = tm.build(X=X1, keep_w=True)
    ref2 = tm.build(W=W2)
    torch.cuda.synchronize()
    g1, w1 = r1.to_numpy(), ref1.to_numpy()
    g2, w2 = r2.to_numpy(), ref2.to_numpy()
    assert g1["status"] == 0 and g2["status"] == 0
    assert g1["W"].tobytes() == w1["W"].tobytes()
    same_tmfg(g1, w1)
    same_tmfg(g2, w2)
    # a third call, larger again, under the paper's rule, after the smaller one
    r3 = _noalloc(n1, L1, X1, None, keep_w=False, flags=binding.RULE_PAPER)
    ref3 = tm.build(X=X1, flags=binding.RULE_PAPER)
    torch.cuda.synchronize()
    g3, w3 = r3.to_numpy(), ref3.to_numpy()
    assert g3["status"] == 0
    same_tmfg(g3, w3)
