"""Batched builds (one graph replay over many instances of uneven n): every instance is
bitwise the result of its own single build, and of the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev, same_tmfg

pytestmark = pytest.mark.gpu


def _mixed_inputs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if i % 5 == 4:
            n = int(rng.integers(4, 300))
            out.append(("W", synth.grid_symmetric(n, seed * 1000 + i, levels=[2, 4, 8][i % 3])))
        else:
            n = int(round(np.exp(rng.uniform(np.log(5), np.log(2500)))))
            L = int(rng.integers(2, 300))
            k = int(rng.integers(1, min(n, 8) + 1))
            sizes = synth.dirichlet_sizes(rng, n, k)
            out.append(("X", synth.planted_clusters(n, L, sizes, (0.3, 1.0), seed=seed * 1000 + i).X))
    return out


def _solo(kind, arr):
    res = tm.build(**{kind: to_dev(arr)}, keep_w=True)
    torch.cuda.synchronize()
    return res.to_numpy()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_solo_and_oracle(graph):
    inputs = _mixed_inputs(40, 11)
    dev = [(k, to_dev(a)) for k, a in inputs]
    b = tm.Batch(dev, keep_w=True, flags=0 if graph else tm.BATCH_NO_GRAPH)
    for rep in range(2):                              # replays give the same results
        results = [r.to_numpy() for r in b.run()]
        torch.cuda.synchronize()
        for (kind, arr), got in zip(inputs, results):
            assert got["status"] == 0
            solo = _solo(kind, arr)
            assert got["W"].tobytes() == solo["W"].tobytes()
            same_tmfg(got, solo)
            if rep == 0 and got["order"].shape[0] <= 400:
                same_tmfg(got, oracle.tmfg_lazy(got["W"]))
    b.close()


def test_batch_c4_sample():
    inst = synth.config_c4(48)
    dev = [("X", to_dev(s.X)) for s in inst]
    b = tm.Batch(dev, keep_w=True)
    results = [r.to_numpy() for r in b.run()]
    torch.cuda.synchronize()
    for s, got in zip(inst, results):
        assert got["status"] == 0
        solo = _solo("X", s.X)
        assert got["W"].tobytes() == solo["W"].tobytes()
        same_tmfg(got, solo)
    # oracle on a few of them, the largest included
    big = int(np.argmax([s.X.shape[0] for s in inst]))
    for i in {0, 1, big}:
        same_tmfg(results[i], oracle.tmfg_lazy(results[i]["W"]))
    b.close()


def test_batch_errors_per_instance():
    good = synth.random_symmetric(30, 1)
    bad = good.copy()
    bad[2, 5] = np.nextafter(bad[2, 5], np.float32(2.0))
    X = synth.config_c1().X.copy()
    X[3] = 7.0
    b = tm.Batch([("W", to_dev(good)), ("W", to_dev(bad)), ("X", to_dev(X))])
    res = b.run()
    torch.cuda.synchronize()
    assert [int(r.status.item()) for r in res] == [0, 4, 5]
    b.close()


def test_build_batch_plan_cache():
    import ctypes
    from paper_2408_09399_amd import binding
    inputs = [("X", to_dev(synth.config_c1().X)), ("W", to_dev(synth.random_symmetric(50, 3)))]
    results = [binding.alloc_result(t.shape[0], t.device) for _, t in inputs]
    jobs = (binding.Job * 2)()
    for i, ((k, t), r) in enumerate(zip(inputs, results)):
        jobs[i] = binding.make_job(t.shape[0], t.shape[1] if k == "X" else 0, t if k == "X" else None,
                                   t if k == "W" else None, r)
    plan = tm.Plan(64, 2)
    for _ in range(2):
        code = binding.lib().tmfg_build_batch(plan.handle, ctypes.cast(jobs, ctypes.c_void_p), 2,
                                             torch.cuda.current_stream().cuda_stream)
        assert code == 0
        torch.cuda.synchronize()
        assert [int(r.status.item()) for r in results] == [0, 0]


def test_autotuned_batch_same_results():
    """The tuner changes launch configurations only: results stay bitwise those of the
    default batch, and the chosen configuration fits every size class present."""
    inst = synth.config_c4(24)
    dev = [("X", to_dev(s.X)) for s in inst]
    ref = tm.Batch(dev)
    want = [r.to_numpy() for r in ref.run()]
    torch.cuda.synchronize()
    tuned = tm.Batch(dev, flags=tm.BATCH_AUTOTUNE)
    cfg = tuned.config()
    assert cfg["tune_trials"] > 0 and cfg["loop_workgroups"] >= 1
    assert any(c >= 0 for c in cfg["sort_config"])
    assert cfg["walk_rounds"] in (64, 16, 8)
    for rep in range(2):
        got = [r.to_numpy() for r in tuned.run()]
        torch.cuda.synchronize()
        for g, w in zip(got, want):
            assert g["status"] == 0
            same_tmfg(g, w)
    base = ref.config()
    assert base["tune_trials"] == 0 and base["walk_rounds"] == 64
    ref.close()
    tuned.close()
