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
    assert (cfg["tune_trials"] > 0 or cfg["from_cache"]) and cfg["loop_workgroups"] >= 1
    assert all(t in (64, 128) for t in cfg["gemm_tile"])
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


def _series_inputs(ns, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i, n in enumerate(ns):
        L = int(rng.integers(30, 400))
        k = int(rng.integers(1, min(n, 8) + 1))
        out.append(("X", synth.planted_clusters(n, L, synth.dirichlet_sizes(rng, n, k), (0.3, 1.0),
                                                seed=seed * 100 + i).X))
    return out


def test_gemm_tiles_give_the_same_bits():
    """The correlation GEMM's tile (128 rows and four waves, or 64 rows and one wave) only
    decides how many waves share a tile: W, and so every output, is the same bits under
    every choice, for instances below and above the 1024 split, and equals the single
    build's (which always uses 128)."""
    inputs = _series_inputs([5, 64, 65, 130, 700, 1023, 1024, 1300, 2100], 31)
    dev = [(k, to_dev(a)) for k, a in inputs]
    b = tm.Batch(dev, keep_w=True)
    base = b.config()
    assert base["gemm_tile"] == [128, 128] and not base["from_cache"]
    want = [r.to_numpy() for r in b.run()]
    torch.cuda.synchronize()
    for tiles in ([64, 64], [64, 128], [128, 64]):
        cfg = dict(base, gemm_tile=tiles)
        b.set_config(cfg)
        assert b.config()["gemm_tile"] == tiles
        for r in b.results:                      # stale outputs must not pass for new ones
            r.W.fill_(float("nan"))
        got = [r.to_numpy() for r in b.run()]
        torch.cuda.synchronize()
        for (kind, arr), g, w in zip(inputs, got, want):
            assert g["status"] == 0
            assert np.array_equal(g["W"].view(np.uint32), w["W"].view(np.uint32)), (tiles, arr.shape)
            same_tmfg(g, w)
    for (kind, arr), w in zip(inputs, want):
        solo = _solo(kind, arr)
        assert np.array_equal(solo["W"].view(np.uint32), w["W"].view(np.uint32))
    b.close()


def test_set_config_rejects_out_of_range_values():
    inputs = _series_inputs([40, 300, 1500], 32)
    b = tm.Batch([(k, to_dev(a)) for k, a in inputs])
    base = b.config()
    bad = [dict(base, gemm_tile=[96, 128]), dict(base, walk_rounds=0), dict(base, walk_rounds=65),
           dict(base, loop_workgroups=0), dict(base, loop_workgroups=base["loop_workgroups"] + 1),
           dict(base, sort_rows_per_wg=-1),
           dict(base, sort_config=[99 if c >= 0 else c for c in base["sort_config"]])]
    for cfg in bad:
        with pytest.raises(RuntimeError):
            b.set_config(cfg)
        assert b.config() == base
    ok = dict(base, walk_rounds=8, loop_workgroups=1, sort_rows_per_wg=4)
    b.set_config(ok)
    got = b.config()
    assert (got["walk_rounds"], got["loop_workgroups"], got["sort_rows_per_wg"]) == (8, 1, 4)
    res = [r.to_numpy() for r in b.run()]
    torch.cuda.synchronize()
    for (kind, arr), g in zip(inputs, res):
        same_tmfg(g, _solo(kind, arr))
    b.close()


def test_tuning_cache_in_process():
    """A second autotuned batch of the same shape takes the first one's choice from the
    process's tuning cache, without timing, and gives the same results."""
    inputs = _series_inputs([37, 210, 1200, 1900, 77], 33)
    dev = [(k, to_dev(a)) for k, a in inputs]
    first = tm.Batch(dev, flags=tm.BATCH_AUTOTUNE)
    c1 = first.config()
    want = [r.to_numpy() for r in first.run()]
    torch.cuda.synchronize()
    second = tm.Batch(dev, flags=tm.BATCH_AUTOTUNE)
    c2 = second.config()
    assert c2["from_cache"] and c2["tune_trials"] == 0
    for k in ("sort_config", "sort_rows_per_wg", "loop_workgroups", "walk_rounds", "gemm_tile"):
        assert c2[k] == c1[k], k
    got = [r.to_numpy() for r in second.run()]
    torch.cuda.synchronize()
    for g, w in zip(got, want):
        same_tmfg(g, w)
    first.close()
    second.close()


_CACHE_SCRIPT = """
import sys, json, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
rng = np.random.default_rng(34)
xs = [synth.planted_clusters(n, 96, synth.dirichlet_sizes(rng, n, 3), (0.3, 1.0), seed=n).X for n in (51, 400, 1100)]
b = tm.Batch([("X", torch.from_numpy(x).cuda()) for x in xs], flags=tm.BATCH_AUTOTUNE)
print(json.dumps(b.config()))
b.close()
"""


def test_tuning_cache_file_across_processes(tmp_path):
    """With TMFG_TUNE_CACHE set, a later process takes the tuned choice from the file."""
    import json
    import os
    import subprocess
    import sys
    repo = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, TMFG_TUNE_CACHE=str(tmp_path / "tune.txt"))
    runs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", _CACHE_SCRIPT, repo], env=env, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        runs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert not runs[0]["from_cache"] and runs[0]["tune_trials"] > 0
    assert runs[1]["from_cache"] and runs[1]["tune_trials"] == 0
    for k in ("sort_config", "sort_rows_per_wg", "loop_workgroups", "walk_rounds", "gemm_tile"):
        assert runs[1][k] == runs[0][k], k
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(lines) == 1 and "\t" in lines[0]
