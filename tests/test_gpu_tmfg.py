"""Full TMFG builds on the GPU, bit-exact against the CPU oracle fed the same W bytes."""
import glob
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev, same_tmfg

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _build_w(W: np.ndarray, plan=None) -> dict:
    res = tm.build(W=to_dev(W), plan=plan)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0, tm.STATUS.get(got["status"])
    return got


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "tmfg_*.json"))),
                         ids=lambda p: os.path.basename(p))
def test_golden(path):
    case = json.load(open(path))
    W = np.asarray(case["W"], dtype=np.float32)
    got = _build_w(W)
    assert got["order"].tolist() == case["order"]
    assert got["edges"].tolist() == case["edges"]
    assert got["steps"].tolist() == case["steps"]
    assert got["step_gain"].tolist() == case["step_gain"]
    assert got["faces"].tolist() == case["faces"]


def test_random_small_many():
    plan = tm.Plan(120, 2)
    for seed in range(60):
        n = 4 + (seed * 13) % 117
        W = synth.random_symmetric(n, 500 + seed)
        got = _build_w(W, plan)
        same_tmfg(got, oracle.tmfg_lazy(W))


def test_tie_heavy_many():
    plan = tm.Plan(300, 2)
    for seed in range(40):
        n = 5 + (seed * 37) % 290
        W = synth.grid_symmetric(n, 900 + seed, levels=[2, 4, 8][seed % 3])
        got = _build_w(W, plan)
        same_tmfg(got, oracle.tmfg_bruteforce(W) if n <= 60 else oracle.tmfg_lazy(W))


def test_all_equal_weights():
    W = np.full((150, 150), 0.5, dtype=np.float32)
    np.fill_diagonal(W, 1.0)
    same_tmfg(_build_w(W), oracle.tmfg_lazy(W))


def test_c1_series_path():
    s = synth.config_c1()
    res = tm.build(X=to_dev(s.X), keep_w=True)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0
    assert np.abs(got["W"].astype(np.float64) - oracle.pearson64(s.X)).max() <= 1e-5
    ref = oracle.tmfg_lazy(got["W"])
    same_tmfg(got, ref)
    oracle.check_tmfg(got["W"], got)


def test_c2_series_path():
    s = synth.config_c2()
    res = tm.build(X=to_dev(s.X), keep_w=True)
    torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0
    same_tmfg(got, oracle.tmfg_lazy(got["W"]))
    oracle.check_tmfg(got["W"], got, planarity=False)


def test_ragged_sizes_series_path():
    plan = tm.Plan(3000, 400)
    for n, L in [(4, 7), (5, 2), (97, 45), (1029, 130), (2777, 399)]:
        s = synth.planted_clusters(n, L, [n // 3, n // 3, n - 2 * (n // 3)], 0.6, seed=n + L)
        res = tm.build(X=to_dev(s.X), plan=plan, keep_w=True)
        torch.cuda.synchronize()
        got = res.to_numpy()
        assert got["status"] == 0, (n, L)
        same_tmfg(got, oracle.tmfg_lazy(got["W"]))


def test_repeat_determinism():
    s = synth.config_c1()
    X = to_dev(s.X)
    plan = tm.Plan(200, 128)
    first = None
    for _ in range(10):
        got = tm.build(X=X, plan=plan, keep_w=True)
        torch.cuda.synchronize()
        d = got.to_numpy()
        blob = b"".join(np.ascontiguousarray(d[k]).tobytes()
                        for k in ("W", "order", "edges", "steps", "step_gain", "faces"))
        first = first or blob
        assert blob == first


@pytest.mark.parametrize("batched", [False, True])
def test_w_out_same_as_w(batched):
    """W_out may be the caller's W itself (a single build, and a batch through the C ABI):
    the build leaves W as it is and gives the oracle's result."""
    import ctypes
    from paper_2408_09399_amd import binding
    n = 300
    W = synth.random_symmetric(n, 41)
    Wd = to_dev(W)
    res = tm.alloc_result(n, Wd.device)
    res.W = Wd
    if batched:
        lib = binding.lib()
        jobs = (binding.Job * 1)()
        jobs[0] = binding.make_job(n, 0, None, Wd, res)
        h = ctypes.c_void_p()
        assert lib.tmfg_batch_create(ctypes.byref(h), ctypes.cast(jobs, ctypes.c_void_p), 1, 0) == 0
        assert lib.tmfg_batch_run(h, None) == 0
        torch.cuda.synchronize()
        assert lib.tmfg_batch_destroy(h) == 0
    else:
        tm.build(W=Wd, out=res)
        torch.cuda.synchronize()
    got = res.to_numpy()
    assert got["status"] == 0
    assert got["W"].tobytes() == W.tobytes()
    same_tmfg(got, oracle.tmfg_lazy(W))


def test_device_errors():
    W = synth.random_symmetric(50, 1)
    W2 = W.copy()
    W2[3, 9] = np.nextafter(W2[3, 9], np.float32(2.0))
    res = tm.build(W=to_dev(W2))
    torch.cuda.synchronize()
    assert int(res.status.item()) == 4
    W3 = W.copy()
    W3[5, 6] = W3[6, 5] = np.inf
    res = tm.build(W=to_dev(W3))
    torch.cuda.synchronize()
    assert int(res.status.item()) == 3
    X = synth.config_c1().X.copy()
    X[7] = 1.0
    res = tm.build(X=to_dev(X))
    torch.cuda.synchronize()
    assert int(res.status.item()) == 5


def test_host_errors():
    with pytest.raises(tm.TmfgError):
        tm.build(W=to_dev(np.eye(3, dtype=np.float32)))
    plan = tm.Plan(100, 50)
    with pytest.raises(tm.TmfgError):
        tm.build(W=to_dev(np.eye(101, dtype=np.float32)), plan=plan)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("n,levels", [(4098, 0), (4099, 0), (4099, 3)])
def test_selection_split_threshold(n, levels):
    """Either side of the size from which the exact rule's selection is shared by four waves
    (more than 128 chunks of 64 faces: n = 4099 has 129 chunks, so three of the four waves
    cover no chunk), on a random and a tie-heavy matrix, bit-exact against the oracle."""
    W = synth.random_symmetric(n, n + levels) if levels == 0 else synth.grid_symmetric(n, n, levels=levels)
    same_tmfg(_build_w(W), oracle.tmfg_lazy(W))
