"""Pearson similarity on the GPU (standardise + FP32-MFMA GEMM) vs the float64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _check_w(W: np.ndarray, R: np.ndarray):
    assert np.isfinite(W).all()
    assert np.abs(W.astype(np.float64) - R).max() <= TOL
    assert np.array_equal(W.view(np.uint32), W.T.view(np.uint32)), "W not bitwise symmetric"
    assert (np.diag(W) == np.float32(1.0)).all()
    assert not (W.view(np.uint32) == 0x80000000).any(), "-0.0 present"
    assert np.abs(W).max() <= 1.0


@pytest.mark.parametrize("n,L", [(4, 2), (200, 128), (129, 33), (777, 301), (1500, 64)])
def test_pearson_small(n, L):
    s = synth.planted_clusters(n, L, [n // 2, n - n // 2], 0.7, seed=n * 31 + L)
    W, st = tm.correlation(to_dev(s.X))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _check_w(W.cpu().numpy(), oracle.pearson64(s.X))


def test_pearson_c2():
    s = synth.config_c2()
    W, st = tm.correlation(to_dev(s.X))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _check_w(W.cpu().numpy(), oracle.pearson64(s.X))


def test_pearson_c3_sampled_rows():
    s = synth.config_c3()
    W, st = tm.correlation(to_dev(s.X))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(s.X.shape[0], 48, replace=False))
    x = s.X.astype(np.float64)
    z = x - x.mean(1, keepdims=True)
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    Wr = W[torch.from_numpy(rows).to(W.device)].cpu().numpy()
    Rr = z[rows] @ z.T
    Rr[np.arange(len(rows)), rows] = 1.0
    assert np.abs(Wr - Rr).max() <= TOL
    # symmetry on the sampled rows: W[r, :] == W[:, r] bitwise
    Wc = W[:, torch.from_numpy(rows).to(W.device)].cpu().numpy().T
    assert np.array_equal(Wr.view(np.uint32), Wc.view(np.uint32))


def test_pearson_errors():
    s = synth.planted_clusters(100, 50, [50, 50], 0.5, seed=3)
    X = s.X.copy()
    X[17] = 2.5                       # constant series
    W, st = tm.correlation(to_dev(X))
    torch.cuda.synchronize()
    assert int(st.item()) == 5
    X = s.X.copy()
    X[3, 7] = np.nan
    W, st = tm.correlation(to_dev(X))
    torch.cuda.synchronize()
    assert int(st.item()) == 3
