import numpy as np

from paper_2408_09399_amd import synth


def test_reproducible_and_shapes():
    a = synth.config_c1()
    b = synth.config_c1()
    assert a.X.dtype == np.float32 and a.X.shape == (200, 128)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.labels, b.labels)
    assert sorted(np.bincount(a.labels).tolist()) == [40] * 5


def test_within_cluster_more_correlated():
    s = synth.config_c1()
    R = np.corrcoef(s.X.astype(np.float64))
    same = s.labels[:, None] == s.labels[None, :]
    off = ~np.eye(200, dtype=bool)
    assert R[same & off].mean() > R[~same].mean() + 0.3


def test_dirichlet_sizes():
    rng = np.random.default_rng(0)
    sz = synth.dirichlet_sizes(rng, 5000, 20)
    assert sz.sum() == 5000 and (sz >= 1).all() and len(sz) == 20


def test_batch_and_trace():
    inst = synth.config_c4(16)
    assert len(inst) == 16
    for s in inst:
        n, L = s.X.shape
        assert 64 <= n <= 4096 and 64 <= L <= 512
    tr = synth.serving_trace(100.0, 20)
    t = [r.t_arrival for r in tr]
    assert t[0] == 0.0 and all(x <= y for x, y in zip(t, t[1:]))
    assert all(r.series.X.shape[1] == 256 for r in tr)


def test_grid_symmetric():
    W = synth.grid_symmetric(20, 3, levels=8)
    assert np.array_equal(W, W.T) and (np.diag(W) == 1).all()
    assert np.all(np.abs(W * 4 - np.round(W * 4)) == 0)
