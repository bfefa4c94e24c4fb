"""DBHT clustering (host-side, tmfg_dbht) and its oracle: a hand-derived 6-vertex case, the
shortest paths against Floyd-Warshall, complete linkage against scipy, the ARI against the
textbook cases and scikit-learn, the bubble tree's invariants, and the library against the
oracle on random, tie-heavy and planted-cluster inputs. The library's DBHT runs on the host,
so these tests need no GPU."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import dbht as dh
import paper_2408_09399_amd as tm
from paper_2408_09399_amd import synth


def _hand_case():
    """n = 6: seed 0,1,2,3; vertex 4 joins face 0 = (0,1,2); vertex 5 joins face 0 = (0,1,4).
    Weights take the values 0.875, 0.5 and -1, whose edge lengths sqrt(2 (1 - w)) are exactly
    0.5, 1 and 2, so every path sum below is exact."""
    n = 6
    W = np.zeros((n, n), dtype=np.float32)
    np.fill_diagonal(W, 1.0)
    w = {(0, 1): 0.875, (0, 2): 0.5, (0, 3): 0.875, (1, 2): 0.5, (1, 3): 0.875, (2, 3): 0.875,
         (0, 4): 0.5, (1, 4): 0.5, (2, 4): -1.0, (0, 5): 0.5, (1, 5): 0.5, (4, 5): 0.875}
    for (a, b), v in w.items():
        W[a, b] = W[b, a] = v
    rec = {"order": np.array([0, 1, 2, 3, 4, 5]),
           "edges": np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3],
                              [4, 0], [4, 1], [4, 2], [5, 0], [5, 1], [5, 4]]),
           "steps": np.array([[0, 0, 1, 2], [0, 0, 1, 4]])}
    return W, rec


def test_hand_case():
    """Bubbles B0 = {0,1,2,3}, B1 = {0,1,2,4} (parent B0, triangle 0,1,2), B2 = {0,1,4,5}
    (parent B1, triangle 0,1,4).
    B0-B1: child side {4,5}: W 0-4, 0-5, 1-4, 1-5, 2-4 = 0.5+0.5+0.5+0.5-1 = 1.0; parent side {3}:
    0-3, 1-3, 2-3 = 2.625 -> towards B0. B1-B2: child side {5}: 0-5, 1-5, 4-5 = 1.875; parent
    side {2,3}: 0-2, 0-3, 1-2, 1-3, 4-2 = 0.5+0.875+0.5+0.875-1 = 1.75 -> towards B2. Converging:
    B0 and B2; B1 reaches both.
    Groups: 0 and 1 weigh 2.25 to B0 against 1.875 to B2; 2 weighs 1.875 to B0 and 0 to B2;
    3 only reaches B0; 4 weighs 0 to B0 and 1.875 to B2; 5 only reaches B2.
    Path lengths: d01 .5, d02 1, d03 .5, d12 1, d13 .5, d23 .5, d04 d05 d14 d15 1, d24 d25 2,
    d34 d35 1.5, d45 .5. Bubbles: 0 and 1 sum 2.0 to B0 against 2.5 to B1; 2 sums 2.5 to B0
    against 4 to B1; 4 sums 2.5 to B2 against 4 to B1.
    Linkage: cell {0,1,2,3}: pairs at 0.5 are (0,1), (0,3), (1,3), (2,3): (0,1) first -> 6;
    then (2,3) at 0.5 before (3,6) -> 7; then (6,7) at 1 -> 8. Cell {4,5} at 0.5 -> 9. Groups:
    largest cross distance d24 = 2 -> 10."""
    W, rec = _hand_case()
    bubbles, parent, tri, creator = dh.bubble_tree(rec["order"], rec["steps"])
    assert bubbles == [(0, 1, 2, 3), (0, 1, 2, 4), (0, 1, 4, 5)]
    assert parent == [-1, 0, 1]
    to_child = dh.directions(W, rec["edges"], bubbles, parent, tri, creator)
    assert to_child[1:] == [False, True]
    sinks, reach = dh.converging(bubbles, parent, to_child)
    assert sinks == [0, 2] and reach == [[0], [0, 2], [2]]
    Z = [[0, 1, 0.5, 2], [2, 3, 0.5, 2], [6, 7, 1.0, 4], [4, 5, 0.5, 2], [8, 9, 2.0, 6]]
    cuts = {1: [0] * 6, 2: [0, 0, 0, 0, 1, 1], 3: [0, 0, 0, 0, 1, 2], 4: [0, 0, 1, 1, 2, 3]}
    for k, want in cuts.items():
        for got in (dh.dbht(W, rec, k), tm.dbht(W, rec["order"], rec["edges"], rec["steps"], k)):
            assert np.asarray(got["group"]).tolist() == [0, 0, 0, 0, 2, 2]
            assert np.asarray(got["bubble"]).tolist() == [0, 0, 0, 0, 2, 2]
            assert np.asarray(got["linkage"]).tolist() == Z
            assert np.asarray(got["labels"]).tolist() == want


def _tmfg(n, seed, grid=False):
    W = synth.grid_symmetric(n, seed, levels=[2, 4, 8][seed % 3]) if grid else synth.random_symmetric(n, seed)
    return W, oracle.tmfg_lazy(W)


@pytest.mark.parametrize("seed", range(6))
def test_shortest_paths(seed):
    n = 5 + 7 * seed
    W, r = _tmfg(n, 900 + seed)
    D = dh.apsp(W, r["edges"])
    assert np.array_equal(D, dh.apsp_plain(W, r["edges"]))
    # Floyd-Warshall sums paths in another order: equal up to rounding
    ln = dh.edge_lengths(W, r["edges"])
    F = np.full((n, n), np.inf)
    np.fill_diagonal(F, 0.0)
    for (a, b), l in zip(r["edges"].tolist(), ln.tolist()):
        F[a, b] = F[b, a] = l
    for k in range(n):
        F = np.minimum(F, F[:, k:k + 1] + F[k:k + 1, :])
    np.testing.assert_allclose(D, F, rtol=1e-12, atol=1e-12)
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)


@pytest.mark.parametrize("seed", range(5))
def test_complete_linkage_against_scipy(seed):
    from scipy.cluster.hierarchy import linkage
    from scipy.spatial.distance import pdist, squareform
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((12 + 5 * seed, 3))
    d = pdist(P)
    rows, next_id, top = dh.complete_linkage(squareform(d), list(range(P.shape[0])), P.shape[0],
                                             [1] * P.shape[0])
    Zs = linkage(d, method="complete")
    mine = np.asarray(rows, dtype=np.float64)
    want = np.column_stack([np.sort(Zs[:, :2], axis=1), Zs[:, 3]])
    assert np.array_equal(mine[:, [0, 1, 3]], want)
    np.testing.assert_array_equal(mine[:, 2], Zs[:, 2])
    assert top == 2 * P.shape[0] - 2


def test_ari():
    assert dh.ari([0, 0, 1, 1], [5, 5, 7, 7]) == 1.0
    # the classic example: ARI of (1,1,2,2,3,3) against (1,1,2,3,3,3)
    # n_ij table [[2,0,0],[0,1,1],[0,0,2]]: sum C(n_ij,2) = 2, rows 3, cols 4, C(6,2) = 15:
    # (2 - 12/15) / (3.5 - 12/15) = 1.2 / 2.7
    assert dh.ari([1, 1, 2, 2, 3, 3], [1, 1, 2, 3, 3, 3]) == pytest.approx(1.2 / 2.7, abs=1e-15)
    from sklearn.metrics import adjusted_rand_score
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 5, 60)
        b = rng.integers(0, 4, 60)
        assert dh.ari(a, b) == pytest.approx(adjusted_rand_score(a, b), abs=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_bubble_tree_invariants(seed):
    n = 4 + 9 * seed
    W, r = _tmfg(n, 300 + seed, grid=seed % 2 == 1)
    bubbles, parent, tri, creator = dh.bubble_tree(r["order"], r["steps"])
    assert len(bubbles) == n - 3
    E = {tuple(sorted(e)) for e in r["edges"].tolist()}
    for k, b in enumerate(bubbles):
        assert all(tuple(sorted(p)) in E for p in itertools.combinations(b, 2))     # a 4-clique
        if k:
            assert 0 <= parent[k] < k
            assert set(tri[k]) <= set(b) and set(tri[k]) <= set(bubbles[parent[k]])
    to_child = dh.directions(W, r["edges"], bubbles, parent, tri, creator)
    sinks, reach = dh.converging(bubbles, parent, to_child)
    assert sinks and all(reach[s] == [s] for s in sinks)
    assert all(set(reach[k]) <= set(sinks) and reach[k] for k in range(len(bubbles)))


@pytest.mark.parametrize("seed", range(24))
def test_library_equals_oracle(seed):
    n = 4 + (seed * 11) % 110
    W, r = _tmfg(n, 700 + seed, grid=seed % 2 == 1)
    k = 1 + seed % min(n, 7)
    o = dh.dbht(W, r, k)
    g = tm.dbht(W, r["order"], r["edges"], r["steps"], k, n_threads=1 + seed % 4)
    for key in ("labels", "group", "bubble", "linkage"):
        assert np.array_equal(np.asarray(o[key]), np.asarray(g[key])), key


def test_planted_clusters_c1():
    s = synth.config_c1()
    W = oracle.pearson64(s.X).astype(np.float32)
    r = oracle.tmfg_lazy(W)
    k = len(set(s.labels.tolist()))
    o = dh.dbht(W, r, k)
    g = tm.dbht(W, r["order"], r["edges"], r["steps"], k)
    for key in ("labels", "group", "bubble", "linkage"):
        assert np.array_equal(np.asarray(o[key]), np.asarray(g[key])), key
    # five well-separated planted clusters of 40 are recovered
    assert dh.ari(s.labels, g["labels"]) > 0.9


def test_argument_errors():
    lib = tm.binding.lib()
    W, rec = _hand_case()
    labels = np.empty(6, np.int32)
    Wp = W.ctypes.data
    o = np.ascontiguousarray(rec["order"], np.int32)
    e = np.ascontiguousarray(rec["edges"], np.int32)
    st = np.ascontiguousarray(rec["steps"], np.int32)
    call = lambda n, k, order=o: lib.tmfg_dbht(n, Wp, order.ctypes.data, e.ctypes.data, st.ctypes.data, k, 1,
                                               labels.ctypes.data, None, None, None)
    assert call(6, 2) == 0
    assert call(3, 1) == 2
    assert call(6, 0) == 2 and call(6, 7) == 2
    bad = o.copy()
    bad[5] = 4                                       # not a permutation
    assert call(6, 2, bad) == 1
    assert lib.tmfg_dbht(6, None, o.ctypes.data, e.ctypes.data, st.ctypes.data, 2, 1, labels.ctypes.data,
                         None, None, None) == 1
