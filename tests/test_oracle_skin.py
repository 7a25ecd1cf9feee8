"""Pins of nearest-node skinning and the node graph."""
import numpy as np
from scipy.spatial import cKDTree

from oracle import replica32, skin


def test_knn_matches_kdtree(scene_cache):
    s = scene_cache("c1")
    idx = skin.knn_fp32(s.surfel_pos, s.node_pos, 4)
    d64, i64 = cKDTree(s.node_pos.astype(np.float64)).query(s.surfel_pos.astype(np.float64), k=4)
    same = np.all(idx == i64, axis=1)
    # FP32 and FP64 orders may differ only at near-ties
    bad = np.flatnonzero(~same)
    key = replica32.sqdist_key(s.surfel_pos[bad], s.node_pos)
    for row, b in enumerate(bad):
        kk = np.sort(key[row])[:5]
        gaps = np.diff(kk)
        assert np.min(gaps) <= 1e-6 * kk[-1], (b, kk)
    assert bad.size <= 1e-3 * idx.shape[0]


def test_knn_tie_break_brute_force():
    # nodes on a lattice with a query at equal distance from several of them
    g = np.array([[x, y, 0.0] for x in (-1, 0, 1) for y in (-1, 0, 1)], dtype=np.float32)
    perm = np.random.default_rng(0).permutation(len(g))
    nodes = g[perm]
    q = np.array([[0.0, 0.0, 0.5], [0.5, 0.5, 0.0], [1.0, 1.0, 0.0]], dtype=np.float32)
    got = skin.knn_fp32(q, nodes, 4)
    key = replica32.sqdist_key(q, nodes)
    for i in range(q.shape[0]):
        ref = [j for _, j in sorted((float(key[i, j]), j) for j in range(len(nodes)))][:4]
        assert list(got[i]) == ref


def test_knn_random_brute_force():
    rng = np.random.default_rng(1)
    # coarse coordinates produce many exact FP32 key ties
    nodes = (rng.integers(0, 6, size=(40, 3)) * 0.25).astype(np.float32)
    q = (rng.integers(0, 12, size=(300, 3)) * 0.125).astype(np.float32)
    got = skin.knn_fp32(q, nodes, 4)
    key = replica32.sqdist_key(q, nodes)
    for i in range(q.shape[0]):
        ref = [j for _, j in sorted((float(key[i, j]), j) for j in range(len(nodes)))][:4]
        assert list(got[i]) == ref


def test_node_graph_excludes_self_and_matches_kdtree(scene_cache):
    s = scene_cache("c1")
    nbr = skin.node_graph(s.node_pos)
    assert nbr.shape == (200, 8)
    assert not np.any(nbr == np.arange(200)[:, None])
    _, i64 = cKDTree(s.node_pos.astype(np.float64)).query(s.node_pos.astype(np.float64), k=9)
    agree = np.mean(np.all(nbr == i64[:, 1:], axis=1))
    assert agree > 0.98


def test_weights_closed_form():
    rng = np.random.default_rng(2)
    nodes = rng.normal(size=(10, 3)).astype(np.float32) * 0.05
    q = rng.normal(size=(20, 3)).astype(np.float32) * 0.05
    idx = skin.knn_fp32(q, nodes, 4)
    sigma = 0.025
    w = skin.skin_weights(q, nodes, idx, sigma)
    # plain definition: w_k = exp(-|x-p_k|^2/(2 sigma^2)) normalised
    raw = np.exp(-np.sum((nodes[idx].astype(np.float64) - q[:, None].astype(np.float64)) ** 2, -1)
                 / (2 * sigma ** 2))
    assert np.allclose(w, raw / raw.sum(1, keepdims=True), rtol=1e-12, atol=1e-300)
    assert np.allclose(w.sum(1), 1.0)
    assert np.all(np.diff(w, axis=1) <= 1e-15)   # nearest first -> non-increasing
