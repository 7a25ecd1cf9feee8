"""Nearest-node skinning and the node graph (brute force).

Sec. 6.5 (Initialization): after the nodes are sub-sampled from the reference
surfels, every surfel is skinned to its nearest nodes in the reference frame,
and the node-graph edges are computed. Sec. 3: the blend weight of node k at x
is exp(-|x - p_k|^2 / (2 sigma_k^2)), sigma_k the node radius (Table 1:
2.5 cm, the node sampling distance).

Readings taken here: K = 4 nearest nodes per surfel, 8 nearest other nodes per
node (a directed graph), exact search instead of the approximate search the
paper uses, and one sigma for every node. The order of nearest nodes is the
ascending FP32 key of `replica32.sqdist_key` with ties going to the lower node
index; the weights themselves are FP64.
"""
from __future__ import annotations

import numpy as np

from . import replica32


def knn_fp32(query: np.ndarray, nodes: np.ndarray, k: int, exclude_self: bool = False,
             chunk: int = 8192) -> np.ndarray:
    """Indices of the k nodes with the smallest FP32 key, ties to the lower
    index, sorted by (key, index). With exclude_self, query i skips node i."""
    nq, nn = query.shape[0], nodes.shape[0]
    if k > nn - (1 if exclude_self else 0):
        raise ValueError("not enough nodes")
    out = np.empty((nq, k), dtype=np.int64)
    for s in range(0, nq, chunk):
        e = min(nq, s + chunk)
        key = replica32.sqdist_key(query[s:e], nodes)
        if exclude_self:
            key[np.arange(e - s), np.arange(s, e)] = np.float32(np.inf)
        kth = np.partition(key, k - 1, axis=1)[:, k - 1]
        mask = key <= kth[:, None]
        cnt = mask.sum(axis=1)
        plain = np.flatnonzero(cnt == k)
        if plain.size:
            cols = np.nonzero(mask[plain])[1].reshape(plain.size, k)  # ascending index
            kv = np.take_along_axis(key[plain], cols, axis=1)
            o = np.argsort(kv, axis=1, kind="stable")
            out[s + plain] = np.take_along_axis(cols, o, axis=1)
        for r in np.flatnonzero(cnt != k):
            o = np.argsort(key[r], kind="stable")
            out[s + r] = o[:k]
    return out


def skin_weights(query: np.ndarray, nodes: np.ndarray, idx: np.ndarray, sigma: float) -> np.ndarray:
    """Normalised FP64 weights w_k / sum(w), w_k = exp(-|x - p_k|^2 / (2 sigma^2)),
    evaluated as exp(-(d_k^2 - d_0^2) / (2 sigma^2)) (the common factor
    exp(-d_0^2/(2 sigma^2)) cancels in the normalisation)."""
    q = query.astype(np.float64)
    p = nodes.astype(np.float64)[idx]
    d2 = np.sum((p - q[:, None, :]) ** 2, axis=-1)
    e = np.exp(-(d2 - d2[:, :1]) / (2.0 * sigma * sigma))
    return e / e.sum(axis=1, keepdims=True)


def skinning(surfel_pos: np.ndarray, node_pos: np.ndarray, sigma: float, K: int = 4):
    idx = knn_fp32(surfel_pos, node_pos, K)
    w = skin_weights(surfel_pos, node_pos, idx, sigma)
    return idx, w


def node_graph(node_pos: np.ndarray, k: int = 8) -> np.ndarray:
    """N_j: the k nearest other nodes of node j (directed, as written in the
    regulariser of Sec. 7, which sums over j and i in N_j)."""
    return knn_fp32(node_pos, node_pos, k, exclude_self=True)
