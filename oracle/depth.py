"""Vertex and normal maps of a depth image in FP64 (Sec. 5).

V(u) = D(u) K^-1 (u^T, 1)^T; the normal at u is estimated from V by central
differences. Readings (the paper gives no filter and no edge rule): a pixel's
normal is defined when the pixel is not on the image border, it and its four
neighbours hold a depth, no neighbour's depth differs from it by more than
edge_gate, and the cross product is nonzero; the normal is oriented towards the
camera. Which pixels have a normal is an integer decision and comes from
`replica32.normal_map`; this module gives the FP64 values.
"""
from __future__ import annotations

import numpy as np


def vertex_map(depth: np.ndarray, cam) -> np.ndarray:
    D = depth.astype(np.float64)
    H, W = D.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    D = np.where(np.isfinite(D) & (D > 0), D, 0.0)
    return np.stack([(xs - cam.cx) / cam.fx * D, (ys - cam.cy) / cam.fy * D, D], axis=-1)


def normal_map(depth: np.ndarray, cam) -> np.ndarray:
    """FP64 unit normals normalize((V(x,y+1)-V(x,y-1)) x (V(x+1,y)-V(x-1,y))),
    negated when they face away from the camera; zero on the border and where
    the cross product vanishes. Validity is decided separately (FP32)."""
    V = vertex_map(depth, cam)
    H, W = depth.shape
    N = np.zeros((H, W, 3))
    if H < 3 or W < 3:
        return N
    a = V[2:, 1:-1] - V[:-2, 1:-1]
    b = V[1:-1, 2:] - V[1:-1, :-2]
    c = np.cross(a, b)
    ln = np.linalg.norm(c, axis=-1, keepdims=True)
    n = np.where(ln > 0, c / np.where(ln > 0, ln, 1.0), 0.0)
    flip = np.sum(n * V[1:-1, 1:-1], axis=-1) > 0
    n[flip] = -n[flip]
    N[1:-1, 1:-1] = n
    return N
