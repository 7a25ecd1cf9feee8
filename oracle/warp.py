"""Dual-quaternion blend of the nearest nodes and its derivatives (FP64).

Sec. 3, Eq. 1: W(x) = normalized(sum_k w_k(x) q_k) over the nearest nodes of
x; Eq. 2: v_live = W(v_ref) v_ref and n_live = rotation(W(v_ref)) n_ref.

Readings (Kavan et al.'s dual-quaternion blending, which the paper cites for
the node representation): each node's quaternion is flipped into the
hemisphere of the surfel's nearest node before blending (q and -q are the same
transform); "normalized" divides by the norm of the real part; the
translation of the normalised blend c = c_r + eps c_d is 2 vec(c_d c_r*)
(the scalar part of c_d c_r*, nonzero when c_d is not orthogonal to c_r, is
dropped). A blend with |b_r|^2 < 1e-12 leaves the surfel undefined.

Written out, with the blend b = b_r + eps b_d and V = (0, v):

    F(b; v) = [vec(b_r V b_r*) + 2 vec(b_d b_r*)] / |b_r|^2

F is homogeneous of degree 0 in b, which is why the weights need no
normalisation and the hemisphere choice of the reference node is irrelevant.
"""
from __future__ import annotations

import numpy as np

from .quat import CONJ, pure, qconj, qleft, qmul, qright, skew

VALID_EPS = 1e-12


def blend(idx: np.ndarray, w: np.ndarray, node_r: np.ndarray, node_d: np.ndarray):
    """b_i = sum_k w_ik s_ik q_{idx_ik}, s_ik = +1 if <r_{idx_i0}, r_{idx_ik}> >= 0
    else -1. Returns b (N,8) and the signs s (N,K)."""
    r = node_r[idx]                       # (N,K,4)
    d = node_d[idx]
    dots = np.sum(r * r[:, :1, :], axis=-1)
    s = np.where(dots >= 0, 1.0, -1.0)
    ws = (w * s)[..., None]
    br = np.sum(ws * r, axis=1)
    bd = np.sum(ws * d, axis=1)
    return np.concatenate([br, bd], axis=-1), s


def apply_blend(b: np.ndarray, v: np.ndarray, n: np.ndarray | None = None):
    """Warp points (and normals) by the normalised blend.

    c = b / |b_r|, c_r = (c0, u): v' = v + 2 c0 (u x v) + 2 u x (u x v)
    + 2 vec(c_d c_r*), n' = n + 2 c0 (u x n) + 2 u x (u x n).
    Returns v', n' (or None) and the validity mask."""
    b = np.asarray(b, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    br2 = np.sum(b[:, :4] ** 2, axis=1)
    valid = br2 >= VALID_EPS
    nr = np.sqrt(np.where(valid, br2, 1.0))
    c = b / nr[:, None]
    c0, u = c[:, 0:1], c[:, 1:4]

    def rot(x):
        ux = np.cross(u, x)
        return x + 2.0 * c0 * ux + 2.0 * np.cross(u, ux)

    t = 2.0 * qmul(c[:, 4:], qconj(c[:, :4]))[:, 1:]
    vl = rot(v) + t
    nl = rot(np.asarray(n, dtype=np.float64)) if n is not None else None
    return vl, nl, valid


def F_homogeneous(b: np.ndarray, v: np.ndarray) -> np.ndarray:
    """F(b; v) in the homogeneous (quotient) form."""
    br, bd = b[:, :4], b[:, 4:]
    V = pure(v)
    num = qmul(qmul(br, V), qconj(br))[:, 1:] + 2.0 * qmul(bd, qconj(br))[:, 1:]
    return num / np.sum(br * br, axis=1)[:, None]


def dF_db(b: np.ndarray, v: np.ndarray) -> np.ndarray:
    """3x8 derivative of F(b; v) with respect to b = (b_r, b_d), by the
    quotient rule on N(b) / D(b):

      dN/db_r = rows 1..3 of R(V b_r*) + L(b_r V) C + 2 L(b_d) C
      dN/db_d = rows 1..3 of 2 R(b_r*)
      dD/db_r = 2 b_r^T,  dD/db_d = 0
      dF/db   = (dN/db - F dD/db) / D

    with C = diag(1,-1,-1,-1) the conjugation (d(x*) = C dx)."""
    b = np.asarray(b, dtype=np.float64)
    br, bd = b[:, :4], b[:, 4:]
    V = pure(v)
    C = np.diag(CONJ)
    brc = qconj(br)
    dN_dbr = qright(qmul(V, brc)) + qleft(qmul(br, V)) @ C + 2.0 * (qleft(bd) @ C)
    dN_dbd = 2.0 * qright(brc)
    D = np.sum(br * br, axis=1)
    F = F_homogeneous(b, v)
    dD_dbr = 2.0 * br
    J = np.zeros((b.shape[0], 3, 8))
    J[:, :, :4] = dN_dbr[:, 1:, :] - F[:, :, None] * dD_dbr[:, None, :]
    J[:, :, 4:] = dN_dbd[:, 1:, :]
    return J / D[:, None, None]


def perturb_matrix(r: np.ndarray, d: np.ndarray, c: np.ndarray) -> np.ndarray:
    """8x6 matrix of the first-order change of a node's dual quaternion under
    the node-centred left perturbation x -> Exp(w)(x - c) + c + tau of its
    transform (c = the node's live position):

      dq = [(0, w/2) r] + eps [(0, w/2) d + (0, (tau - w x c)/2) r]

    Columns: (w, tau)."""
    Rr = qright(r)[:, :, 1:]               # (N,4,3): maps a 3-vector a to (0,a) r
    Rd = qright(d)[:, :, 1:]
    M = np.zeros((r.shape[0], 8, 6))
    M[:, :4, :3] = 0.5 * Rr
    M[:, 4:, :3] = 0.5 * Rd + 0.5 * (Rr @ skew(c))   # tau - w x c = tau + [c]x w
    M[:, 4:, 3:] = 0.5 * Rr
    return M
