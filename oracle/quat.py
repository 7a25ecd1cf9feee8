"""Quaternion and dual-quaternion algebra in FP64.

Quaternions are (w, x, y, z) arrays, the product is Hamilton's:
(a, u)(b, v) = (ab - u.v, a v + b u + u x v). A rigid transform x -> R x + t is
the unit dual quaternion r + eps d with r the rotation quaternion (stored with
w >= 0) and d = 1/2 (0, t) r, the representation the paper takes from Kavan
et al. for the node transforms (Sec. 3).
"""
from __future__ import annotations

import numpy as np

CONJ = np.array([1.0, -1.0, -1.0, -1.0])


def qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    w = a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], axis=-1)
    v = a[..., :1] * b[..., 1:] + b[..., :1] * a[..., 1:] + np.cross(a[..., 1:], b[..., 1:])
    return np.concatenate([w[..., None], v], axis=-1)


def qconj(q: np.ndarray) -> np.ndarray:
    return np.asarray(q, dtype=np.float64) * CONJ


def qleft(a: np.ndarray) -> np.ndarray:
    """4x4 matrix L(a) with a (x) b = L(a) b (batched over leading axes)."""
    a = np.asarray(a, dtype=np.float64)
    w, x, y, z = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    return np.stack([np.stack([w, -x, -y, -z], -1),
                     np.stack([x, w, -z, y], -1),
                     np.stack([y, z, w, -x], -1),
                     np.stack([z, -y, x, w], -1)], -2)


def qright(b: np.ndarray) -> np.ndarray:
    """4x4 matrix R(b) with a (x) b = R(b) a (batched over leading axes)."""
    b = np.asarray(b, dtype=np.float64)
    w, x, y, z = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([np.stack([w, -x, -y, -z], -1),
                     np.stack([x, w, z, -y], -1),
                     np.stack([y, -z, w, x], -1),
                     np.stack([z, y, -x, w], -1)], -2)


def pure(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], axis=-1)


def skew(v: np.ndarray) -> np.ndarray:
    """[v]x with [v]x a = v x a."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def matrix_from_quat(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a unit quaternion: R v = vec(q (0,v) q*)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def quat_from_matrix(R: np.ndarray) -> np.ndarray:
    """Unit quaternion of a rotation matrix (Shepperd's branch on the largest
    of w^2, x^2, y^2, z^2), returned with w >= 0."""
    R = np.asarray(R, dtype=np.float64)
    shp = R.shape[:-2]
    R = R.reshape(-1, 3, 3)
    out = np.empty((R.shape[0], 4))
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    cand = np.stack([tr, R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]], 1)
    k = np.argmax(cand, axis=1)
    for i in range(R.shape[0]):
        m = R[i]
        if k[i] == 0:
            s = 2.0 * np.sqrt(max(1.0 + tr[i], 0.0))
            q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k[i] == 1:
            s = 2.0 * np.sqrt(max(1.0 + m[0, 0] - m[1, 1] - m[2, 2], 0.0))
            q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k[i] == 2:
            s = 2.0 * np.sqrt(max(1.0 - m[0, 0] + m[1, 1] - m[2, 2], 0.0))
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = 2.0 * np.sqrt(max(1.0 - m[0, 0] - m[1, 1] + m[2, 2], 0.0))
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
        q = np.asarray(q)
        q /= np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        out[i] = q
    return out.reshape(shp + (4,))


def canonical(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, dtype=np.float64)
    return np.where(q[..., :1] < 0, -q, q)


def dq_from_rt(R: np.ndarray, t: np.ndarray):
    """(r, d) of x -> R x + t: r = quat(R) with w >= 0, d = 1/2 (0,t) r."""
    r = quat_from_matrix(R)
    d = 0.5 * qmul(pure(t), r)
    return r, d


def rt_from_dq(r: np.ndarray, d: np.ndarray):
    """Inverse of dq_from_rt for a unit dual quaternion: R = R(r), t = 2 vec(d r*)."""
    R = matrix_from_quat(r)
    t = 2.0 * qmul(d, qconj(r))[..., 1:]
    return R, t


def exp_so3(w: np.ndarray) -> np.ndarray:
    """Rotation matrix exp([w]x) by Rodrigues' formula; second-order Taylor
    series for angles below 1e-8."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1)
    K = skew(w)
    K2 = K @ K
    small = th < 1e-8
    ths = np.where(small, 1.0, th)
    a = np.where(small, 1.0, np.sin(ths) / ths)
    b = np.where(small, 0.5, (1.0 - np.cos(ths)) / (ths * ths))
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + a[..., None, None] * K + b[..., None, None] * K2


def se3_to_rt(se3: np.ndarray):
    M = np.asarray(se3, dtype=np.float64).reshape(-1, 3, 4)
    return M[:, :, :3].copy(), M[:, :, 3].copy()


def rt_to_se3(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([R, t[:, :, None]], axis=2).reshape(-1, 12)
