"""Depth-map fusion into the live surfels (Sec. 5 and Sec. 6.1) and the return
of fused surfels to the reference frame (Sec. 6.4). Test infrastructure only:
nothing in the product imports it.

Sec. 5 gives every pixel with a normal a depth surfel: position V(u), normal
N(u), confidence c = exp(-gamma^2 / (2 phi^2)) (phi = 0.6) and radius
r = sqrt(2) d / (f |n_z|), clamped for views more grazing than 75 degrees.
Sec. 6.1 renders the live surfels as unsized points into an index map
super-sampled 4x4 over the depth map, and gives each depth pixel at most one
live surfel from a 4x4 window: surfels farther than delta_distance from the
depth vertex or whose normal is not aligned (dot < delta_normal) are
discarded; of the rest the one with the highest confidence wins, then the
one closest to the depth surfel. The depth surfel is fused into it:
c += c_depth, t_observed = t_now, and v, n, r become confidence-weighted
means. Sec. 6.4 warps live surfels back to the reference frame.

Readings taken here (the paper leaves them open):
* gamma = |u - c| / |c|: the pixel's distance from the principal point
  c = (cx, cy), divided by the principal point's distance from the image
  corner (0, 0) (1 at that corner);
* f = fx; the radius clamp replaces |n_z| by max(|n_z|, cos 75 deg);
* the super-sampled pixel of a live point is (floor(4 hx), floor(4 hy)) with
  hx = fx (x / z) + cx + 1/2 (the depth pixel's own rule scaled by 4, so a
  point's sub-pixel lies in its depth pixel); winner: smallest (z, index)
  as in the solver's index map; every live surfel with a valid blend is
  rendered;
* the 4x4 window of depth pixel u is the block of sub-pixels that map to u;
  a depth pixel takes part only if it has a normal; distance gate
  |v - V(u)|^2 <= delta_distance^2, normal gate n . N(u) >= delta_normal;
  equal confidence and equal distance fall to the lower surfel index;
* the fused normal is renormalised (the weighted mean of unit normals is not
  unit, and the normals feed the correspondence gates of later frames);
* a fused surfel returns to the reference frame through the inverse of its
  own blended transform at the current warp field: v_ref = R^T (v' - t),
  n_ref = R^T n' (R, t of the normalised blend); its skinning is kept;
* depth pixels with a normal that find no surfel are reported as append
  candidates (Sec. 6.4); appending them is a step of its own.

Integer decisions (sub-pixel, winner, gates, selection) are taken in FP32 on
FP32 inputs (the live positions and normals handed in, as the GPU holds
them); attribute arithmetic is FP64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict

import numpy as np

from .quat import qconj, qmul

f32 = np.float32
PHI = 0.6
MAX_VIEW_DEG = 75.0


@dataclass
class FusionParams:
    delta_distance: float = 0.001     # Table 1
    delta_normal: float = 0.85        # Table 1
    phi: float = PHI


def depth_confidence(cam) -> np.ndarray:
    """(H, W) confidence exp(-gamma^2 / (2 phi^2)) of a depth surfel at each pixel."""
    ys, xs = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    gamma2 = ((xs - cam.cx) ** 2 + (ys - cam.cy) ** 2) / (cam.cx ** 2 + cam.cy ** 2)
    return np.exp(-gamma2 / (2.0 * PHI ** 2))


def depth_radius(depth: np.ndarray, N: np.ndarray, cam) -> np.ndarray:
    """(H, W) radius sqrt(2) d / (f |n_z|), |n_z| at least cos(75 deg)."""
    nz = np.maximum(np.abs(N[..., 2]), np.cos(np.deg2rad(MAX_VIEW_DEG)))
    return np.sqrt(2.0) * depth / (cam.fx * nz)


def subpixel(v32: np.ndarray, cam):
    """FP32 super-sampled pixel (sx, sy) of live points and whether it lies in
    the 4W x 4H map with z > 0."""
    v = v32.astype(f32)
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        hx = (f32(cam.fx) * (x / z) + f32(cam.cx)) + f32(0.5)
        hy = (f32(cam.fy) * (y / z) + f32(cam.cy)) + f32(0.5)
        inside = (z > f32(0)) & (hx >= f32(0)) & (hx < f32(cam.width)) & (hy >= f32(0)) & (hy < f32(cam.height))
        sx = np.floor(np.where(inside, f32(4) * hx, f32(0))).astype(np.int64)
        sy = np.floor(np.where(inside, f32(4) * hy, f32(0))).astype(np.int64)
    return sx, sy, inside


def index_map_4x(v32: np.ndarray, cam, valid: np.ndarray) -> np.ndarray:
    """(4H, 4W) map of the surfel with the smallest (FP32 z bits, index) per
    sub-pixel, -1 where none."""
    sx, sy, inside = subpixel(v32, cam)
    inside = inside & valid
    ids = np.flatnonzero(inside)
    W4 = 4 * cam.width
    pix = sy[ids] * W4 + sx[ids]
    zb = v32[ids, 2].astype(f32).view(np.uint32)
    order = np.lexsort((ids, zb, pix))
    ps = pix[order]
    first = np.ones(order.size, dtype=bool)
    first[1:] = ps[1:] != ps[:-1]
    I4 = np.full(W4 * 4 * cam.height, -1, dtype=np.int64)
    I4[ps[first]] = ids[order][first]
    return I4.reshape(4 * cam.height, W4)


def match(I4: np.ndarray, v32: np.ndarray, n32: np.ndarray, conf32: np.ndarray, depth: np.ndarray,
          N32: np.ndarray, nvalid: np.ndarray, cam, fp: FusionParams) -> np.ndarray:
    """(H, W) surfel fused at each depth pixel, -1 where none: the 16
    candidates of the pixel's 4x4 block, FP32 gates, then highest confidence,
    smallest squared distance, lowest index."""
    H, W = cam.height, cam.width
    cand = I4.reshape(H, 4, W, 4).transpose(0, 2, 1, 3).reshape(H, W, 16)
    ys, xs = np.mgrid[0:H, 0:W]
    D = depth.astype(f32)
    Vd = np.stack([((xs.astype(f32) - f32(cam.cx)) / f32(cam.fx)) * D,
                   ((ys.astype(f32) - f32(cam.cy)) / f32(cam.fy)) * D, D], axis=-1)
    has = cand >= 0
    c = np.where(has, cand, 0)
    v = v32.astype(f32)[c]
    n = n32.astype(f32)[c]
    with np.errstate(invalid="ignore", over="ignore"):
        dx = v[..., 0] - Vd[..., None, 0]
        dy = v[..., 1] - Vd[..., None, 1]
        dz = v[..., 2] - Vd[..., None, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        N = N32.astype(f32)
        dot = (n[..., 0] * N[..., None, 0] + n[..., 1] * N[..., None, 1]) + n[..., 2] * N[..., None, 2]
        ok = has & nvalid[..., None] & (d2 <= f32(fp.delta_distance) * f32(fp.delta_distance)) \
            & (dot >= f32(fp.delta_normal))
    conf = np.where(ok, conf32.astype(f32)[c], -np.inf)
    d2m = np.where(ok, d2, np.inf)
    idm = np.where(ok, cand, np.iinfo(np.int64).max)
    # lexicographic: max confidence, then min d2, then min index
    best = np.full((H, W), -1, dtype=np.int64)
    any_ok = ok.any(axis=-1)
    order = np.lexsort((idm, d2m, -conf), axis=-1)
    pick = np.take_along_axis(cand, order[..., :1], axis=-1)[..., 0]
    best[any_ok] = pick[any_ok]
    return best


def fuse(best: np.ndarray, v: np.ndarray, n: np.ndarray, r: np.ndarray, c: np.ndarray, t: np.ndarray,
         Vd: np.ndarray, Nd: np.ndarray, rd: np.ndarray, cd: np.ndarray, t_now: int) -> Dict[str, np.ndarray]:
    """Fused live attributes (FP64) of the surfels chosen by `best`; the
    other surfels keep theirs. Vd, Nd, rd, cd: (H, W, ...) depth surfels."""
    v = np.array(v, dtype=np.float64)
    n = np.array(n, dtype=np.float64)
    r = np.array(r, dtype=np.float64)
    c = np.array(c, dtype=np.float64)
    t = np.array(t, dtype=np.int64)
    ys, xs = np.nonzero(best >= 0)
    s = best[ys, xs]
    assert np.unique(s).size == s.size, "a surfel was chosen by two pixels"
    c_old, c_d = c[s], cd[ys, xs]
    c_new = c_old + c_d
    v[s] = (c_old[:, None] * v[s] + c_d[:, None] * Vd[ys, xs]) / c_new[:, None]
    nn = (c_old[:, None] * n[s] + c_d[:, None] * Nd[ys, xs]) / c_new[:, None]
    n[s] = nn / np.linalg.norm(nn, axis=1, keepdims=True)
    r[s] = (c_old * r[s] + c_d * rd[ys, xs]) / c_new
    c[s] = c_new
    t[s] = t_now
    fused = np.zeros(v.shape[0], dtype=bool)
    fused[s] = True
    return dict(v=v, n=n, r=r, c=c, t=t, fused=fused)


def to_reference(b: np.ndarray, v_live: np.ndarray, n_live: np.ndarray):
    """Inverse of the normalised blend: v = R^T (v' - t), n = R^T n'."""
    b = np.asarray(b, dtype=np.float64)
    c = b / np.linalg.norm(b[:, :4], axis=1, keepdims=True)
    cr = c[:, :4]
    t = 2.0 * qmul(c[:, 4:], qconj(cr))[:, 1:]

    def rot_inv(x):
        q = np.concatenate([np.zeros((x.shape[0], 1)), x], axis=1)
        return qmul(qmul(qconj(cr), q), cr)[:, 1:]

    return rot_inv(np.asarray(v_live, np.float64) - t), rot_inv(np.asarray(n_live, np.float64))
