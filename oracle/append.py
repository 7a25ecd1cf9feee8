"""Append candidates after fusion: live-frame skinning of depth surfels with
the consistency filter (Sec. 6.2, Eq. 7), the compressive-warp test
(Sec. 6.3, Eq. 8) and the weight-sum test of surfel appending (Sec. 6.4),
then the warp back to the reference frame. Test infrastructure only: nothing
in the product imports it.

Sec. 6.2: a depth surfel that fusion matched to no live surfel is skinned to
its nearest nodes of the node graph warped to the live frame; node i of that
set stays only if its live distance to the nearest node, divided by their
reference distance, lies strictly between 1 - eps and 1 + eps (eps = 0.2,
Table 1). Sec. 6.3: a surfel is dropped where the warp back to the
reference frame stretches by more than 1 + eps, the 3x3 derivative
d x_ref / d x_live taken by finite differences. Sec. 6.4: a surfel is dropped
where the sum of its nearest-neighbour weights is below delta_nn.

Readings taken here (the paper leaves them open):
* candidates are the depth pixels with a normal that fusion matched to no live
  surfel; the depth surfel is V(u), N(u) of the frame (FP32 back-projection);
* the live-frame set is the K = 4 nearest live node positions c_j = T_j p_j
  (FP32 key, ties to the lower index, as the reference skinning); the nearest
  one is always kept; the ratio test is taken on squares in FP32,
  (1 - eps)^2 |p_i - p_0|^2 < |c_i - c_0|^2 < (1 + eps)^2 |p_i - p_0|^2;
* weights are the Gaussian exp(-|x - c_j|^2 / (2 sigma^2)) of the kept nodes
  (sigma the node radius); delta_nn compares their plain (unnormalised) sum,
  and its value, which the paper does not give, is 0.3 by default;
* the warp back is the inverse of the normalised blend of the kept nodes'
  transforms with the normalised weights, v_ref = R^T (v - t), n_ref = R^T n;
* the derivative is the central difference with step h = 1 mm along each
  axis, the kept node set fixed and the weights re-evaluated at the offset
  point; "|d x_ref / d x_live|" in 3D is read as its largest singular value
  (the largest stretch of any direction);
* appended surfels carry the depth surfel's radius and confidence (Sec. 5),
  t_init = t_observed = t_now, and come in row-major pixel order;
* an existing surfel is dropped when its confidence is below delta_stable and
  more than t_low_confid frames have passed since its t_init (Table 1: 10 and
  30); the updated surfel array holds the kept surfels in their order, then
  the appended ones (the compaction the complexity paragraph of Sec. 6.7
  describes); the second removal rule (similarity to index-map neighbours) is
  a criterion of Keller et al. the paper does not restate and is not taken.

Integer decisions that have an exact FP32 form (nearest nodes, the ratio test)
are taken in FP32 on the FP32 live node positions handed in, as the GPU holds
them; the weight sum, the warp back and the stretch are FP64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import replica32 as R32
from .fusion import depth_confidence, depth_radius, to_reference
from .skin import knn_fp32
from .warp import blend

f32 = np.float32
FD_STEP = 1e-3


@dataclass
class AppendParams:
    sigma: float = 0.025          # node radius (Table 1)
    eps: float = 0.2              # intrinsic deformation bound (Table 1)
    delta_nn: float = 0.3         # weight-sum threshold (not given by the paper)


def live_skinning(V32: np.ndarray, live32: np.ndarray, ref32: np.ndarray, eps: float):
    """Nearest 4 live nodes of each point and which of them pass the
    consistency test (the nearest always does)."""
    idx = knn_fp32(V32, live32, 4)
    c = live32.astype(f32)[idx]
    p = ref32.astype(f32)[idx]

    def key(a, b):
        dx = a[..., 0] - b[..., 0]
        dy = a[..., 1] - b[..., 1]
        dz = a[..., 2] - b[..., 2]
        return (dx * dx + dy * dy) + dz * dz

    d_live = key(c, c[:, :1])
    d_ref = key(p, p[:, :1])
    lo = f32(1) - f32(eps)
    hi = f32(1) + f32(eps)
    keep = (lo * lo * d_ref < d_live) & (d_live < hi * hi * d_ref)
    keep[:, 0] = True
    return idx, keep


def weights(x: np.ndarray, live: np.ndarray, idx: np.ndarray, keep: np.ndarray, sigma: float) -> np.ndarray:
    """Unnormalised Gaussian weights of the kept nodes (0 for the others)."""
    d2 = np.sum((np.asarray(x, np.float64)[:, None, :] - live.astype(np.float64)[idx]) ** 2, axis=-1)
    return np.where(keep, np.exp(-d2 / (2.0 * sigma * sigma)), 0.0)


def warp_back(x: np.ndarray, n: np.ndarray | None, live: np.ndarray, node_r: np.ndarray, node_d: np.ndarray,
              idx: np.ndarray, keep: np.ndarray, sigma: float):
    """Reference position (and normal) of live points through the inverse of
    the blend of their kept nodes, weights evaluated at the points."""
    w = weights(x, live, idx, keep, sigma)
    w = w / w.sum(axis=1, keepdims=True)
    b, _ = blend(idx, w, node_r, node_d)
    nn = np.zeros_like(x) if n is None else n
    return to_reference(b, x, nn)


def stretch(x: np.ndarray, live, node_r, node_d, idx, keep, sigma, h: float = FD_STEP):
    """Largest singular value of d x_ref / d x_live by central differences."""
    x = np.asarray(x, np.float64)
    F = np.empty((x.shape[0], 3, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        xp, _ = warp_back(x + e, None, live, node_r, node_d, idx, keep, sigma)
        xm, _ = warp_back(x - e, None, live, node_r, node_d, idx, keep, sigma)
        F[:, :, a] = (xp - xm) / (2.0 * h)
    return np.linalg.svd(F, compute_uv=False)[:, 0], F


def append_candidates(match: np.ndarray, depth: np.ndarray, N32: np.ndarray, nvalid: np.ndarray, cam,
                      live32: np.ndarray, ref32: np.ndarray, node_r: np.ndarray, node_d: np.ndarray,
                      ap: AppendParams):
    """Every stage of the append selection for one fused frame.

    match: (H, W) fused surfel per pixel or -1; N32, nvalid: the FP32 normal
    map; live32 / ref32: live and reference node positions (FP32); node_r,
    node_d: the nodes' dual quaternions (FP64)."""
    H, W = cam.height, cam.width
    cand = nvalid & (np.asarray(match) < 0)
    ys, xs = np.nonzero(cand)                    # row-major
    D = depth.astype(f32)
    V32 = R32.backproject(xs, ys, D[ys, xs], cam)
    Nd = N32[ys, xs].astype(np.float64)
    idx, keep = live_skinning(V32, live32, ref32, ap.eps)
    V = V32.astype(np.float64)
    S = weights(V, live32, idx, keep, ap.sigma).sum(axis=1)
    near = S >= ap.delta_nn
    smax = np.full(V.shape[0], np.nan)
    vref = np.full_like(V, np.nan)
    nref = np.full_like(V, np.nan)
    if near.any():
        sel = np.flatnonzero(near)
        smax[sel], _ = stretch(V[sel], live32, node_r, node_d, idx[sel], keep[sel], ap.sigma)
        vref[sel], nref[sel] = warp_back(V[sel], Nd[sel], live32, node_r, node_d, idx[sel], keep[sel], ap.sigma)
    compressive = near & (smax > 1.0 + ap.eps)
    ok = near & ~compressive
    rd = depth_radius(depth.astype(np.float64), N32.astype(np.float64), cam)[ys, xs]
    cd = depth_confidence(cam)[ys, xs]
    return dict(pixel=ys * W + xs, idx=idx, keep=keep, S=S, near=near, stretch=smax, compressive=compressive,
                ok=ok, v_ref=vref, n_ref=nref, radius=rd, conf=cd)


def unstable(conf: np.ndarray, t_init: np.ndarray, t_now: int, stable_conf: float, t_low_confid: int) -> np.ndarray:
    """Surfels removed by the geometry update: confidence below delta_stable
    (FP32 comparison) more than t_low_confid frames after initialisation."""
    c = np.asarray(conf, np.float32)
    return (c < np.float32(stable_conf)) & (int(t_now) - np.asarray(t_init, np.int64) > int(t_low_confid))


def update_surfels(pos, nrm, rad, conf, t_obs, t_init, keep, app: dict, t_now: int):
    """The updated surfel array: kept surfels in order, then the appended ones."""
    ok = app["ok"]
    n_app = int(ok.sum())
    cat = lambda a, b: np.concatenate([np.asarray(a)[keep], b])
    return dict(pos=cat(pos, app["v_ref"][ok]), nrm=cat(nrm, app["n_ref"][ok]), radius=cat(rad, app["radius"][ok]),
                conf=cat(conf, app["conf"][ok]), t_obs=cat(t_obs, np.full(n_app, t_now)),
                t_init=cat(t_init, np.full(n_app, t_now)))
