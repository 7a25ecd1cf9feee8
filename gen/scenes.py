"""Seeded synthetic depth scenes for the per-frame warp-field solve.

This module is shared by the tests, the benchmark and the oracle's fixtures. It
holds scene synthesis only: analytic ray casting of spheres and a bumpy plane,
Poisson-disk node sampling, a ground-truth deformation, triangle rasterisation
of the deformed surface and depth-sensor noise. None of the solver's own
arithmetic lives here. In particular the ground-truth deformation is a linear
blend of per-node rigid motions over 8 nodes (rotation matrices from SciPy),
not the dual-quaternion blend of K=4 nodes the solver fits, and surfel normals
are the analytic surface normals, not the depth-map normals the solver derives.

The workloads stand in for the paper's single-camera depth streams (Sec.
"Results": consumer depth sensor, about 1e5 valid surfels per frame, a few
thousand nodes at the 2.5 cm node sampling distance of Table 1); the datasets
themselves are not used.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclasses.dataclass
class SolverParams:
    """Solver settings a workload is run with (mirrors the C-ABI config)."""
    gn_iters: int = 10
    pcg_iters: int = 10
    lambda_reg: float = 5.0
    node_sigma: float = 0.025
    corr_dist: float = 0.05
    corr_normal: float = 0.5
    edge_gate: float = 0.03
    damping: float = 1e-4
    rigid_iters: int = 0          # rigid alignment steps before the non-rigid ones


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    cam: Camera
    params: SolverParams
    surfel_pos: np.ndarray     # (Ns,3) float32, metres, reference frame
    surfel_nrm: np.ndarray     # (Ns,3) float32, unit, facing the camera
    node_pos: np.ndarray       # (Nn,3) float32
    gt_se3: np.ndarray         # (Nn,12) float64 row-major [R|t], reference -> live
    depth: np.ndarray          # (H,W) float32 live depth, 0 = invalid
    ref_depth: np.ndarray      # (H,W) float32 noise-free reference depth, 0 = miss
    surfel_pixel: np.ndarray   # (Ns,) int64 flat pixel each surfel was cast from
    info: Dict[str, float] = dataclasses.field(default_factory=dict)


# ----------------------------------------------------------------------------
# Analytic surfaces
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Sphere:
    center: Tuple[float, float, float]
    radius: float


@dataclasses.dataclass
class BumpyPlane:
    """z = z0 + amp * sin(2 pi x / period) * cos(2 pi y / period), |x|<=xlim, |y|<=ylim."""
    z0: float
    amp: float
    period: float
    xlim: float
    ylim: float


@dataclasses.dataclass
class Plane:
    """Infinite plane normal . x = offset (unit normal)."""
    normal: Tuple[float, float, float]
    offset: float

    def moved(self, R: np.ndarray, t: np.ndarray) -> "Plane":
        """The plane after x -> R x + t."""
        n = R @ np.asarray(self.normal, dtype=np.float64)
        return Plane(tuple(float(a) for a in n), float(self.offset + n @ t))


def _rays(cam: Camera, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    d = np.empty(px.shape + (3,), dtype=np.float64)
    d[..., 0] = (px - cam.cx) / cam.fx
    d[..., 1] = (py - cam.cy) / cam.fy
    d[..., 2] = 1.0
    return d


def _cast_sphere(s: Sphere, d: np.ndarray):
    c = np.asarray(s.center, dtype=np.float64)
    a = np.einsum("...i,...i->...", d, d)
    b = d @ c
    cc = c @ c - s.radius ** 2
    disc = b * b - a * cc
    hit = disc >= 0.0
    t = np.full(d.shape[:-1], np.inf)
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t0 = (b - sq) / a
    ok = hit & (t0 > 1e-6)
    t[ok] = t0[ok]
    p = d * np.where(ok, t, 0.0)[..., None]
    n = (p - c) / s.radius
    return t, n


def _cast_flat(pl: Plane, d: np.ndarray):
    n = np.asarray(pl.normal, dtype=np.float64)
    nd = d @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        s = pl.offset / nd
    ok = np.isfinite(s) & (s > 1e-6)
    t = np.where(ok, s, np.inf)
    nn = np.where((nd < 0)[..., None], n, -n)
    return t, np.broadcast_to(nn, d.shape).copy()


def _cast_plane(pl: BumpyPlane, d: np.ndarray):
    k = 2.0 * math.pi / pl.period
    dx, dy = d[..., 0].ravel(), d[..., 1].ravel()
    t = np.full(dx.shape, pl.z0)
    act = np.arange(dx.size)
    for _ in range(60):
        ta, ax, ay = t[act], dx[act], dy[act]
        sx, cx = np.sin(k * ta * ax), np.cos(k * ta * ax)
        sy, cy = np.sin(k * ta * ay), np.cos(k * ta * ay)
        f = ta - (pl.z0 + pl.amp * sx * cy)
        fp = 1.0 - pl.amp * k * (cx * cy * ax - sx * sy * ay)
        step = f / fp
        t[act] = ta - step
        act = act[np.abs(step) > 1e-13]
        if act.size == 0:
            break
    t = t.reshape(d.shape[:-1])
    x, y = t * d[..., 0], t * d[..., 1]
    h = pl.z0 + pl.amp * np.sin(k * x) * np.cos(k * y)
    conv = np.abs(t - h) < 1e-10
    inside = (np.abs(x) <= pl.xlim) & (np.abs(y) <= pl.ylim) & conv & (t > 0)
    hx = pl.amp * k * np.cos(k * x) * np.cos(k * y)
    hy = -pl.amp * k * np.sin(k * x) * np.sin(k * y)
    n = np.stack([hx, hy, -np.ones_like(hx)], axis=-1)
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    tt = np.where(inside, t, np.inf)
    return tt, n


def ray_cast(cam: Camera, prims: List, px: np.ndarray, py: np.ndarray):
    """Nearest hit of the rays through pixel coordinates (px, py).

    Returns depth z (inf = miss), the hit point, the unit normal facing the
    camera and the primitive id (-1 = miss)."""
    d = _rays(cam, px, py)
    best_t = np.full(px.shape, np.inf)
    best_n = np.zeros(px.shape + (3,))
    best_id = np.full(px.shape, -1, dtype=np.int32)
    for pid, pr in enumerate(prims):
        if isinstance(pr, Sphere):
            t, n = _cast_sphere(pr, d)
        elif isinstance(pr, Plane):
            t, n = _cast_flat(pr, d)
        else:
            t, n = _cast_plane(pr, d)
        closer = t < best_t
        best_t[closer] = t[closer]
        best_n[closer] = n[closer]
        best_id[closer] = pid
    p = d * np.where(np.isfinite(best_t), best_t, 0.0)[..., None]
    return best_t, p, best_n, best_id


# ----------------------------------------------------------------------------
# Reference surfels and nodes
# ----------------------------------------------------------------------------

def reference_surfels(cam: Camera, prims: List, grazing_cos: float = 0.15, margin: int = 1):
    """Surfels at integer pixel centres where the surface is hit away from
    silhouettes: every pixel within `margin` (Chebyshev distance; 1 = the pixel
    and its neighbours) hits the same primitive and the view ray is not
    grazing. Positions are the hit points, normals analytic."""
    from scipy.ndimage import maximum_filter, minimum_filter
    ys, xs = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    t, p, n, pid = ray_cast(cam, prims, xs, ys)
    hit = np.isfinite(t)
    size = 2 * margin + 1
    lo = minimum_filter(pid, size=size, mode="constant", cval=-1)
    hi = maximum_filter(pid, size=size, mode="constant", cval=-1)
    same = hit & (lo == pid) & (hi == pid)
    view = p / np.maximum(np.linalg.norm(p, axis=-1, keepdims=True), 1e-30)
    facing = -np.einsum("...i,...i->...", n, view)
    keep = same & (facing > grazing_cos)
    flat = np.flatnonzero(keep.ravel())
    pos = p.reshape(-1, 3)[flat].astype(np.float32)
    nrm = n.reshape(-1, 3)[flat].astype(np.float32)
    ref_depth = np.where(hit, t, 0.0).astype(np.float32)
    return pos, nrm, flat.astype(np.int64), ref_depth


def poisson_nodes(pos: np.ndarray, spacing: float, target: int,
                  rng: np.random.Generator) -> np.ndarray:
    """Dart throwing over the surfels in a seeded random order: accept a surfel
    as a node if no accepted node lies closer than `spacing`; stop at `target`.
    Returns the indices of the accepted surfels, in acceptance order.

    Candidates are screened in batches against the nodes accepted before the
    batch; the survivors are then accepted one by one in order, so the result
    equals the one-at-a-time definition."""
    p = pos.astype(np.float64)
    n = p.shape[0]
    order = rng.permutation(n)
    cell = spacing / math.sqrt(3.0)  # at most one node per cell
    lo = p.min(axis=0) - 3 * cell
    dims = np.ceil((p.max(axis=0) - lo) / cell).astype(np.int64) + 4
    grid = np.full(tuple(dims), -1, dtype=np.int64)
    cells = np.floor((p - lo) / cell).astype(np.int64)
    r = np.arange(-2, 3)
    offs = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    s2 = spacing * spacing
    accepted: List[int] = []

    def clear_of_nodes(ids: np.ndarray) -> np.ndarray:
        nb = cells[ids][:, None, :] + offs[None]
        occ = grid[nb[..., 0], nb[..., 1], nb[..., 2]]
        dd = p[np.maximum(occ, 0)] - p[ids][:, None, :]
        d2 = np.where(occ >= 0, np.einsum("bkc,bkc->bk", dd, dd), np.inf)
        return d2.min(axis=1) >= s2

    batch = 4096
    for start in range(0, n, batch):
        cand = order[start:start + batch]
        surv = cand[clear_of_nodes(cand)]
        for i in surv:
            if not clear_of_nodes(np.asarray([i]))[0]:
                continue
            g = cells[i]
            grid[g[0], g[1], g[2]] = i
            accepted.append(int(i))
            if len(accepted) >= target:
                return np.asarray(accepted, dtype=np.int64)
    return np.asarray(accepted, dtype=np.int64)


# ----------------------------------------------------------------------------
# Ground-truth deformation
# ----------------------------------------------------------------------------

def random_node_motion(node_pos: np.ndarray, max_deg: float, max_trans: float,
                       rng: np.random.Generator, smooth_steps: int = 10,
                       graph_k: int = 8) -> np.ndarray:
    """Per-node random rigid motion about the node itself, smoothed.

    Each node draws an axis uniform on the sphere, an angle uniform in
    [0, max_deg] and a translation uniform in a ball of radius max_trans.
    The 6-vectors (rotation vector, translation) are then smoothed by
    `smooth_steps` Jacobi steps xi <- xi/2 + mean(xi over neighbours)/2 on the
    symmetrised 8-nearest-neighbour graph, then rescaled so that the largest
    rotation angle is max_deg and the largest translation max_trans (averaging
    alone would shrink the motion to a small fraction of the bounds).
    Returns (Nn,12) [R|t] with x_live = R (x - p) + p + t written as R x + t'.
    """
    n = node_pos.shape[0]
    axis = rng.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = np.deg2rad(max_deg) * rng.random(n)
    tdir = rng.normal(size=(n, 3))
    tdir /= np.linalg.norm(tdir, axis=1, keepdims=True)
    trad = max_trans * np.cbrt(rng.random(n))
    xi = np.concatenate([axis * ang[:, None], tdir * trad[:, None]], axis=1)
    if smooth_steps > 0 and n > 1:
        k = min(graph_k + 1, n)
        _, nb = cKDTree(node_pos.astype(np.float64)).query(node_pos.astype(np.float64), k=k)
        adj = [set() for _ in range(n)]
        for j in range(n):
            for m in nb[j, 1:]:
                adj[j].add(int(m))
                adj[int(m)].add(j)
        lists = [np.fromiter(sorted(a), dtype=np.int64) for a in adj]
        for _ in range(smooth_steps):
            mean = np.stack([xi[l].mean(axis=0) if l.size else xi[j]
                             for j, l in enumerate(lists)])
            xi = 0.5 * xi + 0.5 * mean
    amax = np.linalg.norm(xi[:, :3], axis=1).max()
    tmax = np.linalg.norm(xi[:, 3:], axis=1).max()
    if amax > 0:
        xi[:, :3] *= np.deg2rad(max_deg) / amax
    if tmax > 0:
        xi[:, 3:] *= max_trans / tmax
    return compose_about_nodes(node_pos, xi)


def compose_about_nodes(node_pos: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """[R|t'] for x -> R (x - p) + p + t with R = Rotation.from_rotvec(xi[:, :3])."""
    R = Rotation.from_rotvec(xi[:, :3]).as_matrix()
    p = node_pos.astype(np.float64)
    tp = p + xi[:, 3:] - np.einsum("nij,nj->ni", R, p)
    out = np.concatenate([R, tp[:, :, None]], axis=2).reshape(-1, 12)
    return out


def blend_motion(points: np.ndarray, node_pos: np.ndarray, se3: np.ndarray,
                 sigma: float, k: int = 8) -> np.ndarray:
    """Ground-truth deformation of points: linear blend of the 3x4 node
    transforms of the k nearest nodes with Gaussian weights (generator only)."""
    p = points.astype(np.float64)
    kk = min(k, node_pos.shape[0])
    dist, nb = cKDTree(node_pos.astype(np.float64)).query(p, k=kk)
    if kk == 1:
        dist, nb = dist[:, None], nb[:, None]
    w = np.exp(-(dist ** 2 - dist[:, :1] ** 2) / (2.0 * sigma * sigma))
    w /= w.sum(axis=1, keepdims=True)
    M = se3.reshape(-1, 3, 4)
    out = np.zeros_like(p)
    for s in range(kk):
        Ms = M[nb[:, s]]
        out += w[:, s:s + 1] * (np.einsum("nij,nj->ni", Ms[:, :, :3], p) + Ms[:, :, 3])
    return out


# ----------------------------------------------------------------------------
# Rendering the deformed surface
# ----------------------------------------------------------------------------

def surface_grid(cam: Camera, prims: List, ss: int = 2):
    """The reference surface sampled on an ss-times supersampled pixel grid
    (ray depth, hit point, primitive id per sample): the mesh that
    raster_deformed deforms. It depends on the camera and the scene only, so a
    stream's frames share it."""
    W2, H2 = cam.width * ss, cam.height * ss
    gy, gx = np.mgrid[0:H2, 0:W2].astype(np.float64)
    px = (gx + 0.5) / ss - 0.5
    py = (gy + 0.5) / ss - 0.5
    t, p, _, pid = ray_cast(cam, prims, px, py)
    return dict(ss=ss, t=t, p=p, pid=pid)


def render_deformed(cam: Camera, prims: List, node_pos: np.ndarray, se3: np.ndarray,
                    sigma: float, edge_gate: float, ss: int = 2,
                    max_edge_px: float = 3.0) -> np.ndarray:
    """Live depth: the reference surface sampled on an ss-times supersampled
    pixel grid, triangulated, deformed by the ground-truth motion and
    z-buffer rasterised at pixel centres. Triangles spanning a silhouette
    (vertices on different primitives or a depth jump above edge_gate) or whose
    projected edges exceed max_edge_px are dropped. Uncovered pixels are 0."""
    return raster_deformed(cam, surface_grid(cam, prims, ss), node_pos, se3, sigma, edge_gate, max_edge_px)


def raster_deformed(cam: Camera, grid: Dict, node_pos: np.ndarray, se3: np.ndarray,
                    sigma: float, edge_gate: float, max_edge_px: float = 3.0) -> np.ndarray:
    """render_deformed on a surface grid already sampled (surface_grid)."""
    ss, t, p, pid = grid["ss"], grid["t"], grid["p"], grid["pid"]
    W2, H2 = cam.width * ss, cam.height * ss
    hit = np.isfinite(t)
    verts = p.reshape(-1, 3)
    vhit = hit.ravel()
    live = np.zeros_like(verts)
    live[vhit] = blend_motion(verts[vhit], node_pos, se3, sigma)
    z = live[:, 2]
    okz = vhit & (z > 1e-6)
    sx = np.where(okz, cam.fx * live[:, 0] / np.where(okz, z, 1.0) + cam.cx, 0.0)
    sy = np.where(okz, cam.fy * live[:, 1] / np.where(okz, z, 1.0) + cam.cy, 0.0)
    tz = t.ravel()
    pidf = pid.ravel()

    idx = np.arange(H2 * W2).reshape(H2, W2)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, :-1].ravel()
    d = idx[1:, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([b, d, c], 1)], 0)
    v0, v1, v2 = tris[:, 0], tris[:, 1], tris[:, 2]
    ok = okz[v0] & okz[v1] & okz[v2]
    ok &= (pidf[v0] == pidf[v1]) & (pidf[v1] == pidf[v2])
    zt = np.stack([tz[v0], tz[v1], tz[v2]], 1)
    with np.errstate(invalid="ignore"):
        ok &= (np.nanmax(zt, 1) - np.nanmin(zt, 1)) <= edge_gate
    X = np.stack([sx[v0], sx[v1], sx[v2]], 1)
    Y = np.stack([sy[v0], sy[v1], sy[v2]], 1)
    for i, j in ((0, 1), (1, 2), (2, 0)):
        ok &= np.hypot(X[:, i] - X[:, j], Y[:, i] - Y[:, j]) <= max_edge_px
    tris, X, Y = tris[ok], X[ok], Y[ok]
    Z = np.stack([z[tris[:, 0]], z[tris[:, 1]], z[tris[:, 2]]], 1)

    best = np.full(cam.width * cam.height, np.inf)
    x0 = np.ceil(X.min(1)).astype(np.int64)
    y0 = np.ceil(Y.min(1)).astype(np.int64)
    x1 = np.floor(X.max(1)).astype(np.int64)
    y1 = np.floor(Y.max(1)).astype(np.int64)
    area = (X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (X[:, 2] - X[:, 0]) * (Y[:, 1] - Y[:, 0])
    nz = np.abs(area) > 1e-12
    span = int(math.ceil(max_edge_px)) + 1
    for oy in range(span):
        for ox in range(span):
            qx = x0 + ox
            qy = y0 + oy
            m = nz & (qx <= x1) & (qy <= y1) & (qx >= 0) & (qy >= 0) \
                & (qx < cam.width) & (qy < cam.height)
            if not np.any(m):
                continue
            Xm, Ym, Zm, am = X[m], Y[m], Z[m], area[m]
            fx_, fy_ = qx[m].astype(np.float64), qy[m].astype(np.float64)
            w0 = ((Xm[:, 1] - fx_) * (Ym[:, 2] - fy_) - (Xm[:, 2] - fx_) * (Ym[:, 1] - fy_)) / am
            w1 = ((Xm[:, 2] - fx_) * (Ym[:, 0] - fy_) - (Xm[:, 0] - fx_) * (Ym[:, 2] - fy_)) / am
            w2 = 1.0 - w0 - w1
            inside = (w0 >= 0) & (w1 >= 0) & (w2 >= 0)
            if not np.any(inside):
                continue
            inv = w0 / Zm[:, 0] + w1 / Zm[:, 1] + w2 / Zm[:, 2]
            zz = 1.0 / inv
            pix = (qy[m] * cam.width + qx[m])
            np.minimum.at(best, pix[inside], zz[inside])
    out = np.where(np.isfinite(best), best, 0.0).reshape(cam.height, cam.width)
    return out


def add_sensor_noise(depth: np.ndarray, noise_std: float, dropout: float,
                     rng: np.random.Generator) -> np.ndarray:
    d = depth.astype(np.float64).copy()
    valid = d > 0
    noise = rng.normal(0.0, noise_std, size=d.shape)
    drop = rng.random(d.shape) < dropout
    d = np.where(valid, d + noise, 0.0)
    d = np.where(drop, 0.0, d)
    d = np.where(d > 0, d, 0.0)
    return d.astype(np.float32)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def _assemble(name, seed, cam, prims, params, n_nodes, spacing, max_deg, max_trans,
              noise, dropout, rng, surfel_subset: Optional[int] = None) -> Scene:
    pos, nrm, pix, ref_depth = reference_surfels(cam, prims)
    if surfel_subset is not None and surfel_subset < pos.shape[0]:
        keep = np.sort(rng.choice(pos.shape[0], size=surfel_subset, replace=False))
        pos, nrm, pix = pos[keep], nrm[keep], pix[keep]
    nodes_i = poisson_nodes(pos, spacing, n_nodes, rng)
    node_pos = pos[nodes_i].copy()
    gt = random_node_motion(node_pos, max_deg, max_trans, rng)
    live = render_deformed(cam, prims, node_pos, gt, params.node_sigma, params.edge_gate)
    depth = add_sensor_noise(live, noise, dropout, rng)
    info = {"n_surfels": float(pos.shape[0]), "n_nodes": float(node_pos.shape[0]),
            "valid_depth": float(np.count_nonzero(depth))}
    return Scene(name, seed, cam, params, pos, nrm, node_pos, gt, depth,
                 ref_depth, pix, info)


def scene_tiny(seed: int = 7) -> Scene:
    """Small case the oracle finishes in well under a second per GN step:
    80x60 view of a sphere (r 0.5 m, centre 1.2 m), 40 nodes at 5 cm."""
    rng = np.random.default_rng(seed)
    cam = Camera(80, 60, 75.0, 75.0, 40.0, 30.0)
    prims = [Sphere((0.0, 0.0, 1.2), 0.5)]
    params = SolverParams(gn_iters=4, pcg_iters=10, lambda_reg=5.0, node_sigma=0.05,
                          corr_dist=0.05, corr_normal=0.5, edge_gate=0.03, damping=1e-4)
    return _assemble("tiny", seed, cam, prims, params, 40, 0.05, 3.0, 0.005,
                     0.001, 0.0, rng)


def scene_c1(seed: int = 1) -> Scene:
    """160x120 (f=150, c=(80,60)) view of a 1 m sphere centred at z=2 m (its
    near point at 1 m), 200 Poisson nodes at 2.5 cm, motion <=3 deg / 5 mm,
    N(0, 1 mm) noise, lambda 2.3, 5 GN x 10 PCG."""
    rng = np.random.default_rng(seed)
    cam = Camera(160, 120, 150.0, 150.0, 80.0, 60.0)
    prims = [Sphere((0.0, 0.0, 2.0), 1.0)]
    params = SolverParams(gn_iters=5, pcg_iters=10, lambda_reg=2.3, node_sigma=0.025,
                          corr_dist=0.05, corr_normal=0.5, edge_gate=0.03, damping=1e-4)
    return _assemble("c1", seed, cam, prims, params, 200, 0.025, 3.0, 0.005,
                     0.001, 0.0, rng)


def corner_prims() -> List:
    """Inside corner of a box seen from the camera: floor, left wall, back wall."""
    return [Plane((0.0, -1.0, 0.0), -0.35), Plane((1.0, 0.0, 0.0), -0.45),
            Plane((0.0, 0.0, -1.0), -1.5)]


def c2_prims() -> List:
    return [Sphere((-0.30, -0.10, 1.00), 0.20),
            Sphere((0.25, 0.05, 1.05), 0.15),
            Sphere((0.00, 0.25, 1.25), 0.18),
            BumpyPlane(1.45, 0.03, 0.25, 0.75, 0.55)]


def scene_c2(seed: int = 2) -> Scene:
    """640x480 (f=570, c=(320,240)): three spheres in front of a bumpy plane
    (depth 0.8-1.5 m), ~2000 Poisson nodes at 2.5 cm, motion <=8 deg / 2 cm,
    N(0, 1.5 mm) noise with 5% dropout, lambda 5, 10 GN x 10 PCG."""
    rng = np.random.default_rng(seed)
    cam = Camera(640, 480, 570.0, 570.0, 320.0, 240.0)
    params = SolverParams(gn_iters=10, pcg_iters=10, lambda_reg=5.0, node_sigma=0.025,
                          corr_dist=0.05, corr_normal=0.5, edge_gate=0.03, damping=1e-4)
    return _assemble("c2", seed, cam, c2_prims(), params, 2000, 0.025, 8.0, 0.02,
                     0.0015, 0.05, rng)


def scene_random(seed: int, size: Optional[Tuple[int, int]] = None,
                 n_nodes: Optional[int] = None, n_surfels: Optional[int] = None) -> Scene:
    """One stream of the uneven multi-stream workload: image 320x240 or
    640x480, three random spheres (radius 0.1-0.25 m, near point 0.8-1.3 m),
    a bumpy plane with probability 1/2, a node target in [300, 4000] (spacing
    shrinks from 2.5 cm by 0.9 until reachable, sigma = spacing) and a surfel
    target in [4k, min(300k, 0.95 Npx)]; motion and noise as the 640x480 case."""
    rng = np.random.default_rng(seed)
    if size is None:
        size = (320, 240) if rng.random() < 0.5 else (640, 480)
    w, h = size
    f = 570.0 * w / 640.0
    cam = Camera(w, h, f, f, w / 2.0, h / 2.0)
    prims: List = []
    for _ in range(3):
        r = 0.10 + 0.15 * rng.random()
        near = 0.8 + 0.5 * rng.random()
        cxy = rng.uniform(-0.35, 0.35, size=2) * (near + r)
        prims.append(Sphere((float(cxy[0]), float(cxy[1]) * 0.75, near + r), r))
    if rng.random() < 0.5:
        prims.append(BumpyPlane(1.45, 0.03, 0.25, 0.75, 0.55))
    tgt_nodes = int(rng.integers(300, 4001)) if n_nodes is None else n_nodes
    npx = w * h
    tgt_surf = int(rng.integers(4000, int(min(300000, 0.95 * npx)) + 1)) if n_surfels is None else n_surfels
    pos, nrm, pix, ref_depth = reference_surfels(cam, prims)
    sub = min(tgt_surf, pos.shape[0])
    keep = np.sort(rng.choice(pos.shape[0], size=sub, replace=False))
    pos, nrm, pix = pos[keep], nrm[keep], pix[keep]
    spacing = 0.025
    while True:
        nodes_i = poisson_nodes(pos, spacing, tgt_nodes, rng)
        if nodes_i.size >= tgt_nodes or spacing < 0.004:
            break
        spacing *= 0.9
    node_pos = pos[nodes_i].copy()
    params = SolverParams(gn_iters=10, pcg_iters=10, lambda_reg=5.0, node_sigma=spacing,
                          corr_dist=0.05, corr_normal=0.5, edge_gate=0.03, damping=1e-4)
    gt = random_node_motion(node_pos, 8.0, 0.02, rng)
    live = render_deformed(cam, prims, node_pos, gt, spacing, params.edge_gate)
    depth = add_sensor_noise(live, 0.0015, 0.05, rng)
    info = {"n_surfels": float(pos.shape[0]), "n_nodes": float(node_pos.shape[0]),
            "valid_depth": float(np.count_nonzero(depth)), "spacing": spacing}
    info["prims"] = prims
    return Scene(f"random{seed}", seed, cam, params, pos, nrm, node_pos, gt, depth,
                 ref_depth, pix, info)


def motion_walk(scene: Scene, n_frames: int, seed: int, max_deg: float = 2.0,
                max_trans: float = 0.005) -> List[np.ndarray]:
    """Ground truth of a stream's frames: frame 0 is the scene's, and frame f
    is a fresh smoothed random step (rotation <= max_deg about each node's
    live position, translation <= max_trans) composed after frame f - 1's.
    Returns the (Nn,12) [R|t] of every frame."""
    rng = np.random.default_rng(seed)
    M = [scene.gt_se3.reshape(-1, 3, 4)]
    p = scene.node_pos.astype(np.float64)
    for _ in range(1, n_frames):
        prev = M[-1]
        live = np.einsum("nij,nj->ni", prev[:, :, :3], p) + prev[:, :, 3]
        step = random_node_motion(live, max_deg, max_trans, rng).reshape(-1, 3, 4)
        R = step[:, :, :3] @ prev[:, :, :3]
        t = np.einsum("nij,nj->ni", step[:, :, :3], prev[:, :, 3]) + step[:, :, 3]
        M.append(np.concatenate([R, t[:, :, None]], axis=2))
    return [m.reshape(-1, 12) for m in M]


def stream_frames(scene: Scene, n_frames: int, seed: int) -> List[np.ndarray]:
    """Depth frames of a stream of the uneven-streams workload (a scene made by
    scene_random): frame 0 is the scene's depth, frames 1.. render the walk of
    motion_walk with the same sensor noise and dropout, each with its own
    noise draw."""
    prims = scene.info["prims"]
    grid = surface_grid(scene.cam, prims)
    rng = np.random.default_rng(seed + 7919)
    out = [scene.depth]
    for se3 in motion_walk(scene, n_frames, seed)[1:]:
        live = raster_deformed(scene.cam, grid, scene.node_pos, se3, scene.params.node_sigma,
                               scene.params.edge_gate)
        out.append(add_sensor_noise(live, 0.0015, 0.05, rng))
    return out


SCENES = {"tiny": scene_tiny, "c1": scene_c1, "c2": scene_c2, "random": scene_random}


def make_scene(name: str, seed: Optional[int] = None) -> Scene:
    fn = SCENES[name]
    return fn() if seed is None else fn(seed)
