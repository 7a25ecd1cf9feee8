"""FP32 decision replica.

Every floating-point comparison that decides an integer output of the solve is
taken here in IEEE FP32, one rounding per operation (NumPy float32 ufuncs: no
fused multiply-add, correctly rounded division and square root) and in the
operation order written below. The decisions are:

* the nearest-node key ((dx*dx + dy*dy) + dz*dz), dx = x_surfel - x_node
  (skinning and node graph, Sec. 6.5 and Sec. 3);
* back-projection X = ((u - cx)/fx) * d, Y = ((v - cy)/fy) * d, Z = d (Sec. 5);
* the normal-map validity (depth present at the pixel and its 4 neighbours,
  |D(nb) - D(u)| <= edge_gate, nonzero cross product) and the normal itself
  (central differences, cross product, division by its length, orientation
  towards the camera) (Sec. 5);
* the pixel of a projection, floor(fx*(x/z) + cx + 0.5) (Sec. 6.1, 7);
* the index-map winner: smallest (FP32 z bits, surfel index) (Sec. 7);
* the correspondence gates |v - V(u)|^2 < dist^2 and n . N(u) > cos (Sec. 7);
* with splats (Sec. 7, surfels as opaque discs): the footprint box, the
  ray-disc coverage test and the hit depth (see splat_index_map).

Nothing in this module is an FP64 quantity of the oracle; it only decides.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def sqdist_key(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Pairwise FP32 keys ((dx*dx + dy*dy) + dz*dz), shape (len(a), len(b))."""
    a = a.astype(f32)
    b = b.astype(f32)
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def backproject(ux: np.ndarray, uy: np.ndarray, d: np.ndarray, cam) -> np.ndarray:
    x = ux.astype(f32)
    y = uy.astype(f32)
    d = d.astype(f32)
    X = ((x - f32(cam.cx)) / f32(cam.fx)) * d
    Y = ((y - f32(cam.cy)) / f32(cam.fy)) * d
    return np.stack([X, Y, d], axis=-1)


def depth_valid(depth: np.ndarray) -> np.ndarray:
    d = depth.astype(f32)
    with np.errstate(invalid="ignore"):
        return np.isfinite(d) & (d > f32(0))


def normal_map(depth: np.ndarray, cam, edge_gate: float):
    """FP32 normal map and its validity mask (H, W, 3), (H, W)."""
    D = depth.astype(f32)
    H, W = D.shape
    valid = depth_valid(D)
    Dz = np.where(valid, D, f32(0))
    ys, xs = np.mgrid[0:H, 0:W]
    V = backproject(xs, ys, Dz, cam)
    N = np.zeros((H, W, 3), dtype=f32)
    ok = np.zeros((H, W), dtype=bool)
    if H < 3 or W < 3:
        return N, ok
    c = valid[1:-1, 1:-1]
    gate = f32(edge_gate)
    Dc = Dz[1:-1, 1:-1]
    for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        nb_valid = valid[1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
        nb = Dz[1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
        with np.errstate(invalid="ignore"):
            c = c & nb_valid & (np.abs(nb - Dc) <= gate)
    a = V[2:, 1:-1] - V[:-2, 1:-1]      # V(x, y+1) - V(x, y-1)
    b = V[1:-1, 2:] - V[1:-1, :-2]      # V(x+1, y) - V(x-1, y)
    c0 = a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1]
    c1 = a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2]
    c2 = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
        nn = (c0 * c0 + c1 * c1) + c2 * c2
        c = c & (nn > f32(0)) & np.isfinite(nn)
        ln = np.sqrt(np.where(c, nn, f32(1)))
        n0 = c0 / ln
        n1 = c1 / ln
        n2 = c2 / ln
        Vc = V[1:-1, 1:-1]
        dot = (n0 * Vc[..., 0] + n1 * Vc[..., 1]) + n2 * Vc[..., 2]
    flip = dot > f32(0)
    n0 = np.where(flip, -n0, n0)
    n1 = np.where(flip, -n1, n1)
    n2 = np.where(flip, -n2, n2)
    inner = np.stack([n0, n1, n2], -1)
    N[1:-1, 1:-1] = np.where(c[..., None], inner, f32(0))
    ok[1:-1, 1:-1] = c
    return N, ok


def project(v: np.ndarray, cam):
    """Pixel (ux, uy) of FP32 points and whether it lies in the image with z > 0."""
    v = v.astype(f32)
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        px = f32(cam.fx) * (x / z) + f32(cam.cx)
        py = f32(cam.fy) * (y / z) + f32(cam.cy)
        hx = px + f32(0.5)
        hy = py + f32(0.5)
        inside = (z > f32(0)) & (hx >= f32(0)) & (hx < f32(cam.width)) \
            & (hy >= f32(0)) & (hy < f32(cam.height))
    ux = np.where(inside, np.floor(np.where(inside, hx, f32(0))), f32(0)).astype(np.int64)
    uy = np.where(inside, np.floor(np.where(inside, hy, f32(0))), f32(0)).astype(np.int64)
    return ux, uy, inside


def index_map(v: np.ndarray, cam, valid: np.ndarray | None = None) -> np.ndarray:
    """Index map: per pixel the surfel with the smallest (z, index) among the
    surfels projecting there, -1 where none does. `valid` masks surfels out."""
    ux, uy, inside = project(v, cam)
    if valid is not None:
        inside = inside & valid
    z = v[:, 2].astype(f32)
    ids = np.flatnonzero(inside)
    pix = uy[ids] * cam.width + ux[ids]
    zb = z[ids].view(np.uint32)
    order = np.lexsort((ids, zb, pix))
    pix_s = pix[order]
    first = np.ones(order.size, dtype=bool)
    first[1:] = pix_s[1:] != pix_s[:-1]
    I = np.full(cam.width * cam.height, -1, dtype=np.int64)
    I[pix_s[first]] = ids[order][first]
    return I.reshape(cam.height, cam.width)


def correspondence(v: np.ndarray, n: np.ndarray, I: np.ndarray, depth: np.ndarray,
                   N32: np.ndarray, nvalid: np.ndarray, cam, corr_dist: float,
                   corr_normal: float, valid: np.ndarray | None = None):
    """Projective correspondence (FP32 gates). Returns the mask of matched
    surfels and their pixels (ux, uy)."""
    v = v.astype(f32)
    n = n.astype(f32)
    ux, uy, inside = project(v, cam)
    if valid is not None:
        inside = inside & valid
    m = inside.copy()
    ids = np.arange(v.shape[0])
    m &= I[uy, ux] == ids
    m &= nvalid[uy, ux]
    D = depth.astype(f32)[uy, ux]
    Vd = backproject(ux, uy, D, cam)
    Nd = N32[uy, ux]
    with np.errstate(invalid="ignore", over="ignore"):
        dx = v[:, 0] - Vd[:, 0]
        dy = v[:, 1] - Vd[:, 1]
        dz = v[:, 2] - Vd[:, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        dist2 = f32(corr_dist) * f32(corr_dist)
        m &= d2 < dist2
        dot = (n[:, 0] * Nd[:, 0] + n[:, 1] * Nd[:, 1]) + n[:, 2] * Nd[:, 2]
        m &= dot > f32(corr_normal)
    return m, ux, uy


SPLAT_MAX_PX = 4          # half-size cap of a splat's pixel box


def splat_index_map(v: np.ndarray, n: np.ndarray, radius: np.ndarray, cam, valid: np.ndarray | None = None):
    """Index map of opaque disc splats: per pixel the surfel with the smallest
    (FP32 hit depth bits, index), -1 where none.

    A surfel whose centre projects into the image to pixel (ux, uy) (the point
    rule of `project`) is tried on the pixels of the box ux +- h, uy +- h
    (clipped to the image), h = min(4, ceil(fx r / z)) in FP32. The ray of
    pixel u is d = ((u_x - cx)/fx, (u_y - cy)/fy, 1); with nd = n . d and
    nv = n . v, the hit is t = nv / nd, P = t d, and the pixel is covered if
    nd != 0, t > 0 and |P - v|^2 <= r^2; its depth is t. A surfel of radius 0
    is an unsized point: its centre pixel at depth z."""
    v = v.astype(f32)
    n = n.astype(f32)
    r = np.asarray(radius, f32)
    ux0, uy0, inside = project(v, cam)
    if valid is not None:
        inside = inside & valid
    W, H = cam.width, cam.height
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        rho = (f32(cam.fx) * r) / v[:, 2]
        h = np.where(inside, np.minimum(SPLAT_MAX_PX, np.ceil(np.where(inside, rho, f32(0)))), 0).astype(np.int64)
    pix_l, key_l, id_l = [], [], []
    ids_all = np.arange(v.shape[0])
    for oy in range(-SPLAT_MAX_PX, SPLAT_MAX_PX + 1):
        for ox in range(-SPLAT_MAX_PX, SPLAT_MAX_PX + 1):
            sel = inside & (np.abs(ox) <= h) & (np.abs(oy) <= h)
            ux = ux0 + ox
            uy = uy0 + oy
            sel &= (ux >= 0) & (ux < W) & (uy >= 0) & (uy < H)
            ids = ids_all[sel]
            if ids.size == 0:
                continue
            vx, vy, vz = v[ids, 0], v[ids, 1], v[ids, 2]
            nx, ny, nz = n[ids, 0], n[ids, 1], n[ids, 2]
            point = r[ids] == f32(0)
            with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
                dx = (ux[ids].astype(f32) - f32(cam.cx)) / f32(cam.fx)
                dy = (uy[ids].astype(f32) - f32(cam.cy)) / f32(cam.fy)
                nd = (nx * dx + ny * dy) + nz
                nv = (nx * vx + ny * vy) + nz * vz
                t = nv / nd
                ex = t * dx - vx
                ey = t * dy - vy
                ez = t - vz
                e2 = (ex * ex + ey * ey) + ez * ez
                cov = (nd != f32(0)) & (t > f32(0)) & (e2 <= r[ids] * r[ids])
            centre = (ox == 0) & (oy == 0)
            take = np.where(point, centre, cov)
            depth = np.where(point, vz, t)
            pix_l.append((uy[ids] * W + ux[ids])[take])
            key_l.append(depth[take].astype(f32).view(np.uint32))
            id_l.append(ids[take])
    I = np.full(W * H, -1, dtype=np.int64)
    if pix_l:
        pix = np.concatenate(pix_l)
        key = np.concatenate(key_l)
        idv = np.concatenate(id_l)
        order = np.lexsort((idv, key, pix))
        ps = pix[order]
        first = np.ones(order.size, dtype=bool)
        first[1:] = ps[1:] != ps[:-1]
        I[ps[first]] = idv[order][first]
    return I.reshape(H, W)


def splat_pairs(v: np.ndarray, n: np.ndarray, I: np.ndarray, depth: np.ndarray, N32: np.ndarray,
                nvalid: np.ndarray, cam, corr_dist: float, corr_normal: float):
    """Pixel-driven pairs of a splat index map: pixel u with a normal pairs
    with its winner k if |v_k - V(u)|^2 < dist^2 and n_k . N(u) > cos (FP32,
    the surfel's centre and normal). Returns the surfel and pixel (x, y) of
    every pair, in row-major pixel order."""
    v = v.astype(f32)
    n = n.astype(f32)
    uy, ux = np.nonzero((I >= 0) & nvalid)
    k = I[uy, ux]
    D = depth.astype(f32)[uy, ux]
    Vd = backproject(ux, uy, D, cam)
    Nd = N32[uy, ux]
    with np.errstate(invalid="ignore", over="ignore"):
        dx = v[k, 0] - Vd[:, 0]
        dy = v[k, 1] - Vd[:, 1]
        dz = v[k, 2] - Vd[:, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        dot = (n[k, 0] * Nd[:, 0] + n[k, 1] * Nd[:, 1]) + n[k, 2] * Nd[:, 2]
        ok = (d2 < f32(corr_dist) * f32(corr_dist)) & (dot > f32(corr_normal))
    return k[ok], ux[ok], uy[ok]
