"""Gauss-Newton estimate of the node transforms for one depth frame (FP64).

Sec. 7: the node transforms T_j are estimated from the new depth D, the
previous warp field and the reference surfels by minimising
E_depth + lambda E_regulation with Gauss-Newton. Sec. 8: J^T J is built, then
the linear system J^T J x = J^T e is solved; at most 10 iterations. Sec. 4: the
warp field starts from the previous frame's.

Readings taken here: e = -r, so each step solves (H + mu I) Delta = -g with
H = J^T J (rows of the regulariser weighted by sqrt(lambda)), g = J^T r and a
small damping mu on all 6N diagonal entries (it keeps the system positive
definite where the data term leaves a node's motion unobserved and does not
move the Gauss-Newton fixed point g = 0). The solve is either a dense Cholesky
factorisation (the reference answer) or block-Jacobi preconditioned conjugate
gradients from x0 = 0 run for exactly a given number of iterations (stopping
early only if r^T z = 0). Every frame runs exactly gn_iters iterations.
The node update is T_k <- Delta_k(xi_k) o T_k with the exact SO(3)
exponential.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import assoc, depth as depthmod, rigid, skin
from .quat import dq_from_rt, exp_so3, rt_to_se3, se3_to_rt
from .terms import arap_jacobians, arap_residuals, data_jacobian, data_residuals
from .warp import apply_blend, blend


@dataclasses.dataclass
class Problem:
    """Everything fixed during one frame solve."""
    cam: object
    surfel_pos: np.ndarray
    surfel_nrm: np.ndarray
    node_pos: np.ndarray
    idx: np.ndarray            # (Ns,4) skinning
    w: np.ndarray              # (Ns,4) FP64 weights
    nbr: np.ndarray            # (Nn,8) node graph
    frame: assoc.DepthFrame
    V64: np.ndarray            # (H,W,3) FP64 vertex map
    N64: np.ndarray            # (H,W,3) FP64 normal map
    lambda_reg: float
    damping: float
    corr_dist: float
    corr_normal: float
    visible: Optional[np.ndarray] = None     # surfels rendered into the index map (None: all)
    splat_radius: Optional[np.ndarray] = None  # render opaque disc splats of these radii (None: points)


def visible_surfels(conf: np.ndarray, t_observed: np.ndarray, t_now: int, stable_conf: float,
                    recent_frames: int) -> np.ndarray:
    """Sec. 7: only stable surfels (confidence > delta_stable) and surfels
    observed within the last delta_recent frames are rendered (FP32
    confidence comparison). The paper adds the recent ones only in the first
    frames and after a reinitialisation: recent_frames < 0 leaves them out."""
    c = np.asarray(conf, np.float32)
    stable = c > np.float32(stable_conf)
    if recent_frames < 0:
        return stable
    return stable | (int(t_now) - np.asarray(t_observed, np.int64) <= int(recent_frames))


def make_problem(cam, surfel_pos, surfel_nrm, node_pos, depth, params,
                 idx=None, w=None, nbr=None, visible=None, splat_radius=None) -> Problem:
    if idx is None or w is None:
        idx, w = skin.skinning(surfel_pos, node_pos, params.node_sigma)
    if nbr is None:
        nbr = skin.node_graph(node_pos)
    frame = assoc.prepare_depth(depth, cam, params.edge_gate)
    return Problem(cam, np.asarray(surfel_pos, np.float32), np.asarray(surfel_nrm, np.float32),
                   np.asarray(node_pos, np.float32), idx, w, nbr, frame,
                   depthmod.vertex_map(depth, cam), depthmod.normal_map(depth, cam),
                   float(params.lambda_reg), float(params.damping),
                   float(params.corr_dist), float(params.corr_normal),
                   None if visible is None else np.asarray(visible, bool),
                   None if splat_radius is None else np.asarray(splat_radius, np.float32))


def node_tables(node_pos: np.ndarray, R: np.ndarray, t: np.ndarray):
    """Dual quaternions (r, d) of the node transforms and live node positions."""
    r, d = dq_from_rt(R, t)
    c = np.einsum("nij,nj->ni", R, node_pos.astype(np.float64)) + t
    return r, d, c


def warp_surfels(pb: Problem, R: np.ndarray, t: np.ndarray):
    r, d, c = node_tables(pb.node_pos, R, t)
    b, s = blend(pb.idx, pb.w, r, d)
    v, n, valid = apply_blend(b, pb.surfel_pos, pb.surfel_nrm)
    if pb.visible is not None:
        valid = valid & pb.visible          # not rendered: in no index map, matched nowhere
    return dict(r=r, d=d, c=c, b=b, s=s, v=v, n=n, valid=valid)


def linearize(pb: Problem, R: np.ndarray, t: np.ndarray, corr_map: Optional[np.ndarray] = None) -> Dict:
    """Residuals, Jacobians and energies at the current transforms, with the
    association re-done at this state.

    corr_map (H,W; surfel index or -1), when given, supplies the
    correspondences instead: surfel i is matched to the pixel that holds i.
    This is for comparing arithmetic with an implementation whose FP32
    decisions fell the other way at a near-tie (a projection on a pixel
    boundary, a gate at its threshold); the association itself is the one
    decided here."""
    ws = warp_surfels(pb, R, t)
    if pb.splat_radius is not None:
        return _linearize_pairs(pb, R, t, ws, corr_map)
    I, m, ux, uy = assoc.associate(ws["v"], ws["n"], ws["valid"], pb.frame, pb.cam,
                                   pb.corr_dist, pb.corr_normal)
    if corr_map is not None:
        cm = np.asarray(corr_map).ravel()
        pix = np.flatnonzero(cm >= 0)
        m = np.zeros_like(m)
        ux, uy = ux.copy(), uy.copy()
        W = pb.cam.width
        m[cm[pix]] = True
        ux[cm[pix]] = pix % W
        uy[cm[pix]] = pix // W
    ci = np.flatnonzero(m)
    Vd = pb.V64[uy[ci], ux[ci]]
    Nd = pb.N64[uy[ci], ux[ci]]
    r_data = data_residuals(ws["v"][ci], Vd, Nd)
    J_data = data_jacobian(ws["b"][ci], pb.surfel_pos[ci].astype(np.float64), Nd,
                           pb.w[ci], ws["s"][ci], ws["r"], ws["d"], ws["c"], pb.idx[ci])
    r_arap = arap_residuals(pb.node_pos, R, t, pb.nbr)
    Jj, Jm = arap_jacobians(pb.node_pos, R, pb.nbr)
    corr_map = np.full(I.shape, -1, dtype=np.int64)
    corr_map[uy[ci], ux[ci]] = ci
    return dict(ws=ws, I=I, corr=m, corr_idx=ci, ux=ux, uy=uy, corr_map=corr_map,
                r_data=r_data, J_data=J_data, r_arap=r_arap, Jj=Jj, Jm=Jm,
                e_data=float(np.sum(r_data ** 2)), e_reg=float(np.sum(r_arap ** 2)))


def _linearize_pairs(pb: Problem, R: np.ndarray, t: np.ndarray, ws: Dict, corr_map: Optional[np.ndarray]):
    """Splat rendering: one data row per pair (surfel, pixel); a surfel can
    hold several. corr_map, when given, supplies the pairs (pixel -> surfel)."""
    I, k, ux, uy = assoc.associate_splats(ws["v"], ws["n"], pb.splat_radius, ws["valid"], pb.frame, pb.cam,
                                          pb.corr_dist, pb.corr_normal)
    if corr_map is not None:
        cm = np.asarray(corr_map)
        uy, ux = np.nonzero(cm >= 0)
        k = cm[uy, ux]
    Vd = pb.V64[uy, ux]
    Nd = pb.N64[uy, ux]
    r_data = data_residuals(ws["v"][k], Vd, Nd)
    J_data = data_jacobian(ws["b"][k], pb.surfel_pos[k].astype(np.float64), Nd,
                           pb.w[k], ws["s"][k], ws["r"], ws["d"], ws["c"], pb.idx[k])
    r_arap = arap_residuals(pb.node_pos, R, t, pb.nbr)
    Jj, Jm = arap_jacobians(pb.node_pos, R, pb.nbr)
    cmap = np.full(I.shape, -1, dtype=np.int64)
    cmap[uy, ux] = k
    corr = np.zeros(pb.surfel_pos.shape[0], dtype=bool)
    corr[k] = True
    return dict(ws=ws, I=I, corr=corr, corr_idx=k, pair_ux=ux, pair_uy=uy, corr_map=cmap,
                r_data=r_data, J_data=J_data, r_arap=r_arap, Jj=Jj, Jm=Jm,
                e_data=float(np.sum(r_data ** 2)), e_reg=float(np.sum(r_arap ** 2)))


def stacked_jacobian(pb: Problem, lin: Dict):
    """Sparse J (rows: correspondences, then 3 rows per directed edge scaled
    by sqrt(lambda)) and the matching residual vector."""
    nn = pb.node_pos.shape[0]
    ci = lin["corr_idx"]
    nc = ci.size
    idx = pb.idx[ci]
    cols_d = (6 * idx[:, :, None] + np.arange(6)).reshape(nc, 24)
    vals_d = lin["J_data"].reshape(nc, 24)
    rows_d = np.repeat(np.arange(nc), 24)
    sl = np.sqrt(pb.lambda_reg)
    nbr = pb.nbr
    ne = nbr.size
    j = np.repeat(np.arange(nn), nbr.shape[1])
    m = nbr.ravel()
    Jj = lin["Jj"].reshape(ne, 3, 6)
    Jm = lin["Jm"].reshape(ne, 3, 6)
    rows_a = nc + (3 * np.arange(ne)[:, None] + np.arange(3))[:, :, None]  # (ne,3,1)
    rows_a = np.broadcast_to(rows_a, (ne, 3, 12))
    cols_a = np.concatenate([np.broadcast_to((6 * j[:, None] + np.arange(6))[:, None, :], (ne, 3, 6)),
                             np.broadcast_to((6 * m[:, None] + np.arange(6))[:, None, :], (ne, 3, 6))], 2)
    vals_a = sl * np.concatenate([Jj, Jm], 2)
    rows = np.concatenate([rows_d, rows_a.ravel()])
    cols = np.concatenate([cols_d.ravel(), cols_a.ravel()])
    vals = np.concatenate([vals_d.ravel(), vals_a.ravel()])
    J = sp.csr_matrix((vals, (rows, cols)), shape=(nc + 3 * ne, 6 * nn))
    res = np.concatenate([lin["r_data"], sl * lin["r_arap"].reshape(-1)])
    return J, res


def normal_equations(pb: Problem, lin: Dict):
    """A = J^T J + mu I (sparse CSR, 6N x 6N) and g = J^T r."""
    J, res = stacked_jacobian(pb, lin)
    n = J.shape[1]
    A = (J.T @ J).tocsr() + pb.damping * sp.identity(n, format="csr")
    g = J.T @ res
    return A.tocsr(), np.asarray(g).ravel()


def solve_cholesky(A, g: np.ndarray) -> np.ndarray:
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    c = scipy.linalg.cho_factor(Ad, lower=False, overwrite_a=True, check_finite=False)
    return -scipy.linalg.cho_solve(c, g, check_finite=False)


def block_jacobi(A, nn: int) -> np.ndarray:
    """(nn,6,6) inverses of the 6x6 diagonal blocks of A."""
    A = A.tocsr() if sp.issparse(A) else sp.csr_matrix(A)
    blocks = np.zeros((nn, 6, 6))
    for k in range(6):
        for l in range(6):
            blocks[:, k, l] = np.asarray(A[np.arange(nn) * 6 + k, np.arange(nn) * 6 + l]).ravel()
    return np.linalg.inv(blocks)


def solve_pcg(A, g: np.ndarray, iters: int, return_trace: bool = False):
    """Block-Jacobi PCG from x0 = 0 for exactly `iters` iterations on
    A Delta = -g (stops early only if rho = r^T z is exactly 0)."""
    nn = g.size // 6
    Minv = block_jacobi(A, nn)

    def prec(v):
        return np.einsum("nij,nj->ni", Minv, v.reshape(nn, 6)).ravel()

    x = np.zeros_like(g)
    r = -g.copy()
    z = prec(r)
    p = z.copy()
    rho = float(r @ z)
    trace: List[float] = []
    for _ in range(iters):
        if rho == 0.0:
            break
        q = A @ p
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = prec(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        trace.append(float(np.linalg.norm(r)))
    return (x, trace) if return_trace else x


def update_nodes(node_pos: np.ndarray, R: np.ndarray, t: np.ndarray, delta: np.ndarray):
    """T_k <- Delta_k o T_k: R' = Exp(w) R, t' = Exp(w)(t - c) + c + tau,
    c = R p + t the node's live position."""
    D = delta.reshape(-1, 6)
    E = exp_so3(D[:, :3])
    c = np.einsum("nij,nj->ni", R, node_pos.astype(np.float64)) + t
    R2 = E @ R
    t2 = np.einsum("nij,nj->ni", E, t - c) + c + D[:, 3:]
    return R2, t2


def gn_solve(pb: Problem, se3_init: np.ndarray, gn_iters: int, pcg_iters: Optional[int] = 10,
             linear: str = "pcg", final_energy: bool = False, keep: Optional[List[int]] = None,
             rigid_iters: int = 0, corr_maps: Optional[List[np.ndarray]] = None):
    """Run exactly gn_iters Gauss-Newton iterations from se3_init (after
    rigid_iters steps of rigid alignment composed into the nodes, see rigid.py).

    linear = "chol" solves each step exactly (dense Cholesky), "pcg" runs
    block-Jacobi PCG for pcg_iters iterations. Returns the final (Nn,12) [R|t]
    and a trace with the energies, correspondence counts and, for iterations
    listed in `keep`, the full linearisation. corr_maps[it], when given,
    supplies iteration it's correspondences (see linearize)."""
    R, t = se3_to_rt(se3_init)
    trace: Dict = dict(e_data=[], e_reg=[], n_corr=[], pcg_resid=[], lin={}, steps=[])
    if rigid_iters > 0:
        Rc, tc, trace["rigid"] = rigid.rigid_align(pb, warp_surfels(pb, R, t), rigid_iters, pb.damping)
        R, t = rigid.compose(R, t, Rc, tc)
    for it in range(gn_iters):
        lin = linearize(pb, R, t, None if corr_maps is None else corr_maps[it])
        trace["e_data"].append(lin["e_data"])
        trace["e_reg"].append(lin["e_reg"])
        trace["n_corr"].append(int(lin["corr_idx"].size))
        A, g = normal_equations(pb, lin)
        if linear == "chol":
            delta = solve_cholesky(A, g)
            trace["pcg_resid"].append(float(np.linalg.norm(A @ delta + g)))
        else:
            delta, rt = solve_pcg(A, g, pcg_iters, return_trace=True)
            trace["pcg_resid"].append(rt[-1] if rt else 0.0)
        if keep is not None and it in keep:
            lin = dict(lin)
            lin["A"], lin["g"], lin["delta"] = A, g, delta
            trace["lin"][it] = lin
        trace["steps"].append(delta)
        R, t = update_nodes(pb.node_pos, R, t, delta)
    if final_energy:
        lin = linearize(pb, R, t)
        trace["e_final"] = (lin["e_data"], lin["e_reg"], int(lin["corr_idx"].size))
    return rt_to_se3(R, t), trace


def oracle_solve(cam, surfel_pos, surfel_nrm, node_pos, depth, params,
                 se3_init=None, linear: str = "pcg", visible=None, splat_radius=None, **kw):
    """One frame solve from a scene's inputs (skinning and graph included)."""
    pb = make_problem(cam, surfel_pos, surfel_nrm, node_pos, depth, params, visible=visible,
                      splat_radius=splat_radius)
    if se3_init is None:
        se3_init = identity_se3(node_pos.shape[0])
    kw.setdefault("rigid_iters", getattr(params, "rigid_iters", 0))
    return gn_solve(pb, se3_init, params.gn_iters, params.pcg_iters, linear=linear, **kw)


def identity_se3(n: int) -> np.ndarray:
    out = np.zeros((n, 12))
    out[:, 0] = out[:, 5] = out[:, 10] = 1.0
    return out
