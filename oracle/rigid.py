"""Rigid alignment before the non-rigid solve (FP64). Test infrastructure only.

Sec. 7 (last paragraph before Sec. 8): before the non-rigid estimation a rigid
alignment is performed with the method of KinectFusion, i.e. projective
point-to-plane ICP of one rigid transform.

Readings taken here:
* the rigid transform T = (R_c, t_c) acts after the current warp field: the
  live surfels are y_i = R_c v'_i + t_c (normals R_c n'_i), v'_i the surfels
  warped by the node transforms;
* association, gates and the index map are those of the data term (Sec. 7),
  taken on y_i;
* residual r_i = N(u_i)^T (y_i - V(u_i)); Gauss-Newton on a left twist about
  the camera origin, T <- (Exp(w) R_c, Exp(w) t_c + tau); the linearised
  residual is r_i + J_i . xi with J_i = (y_i x N(u_i), N(u_i));
* each step solves (sum J_i J_i^T + mu I) xi = -sum J_i r_i (mu = the
  solver's damping), a fixed number of steps, no early exit;
* the result is composed into every node, T_k <- T o T_k, before the
  non-rigid Gauss-Newton iterations.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from . import assoc
from .quat import exp_so3


def rigid_linearize(pb, ws: Dict, Rc: np.ndarray, tc: np.ndarray):
    """Residuals, 6-column Jacobian and correspondence indices of the rigid
    alignment at T = (Rc, tc), from the warped surfels `ws` (see
    solve.warp_surfels)."""
    y = ws["v"] @ Rc.T + tc
    ny = ws["n"] @ Rc.T
    _, m, ux, uy = assoc.associate(y, ny, ws["valid"], pb.frame, pb.cam, pb.corr_dist, pb.corr_normal)
    ci = np.flatnonzero(m)
    Vd = pb.V64[uy[ci], ux[ci]]
    Nd = pb.N64[uy[ci], ux[ci]]
    yc = y[ci]
    r = np.sum(Nd * (yc - Vd), axis=1)
    J = np.concatenate([np.cross(yc, Nd), Nd], axis=1)
    return r, J, ci


def rigid_step(r: np.ndarray, J: np.ndarray, damping: float) -> np.ndarray:
    """xi = (w, tau) solving (J^T J + mu I) xi = -J^T r."""
    A = J.T @ J + damping * np.eye(6)
    return -np.linalg.solve(A, J.T @ r)


def apply_step(Rc: np.ndarray, tc: np.ndarray, xi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    E = exp_so3(xi[None, :3])[0]
    return E @ Rc, E @ tc + xi[3:]


def rigid_align(pb, ws: Dict, iters: int, damping: float):
    """`iters` point-to-plane ICP steps from the identity; returns (Rc, tc)
    and a trace of the energies and correspondence counts at each step."""
    Rc, tc = np.eye(3), np.zeros(3)
    trace: Dict[str, List] = dict(e=[], n_corr=[], steps=[])
    for _ in range(iters):
        r, J, ci = rigid_linearize(pb, ws, Rc, tc)
        trace["e"].append(float(r @ r))
        trace["n_corr"].append(int(ci.size))
        xi = rigid_step(r, J, damping)
        trace["steps"].append(xi)
        Rc, tc = apply_step(Rc, tc, xi)
    return Rc, tc, trace


def compose(R: np.ndarray, t: np.ndarray, Rc: np.ndarray, tc: np.ndarray):
    """Node transforms after the rigid alignment: T_k <- T o T_k."""
    return np.einsum("ij,njk->nik", Rc, R), t @ Rc.T + tc
