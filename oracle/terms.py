"""Residuals, energies and Jacobians of the two energy terms (Sec. 7), FP64.

E_total = E_depth + lambda E_regulation (Sec. 7, energy equation), with

  E_depth = sum over (s_model, s_depth) in P of (n_depth^T (v_model - v_depth))^2
  E_regulation = sum_j sum_{i in N_j} |T_j p_j - T_i p_j|^2.

Parameterisation (the paper does not give one): node k's transform is
perturbed on the left about its live position c_k = T_k p_k,
T_k <- Delta_k o T_k with Delta_k(x) = Exp(w_k)(x - c_k) + c_k + tau_k and the
unknown xi_k = (w_k, tau_k). Association is held fixed while differentiating.
"""
from __future__ import annotations

import numpy as np

from .quat import skew
from .warp import dF_db, perturb_matrix


def data_residuals(v_live: np.ndarray, Vd: np.ndarray, Nd: np.ndarray) -> np.ndarray:
    """r_i = N(u_i)^T (v_i - V(u_i))."""
    return np.sum(Nd * (v_live - Vd), axis=1)


def data_jacobian(b: np.ndarray, v_ref: np.ndarray, Nd: np.ndarray, w: np.ndarray,
                  s: np.ndarray, node_r: np.ndarray, node_d: np.ndarray,
                  node_c: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """(N,K,6) Jacobian of r_i with respect to xi of its K nodes:
    J_ik = N(u_i)^T dF/db(b_i; v_i) w_ik s_ik M(q_k, c_k) (chain rule through
    the blend b_i = sum_k w_ik s_ik q_k)."""
    G = np.einsum("ni,nij->nj", Nd, dF_db(b, v_ref))            # (N,8)
    K = idx.shape[1]
    out = np.zeros((b.shape[0], K, 6))
    for k in range(K):
        nk = idx[:, k]
        M = perturb_matrix(node_r[nk], node_d[nk], node_c[nk])  # (N,8,6)
        out[:, k, :] = (w[:, k] * s[:, k])[:, None] * np.einsum("nj,njc->nc", G, M)
    return out


def arap_residuals(node_pos: np.ndarray, R: np.ndarray, t: np.ndarray,
                   nbr: np.ndarray) -> np.ndarray:
    """(N,k,3) residuals r_jm = T_j p_j - T_m p_j for m in N_j."""
    p = node_pos.astype(np.float64)
    c = np.einsum("nij,nj->ni", R, p) + t                          # T_j p_j
    Rm = R[nbr]                                                    # (N,k,3,3)
    Tm_pj = np.einsum("nkij,nj->nki", Rm, p) + t[nbr]
    return c[:, None, :] - Tm_pj


def arap_jacobians(node_pos: np.ndarray, R: np.ndarray, nbr: np.ndarray):
    """d r_jm / d xi_j = [0 | I] and d r_jm / d xi_m = [[y]x | -I] with
    y = T_m p_j - c_m = R_m (p_j - p_m). Returns (Jj, Jm), each (N,k,3,6)."""
    p = node_pos.astype(np.float64)
    n, k = nbr.shape
    y = np.einsum("nkij,nkj->nki", R[nbr], p[:, None, :] - p[nbr])
    Jj = np.zeros((n, k, 3, 6))
    Jj[..., 3:] = np.eye(3)
    Jm = np.zeros((n, k, 3, 6))
    Jm[..., :3] = skew(y)
    Jm[..., 3:] = -np.eye(3)
    return Jj, Jm
