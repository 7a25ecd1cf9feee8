"""Pins of residuals, Jacobians and the Gauss-Newton system (finite differences)."""
import numpy as np
import pytest

from oracle import quat as Q
from oracle import solve as S
from oracle.terms import arap_jacobians, arap_residuals


def _perturbed(pb, R, t, k, xi):
    """State with node k moved by Delta_k(xi) o T_k (exact exponential)."""
    R2, t2 = R.copy(), t.copy()
    c = R[k] @ pb.node_pos[k].astype(np.float64) + t[k]
    E = Q.exp_so3(xi[:3][None])[0]
    R2[k] = E @ R[k]
    t2[k] = E @ (t[k] - c) + c + xi[3:]
    return R2, t2


def _frozen_residuals(pb, lin, R, t):
    """Stacked residual vector at (R, t) with the association of `lin` frozen:
    data rows for the same surfels against the same pixels, then sqrt(lambda)
    times the regulariser rows."""
    ws = S.warp_surfels(pb, R, t)
    ci = lin["corr_idx"]
    uy, ux = lin["uy"][ci], lin["ux"][ci]
    Vd, Nd = pb.V64[uy, ux], pb.N64[uy, ux]
    rd = np.sum(Nd * (ws["v"][ci] - Vd), axis=1)
    ra = arap_residuals(pb.node_pos, R, t, pb.nbr).reshape(-1)
    return np.concatenate([rd, np.sqrt(pb.lambda_reg) * ra])


@pytest.fixture(scope="module")
def tiny_state(scene_cache):
    s = scene_cache("tiny")
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params)
    R, t = Q.se3_to_rt(s.gt_se3)
    # move away from the ground truth so that node transforms all differ
    rng = np.random.default_rng(9)
    for k in range(R.shape[0]):
        R, t = _perturbed(pb, R, t, k, np.r_[rng.normal(size=3) * 0.02, rng.normal(size=3) * 0.003])
    lin = S.linearize(pb, R, t)
    return pb, R, t, lin


def test_data_jacobian_finite_differences(tiny_state):
    pb, R, t, lin = tiny_state
    ci = lin["corr_idx"]
    nc = ci.size
    assert nc > 1000
    h = 1e-6
    worst = 0.0
    scale = np.abs(lin["J_data"]).max()
    for k in range(0, pb.node_pos.shape[0], 3):
        rows, slots = np.nonzero(pb.idx[ci] == k)
        if rows.size == 0:
            continue
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            rp = _frozen_residuals(pb, lin, *_perturbed(pb, R, t, k, e))[:nc]
            rm = _frozen_residuals(pb, lin, *_perturbed(pb, R, t, k, -e))[:nc]
            fd = (rp - rm) / (2 * h)
            an = lin["J_data"][rows, slots, c]
            worst = max(worst, np.max(np.abs(fd[rows] - an)))
            others = np.setdiff1d(np.arange(nc), rows)
            assert np.max(np.abs(fd[others])) < 1e-9
    assert worst < 1e-6 * max(scale, 1.0)


def test_data_jacobian_equal_transforms_closed_form(scene_cache):
    s = scene_cache("tiny")
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params)
    n = s.node_pos.shape[0]
    Rr = Q.exp_so3(np.array([0.03, -0.02, 0.05]))
    R = np.repeat(Rr[None], n, 0)
    t = np.repeat(np.array([[0.004, -0.002, 0.003]]), n, 0)
    lin = S.linearize(pb, R, t)
    ci = lin["corr_idx"]
    v = lin["ws"]["v"][ci]
    Nd = pb.N64[lin["uy"][ci], lin["ux"][ci]]
    c = lin["ws"]["c"][pb.idx[ci]]                       # (Nc,4,3)
    w = pb.w[ci]
    ref = np.concatenate([np.cross(v[:, None, :] - c, Nd[:, None, :]),
                          np.broadcast_to(Nd[:, None, :], c.shape)], axis=2) * w[..., None]
    assert np.allclose(lin["J_data"], ref, atol=1e-10)


def test_arap_jacobian_finite_differences(tiny_state):
    pb, R, t, _ = tiny_state
    Jj, Jm = arap_jacobians(pb.node_pos, R, pb.nbr)
    h = 1e-6
    for k in range(0, pb.node_pos.shape[0], 4):
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            rp = arap_residuals(pb.node_pos, *_perturbed(pb, R, t, k, e), pb.nbr)
            rm = arap_residuals(pb.node_pos, *_perturbed(pb, R, t, k, -e), pb.nbr)
            fd = (rp - rm) / (2 * h)                          # (N,8,3)
            an = np.zeros_like(fd)
            an[k] += Jj[k, :, :, c]
            an += np.where((pb.nbr == k)[..., None], Jm[..., c], 0.0)
            assert np.allclose(fd, an, atol=1e-8), (k, c)


def test_normal_equations_match_fd_jacobian(tiny_state):
    pb, R, t, lin = tiny_state
    A, g = S.normal_equations(pb, lin)
    nn = pb.node_pos.shape[0]
    h = 1e-6
    r0 = _frozen_residuals(pb, lin, R, t)
    Jfd = np.zeros((r0.size, 6 * nn))
    for k in range(nn):
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Jfd[:, 6 * k + c] = (_frozen_residuals(pb, lin, *_perturbed(pb, R, t, k, e))
                                 - _frozen_residuals(pb, lin, *_perturbed(pb, R, t, k, -e))) / (2 * h)
    Ad = A.toarray()
    Hfd = Jfd.T @ Jfd + pb.damping * np.eye(6 * nn)
    assert np.allclose(Ad, Ad.T, atol=0)
    assert np.linalg.norm(Ad - Hfd) <= 1e-6 * np.linalg.norm(Hfd)
    assert np.linalg.norm(g - Jfd.T @ r0) <= 1e-6 * max(np.linalg.norm(g), 1e-12)
    # the stacked residual carries the energy: E_data + lambda E_reg
    assert np.isclose(r0 @ r0, lin["e_data"] + pb.lambda_reg * lin["e_reg"], rtol=1e-12)
    ev = np.linalg.eigvalsh(Ad)
    assert ev.min() >= pb.damping * (1 - 1e-6)
