"""Pins of the rigid alignment (oracle/rigid.py) against facts that do not
come from its own formulas: finite differences of the residual, exact
recovery of a rigidly moved surface, the identity frame, and the
left-equivariance of the dual-quaternion blend that the composition into the
nodes relies on."""
import numpy as np
from scipy.spatial.transform import Rotation

from gen.scenes import SolverParams
from oracle import quat as Q
from oracle import rigid as RG
from oracle import solve as S
from test_oracle_solve import _rigid_scene, exact_identity_problem


def test_jacobian_matches_finite_differences(scene_cache):
    s = scene_cache("tiny")
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params)
    R, t = Q.se3_to_rt(s.gt_se3)
    ws = S.warp_surfels(pb, R, t)
    rng = np.random.default_rng(3)
    Rc = Rotation.from_rotvec(rng.normal(size=3) * 0.01).as_matrix()
    tc = rng.normal(size=3) * 0.002
    r, J, ci = RG.rigid_linearize(pb, ws, Rc, tc)
    assert ci.size > 50
    # residual of the frozen correspondences as a function of the twist
    y_all = ws["v"] @ Rc.T + tc
    _, _, ux, uy = S.assoc.associate(y_all, ws["n"] @ Rc.T, ws["valid"], pb.frame, pb.cam, pb.corr_dist,
                                     pb.corr_normal)
    y0 = y_all[ci]
    Vd, Nd = pb.V64[uy[ci], ux[ci]], pb.N64[uy[ci], ux[ci]]

    def res(xi):
        E = Rotation.from_rotvec(xi[:3]).as_matrix()
        y = y0 @ E.T + xi[3:]
        return np.sum(Nd * (y - Vd), axis=1)

    h = 1e-6
    fd = np.stack([(res(h * e) - res(-h * e)) / (2 * h) for e in np.eye(6)], axis=1)
    assert np.allclose(res(np.zeros(6)), r, atol=1e-12)
    assert np.max(np.abs(fd - J)) <= 1e-6 * max(1.0, np.max(np.abs(J)))


def test_recovers_a_rigid_motion_exactly():
    cam, pos, nrm, nodes, depth, params, Rs, ts = _rigid_scene()
    pb = S.make_problem(cam, pos, nrm, nodes, depth, params)
    R, t = Q.se3_to_rt(S.identity_se3(nodes.shape[0]))
    Rc, tc, tr = RG.rigid_align(pb, S.warp_surfels(pb, R, t), 8, params.damping)
    ang = Rotation.from_matrix(Rc @ Rs.T).magnitude()
    assert ang < 1e-6, ang
    assert np.linalg.norm(tc - ts) < 1e-6
    assert tr["e"][-1] < 1e-10 * tr["e"][0]


def test_identity_frame_gives_a_zero_step():
    cam, depth, pos, nrm, nodes, params = exact_identity_problem()
    pb = S.make_problem(cam, pos, nrm, nodes, depth, params)
    R, t = Q.se3_to_rt(S.identity_se3(nodes.shape[0]))
    Rc, tc, tr = RG.rigid_align(pb, S.warp_surfels(pb, R, t), 2, params.damping)
    assert all(np.all(x == 0) for x in tr["steps"])
    assert np.array_equal(Rc, np.eye(3)) and np.array_equal(tc, np.zeros(3))


def test_composed_nodes_warp_like_the_rigid_transform_after_the_blend(scene_cache):
    # blending T o T_k equals T applied to the blend of T_k (left-multiplying
    # every node's dual quaternion by one unit dual quaternion keeps the
    # hemisphere signs and commutes with the normalisation)
    s = scene_cache("tiny")
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params)
    R, t = Q.se3_to_rt(s.gt_se3)
    Rc = Rotation.from_rotvec([0.05, -0.02, 0.03]).as_matrix()
    tc = np.array([0.01, -0.02, 0.005])
    a = S.warp_surfels(pb, *RG.compose(R, t, Rc, tc))
    b = S.warp_surfels(pb, R, t)
    assert np.allclose(a["v"], b["v"] @ Rc.T + tc, atol=1e-12)
    assert np.allclose(a["n"], b["n"] @ Rc.T, atol=1e-12)
    assert np.array_equal(a["valid"], b["valid"])


def test_rigid_then_nonrigid_solve_runs_and_lowers_the_energy(scene_cache):
    s = scene_cache("tiny")
    params = SolverParams(**{**s.params.__dict__, "rigid_iters": 3})
    se3, tr = S.oracle_solve(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, params,
                             linear="chol", final_energy=True)
    assert len(tr["rigid"]["e"]) == 3 and tr["rigid"]["e"][-1] <= tr["rigid"]["e"][0]
    ef = tr["e_final"][0] + params.lambda_reg * tr["e_final"][1]
    assert ef < tr["e_data"][0] + params.lambda_reg * tr["e_reg"][0]
