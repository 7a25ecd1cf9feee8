"""Pins of the oracle's quaternion algebra against SciPy's rotations."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import quat as Q

rng = np.random.default_rng(11)


def _rand_quats(n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _scipy_q(q):  # scipy is scalar-last
    return Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1))


def test_matrix_from_quat_matches_scipy():
    q = _rand_quats(50)
    assert np.allclose(Q.matrix_from_quat(q), _scipy_q(q).as_matrix(), atol=1e-12)


def test_product_composes_rotations():
    a, b = _rand_quats(50), _rand_quats(50)
    Rab = Q.matrix_from_quat(Q.qmul(a, b))
    ref = _scipy_q(a).as_matrix() @ _scipy_q(b).as_matrix()
    assert np.allclose(Rab, ref, atol=1e-12)


def test_left_right_matrices():
    a, b = rng.normal(size=(20, 4)), rng.normal(size=(20, 4))
    ab = Q.qmul(a, b)
    assert np.allclose(np.einsum("nij,nj->ni", Q.qleft(a), b), ab)
    assert np.allclose(np.einsum("nij,nj->ni", Q.qright(b), a), ab)


def test_quat_from_matrix_roundtrip_and_canonical():
    R = Rotation.random(200, random_state=3).as_matrix()
    q = Q.quat_from_matrix(R)
    assert np.all(q[:, 0] >= 0)
    assert np.allclose(Q.matrix_from_quat(q), R, atol=1e-12)
    # near-180 degree rotations take the non-trace branches
    R2 = Rotation.from_rotvec(np.array([[np.pi - 1e-9, 0, 0], [0, np.pi, 0], [0, 0, 3.1]])).as_matrix()
    assert np.allclose(Q.matrix_from_quat(Q.quat_from_matrix(R2)), R2, atol=1e-9)


def test_exp_so3_matches_scipy():
    w = rng.normal(size=(100, 3)) * rng.uniform(0, 2, size=(100, 1))
    assert np.allclose(Q.exp_so3(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-12)
    tiny = np.array([[1e-10, -2e-10, 3e-11]])
    assert np.allclose(Q.exp_so3(tiny), Rotation.from_rotvec(tiny).as_matrix(), atol=1e-18)


@pytest.mark.parametrize("n", [1, 30])
def test_dual_quaternion_applies_rigid_transform(n):
    R = Rotation.random(n, random_state=5).as_matrix()
    t = rng.normal(size=(n, 3))
    r, d = Q.dq_from_rt(R, t)
    x = rng.normal(size=(n, 3))
    # r (0,x) r* + 2 d r*  must equal R x + t
    rot = Q.qmul(Q.qmul(r, Q.pure(x)), Q.qconj(r))[:, 1:]
    tr = 2.0 * Q.qmul(d, Q.qconj(r))[:, 1:]
    assert np.allclose(rot + tr, np.einsum("nij,nj->ni", R, x) + t, atol=1e-12)
    R2, t2 = Q.rt_from_dq(r, d)
    assert np.allclose(R2, R, atol=1e-12) and np.allclose(t2, t, atol=1e-12)
