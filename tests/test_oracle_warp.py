"""Pins of the dual-quaternion blend (Eq. 1, Eq. 2) and its derivatives."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import quat as Q
from oracle import warp as Wp

rng = np.random.default_rng(21)


def _nodes(n, max_deg=30.0, max_t=0.1):
    rv = rng.normal(size=(n, 3))
    rv *= np.deg2rad(max_deg) * rng.random((n, 1)) / np.linalg.norm(rv, axis=1, keepdims=True)
    R = Rotation.from_rotvec(rv).as_matrix()
    t = rng.uniform(-max_t, max_t, size=(n, 3))
    r, d = Q.dq_from_rt(R, t)
    return R, t, r, d


def test_single_node_is_exact_rigid_transform():
    R, t, r, d = _nodes(5)
    v = rng.normal(size=(50, 3))
    nv = rng.normal(size=(50, 3))
    nv /= np.linalg.norm(nv, axis=1, keepdims=True)
    for k in range(5):
        idx = np.full((50, 4), k)
        w = rng.random((50, 4)) + 0.1
        b, _ = Wp.blend(idx, w, r, d)
        vl, nl, ok = Wp.apply_blend(b, v, nv)
        assert ok.all()
        assert np.allclose(vl, v @ R[k].T + t[k], atol=1e-12)
        assert np.allclose(nl, nv @ R[k].T, atol=1e-12)


def test_equal_transforms_blend_to_that_transform_and_sign_invariance():
    R, t, r, d = _nodes(1)
    r4 = np.repeat(r, 4, 0)
    d4 = np.repeat(d, 4, 0)
    # node 2 stored with the opposite sign: the same transform
    r4[2] *= -1
    d4[2] *= -1
    idx = np.tile(np.arange(4), (30, 1))
    w = rng.random((30, 4)) + 0.01
    v = rng.normal(size=(30, 3))
    b, s = Wp.blend(idx, w, r4, d4)
    assert np.all(s[:, 2] == -1) and np.all(s[:, [0, 1, 3]] == 1)
    vl, _, _ = Wp.apply_blend(b, v)
    assert np.allclose(vl, v @ R[0].T + t[0], atol=1e-12)


def test_weight_scale_and_reference_sign_invariance():
    R, t, r, d = _nodes(8)
    idx = np.array([rng.choice(8, 4, replace=False) for _ in range(40)])
    w = rng.random((40, 4)) + 0.05
    v = rng.normal(size=(40, 3)) * 0.2
    b1, _ = Wp.blend(idx, w, r, d)
    b2, _ = Wp.blend(idx, 7.3 * w, r, d)
    r_flip, d_flip = r.copy(), d.copy()
    r_flip[idx[:, 0]] *= -1      # flip every reference node
    d_flip[idx[:, 0]] *= -1
    b3, _ = Wp.blend(idx, w, r_flip, d_flip)
    v1, _, _ = Wp.apply_blend(b1, v)
    v2, _, _ = Wp.apply_blend(b2, v)
    v3, _, _ = Wp.apply_blend(b3, v)
    assert np.allclose(v1, v2, atol=1e-12) and np.allclose(v1, v3, atol=1e-12)


def test_identity_blend_is_exact():
    r = np.tile([1.0, 0, 0, 0], (6, 1))
    d = np.zeros((6, 4))
    idx = np.array([rng.choice(6, 4, replace=False) for _ in range(100)])
    w = rng.random((100, 4))
    w /= w.sum(1, keepdims=True)
    v = rng.normal(size=(100, 3))
    n = rng.normal(size=(100, 3))
    b, _ = Wp.blend(idx, w, r, d)
    vl, nl, _ = Wp.apply_blend(b, v, n)
    assert np.array_equal(vl, v) and np.array_equal(nl, n)


def test_homogeneous_form_equals_normalised_form():
    R, t, r, d = _nodes(8)
    idx = np.array([rng.choice(8, 4, replace=False) for _ in range(60)])
    w = rng.random((60, 4)) + 0.05
    v = rng.normal(size=(60, 3))
    b, _ = Wp.blend(idx, w, r, d)
    vl, _, _ = Wp.apply_blend(b, v)
    assert np.allclose(Wp.F_homogeneous(b, v), vl, atol=1e-12)


def test_dF_db_finite_differences():
    R, t, r, d = _nodes(8)
    idx = np.array([rng.choice(8, 4, replace=False) for _ in range(20)])
    w = rng.random((20, 4)) + 0.05
    v = rng.normal(size=(20, 3))
    b, _ = Wp.blend(idx, w, r, d)
    J = Wp.dF_db(b, v)
    h = 1e-6
    for j in range(8):
        e = np.zeros(8)
        e[j] = h
        fd = (Wp.apply_blend(b + e, v)[0] - Wp.apply_blend(b - e, v)[0]) / (2 * h)
        assert np.allclose(J[:, :, j], fd, rtol=1e-6, atol=1e-7), j


def test_perturb_matrix_finite_differences():
    R, t, r, d = _nodes(6, max_deg=60)
    p = rng.normal(size=(6, 3)) * 0.3
    c = np.einsum("nij,nj->ni", R, p) + t
    M = Wp.perturb_matrix(r, d, c)
    h = 1e-6
    for j in range(6):
        xi = np.zeros((6, 6))
        xi[:, j] = h

        def dq(sign):
            E = Q.exp_so3(sign * xi[:, :3])
            R2 = E @ R
            t2 = np.einsum("nij,nj->ni", E, t - c) + c + sign * xi[:, 3:]
            r2, d2 = Q.dq_from_rt(R2, t2)
            # keep the hemisphere of the unperturbed quaternion
            sg = np.where(np.sum(r2 * r, 1) < 0, -1.0, 1.0)[:, None]
            return np.concatenate([r2 * sg, d2 * sg], 1)
        fd = (dq(1) - dq(-1)) / (2 * h)
        assert np.allclose(M[:, :, j], fd, atol=1e-7), j
