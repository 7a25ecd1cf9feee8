"""Seeded scene generator: determinism and workload shape."""
import numpy as np

from gen.scenes import make_scene, scene_random


def test_seeded_determinism():
    a = make_scene("tiny")
    b = make_scene("tiny")
    for f in ("surfel_pos", "surfel_nrm", "node_pos", "gt_se3", "depth"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = make_scene("tiny", seed=8)
    assert not np.array_equal(a.depth, c.depth)


def test_c1_shape(scene_cache):
    s = scene_cache("c1")
    assert s.depth.shape == (120, 160) and s.depth.dtype == np.float32
    assert s.node_pos.shape == (200, 3)
    # about 18k surfels on the unit sphere's near cap (stated as ~15k)
    assert 15000 <= s.surfel_pos.shape[0] <= 19200
    nrm = np.linalg.norm(s.surfel_nrm.astype(np.float64), axis=1)
    assert np.allclose(nrm, 1.0, atol=1e-6)
    # normals face the camera
    assert np.all(np.sum(s.surfel_nrm * s.surfel_pos, axis=1) < 0)
    # node spacing: at least 2.5 cm apart
    from scipy.spatial import cKDTree
    d, _ = cKDTree(s.node_pos).query(s.node_pos, k=2)
    assert d[:, 1].min() >= 0.025 - 1e-6


def test_gt_motion_bounds(scene_cache):
    s = scene_cache("c1")
    M = s.gt_se3.reshape(-1, 3, 4)
    ang = np.degrees(np.arccos(np.clip((np.trace(M[:, :, :3], axis1=1, axis2=2) - 1) / 2, -1, 1)))
    assert ang.max() <= 3.0 + 1e-9
    p = s.node_pos.astype(np.float64)
    disp = np.einsum("nij,nj->ni", M[:, :, :3], p) + M[:, :, 3] - p
    assert np.linalg.norm(disp, axis=1).max() <= 0.005 + 1e-9


def test_random_stream_ranges():
    s = scene_random(400, size=(320, 240), n_nodes=300, n_surfels=5000)
    assert s.depth.shape == (240, 320)
    assert s.surfel_pos.shape[0] == 5000
    assert s.node_pos.shape[0] == 300
