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


def test_motion_walk_steps_are_fresh_and_bounded():
    """The served streams' frames: every step of the walk is a rotation of at
    most 2 deg about each node's live position plus a translation of at most
    5 mm, composed after the previous frame's motion; frame 0 is the scene's."""
    from scipy.spatial.transform import Rotation

    from gen.scenes import motion_walk
    s = scene_random(401, size=(320, 240), n_nodes=300, n_surfels=6000)
    walk = motion_walk(s, 4, seed=11)
    assert len(walk) == 4 and np.array_equal(walk[0], s.gt_se3.reshape(-1, 12))
    p = s.node_pos.astype(np.float64)
    for a, b in zip(walk[:-1], walk[1:]):
        A, B = a.reshape(-1, 3, 4), b.reshape(-1, 3, 4)
        # the step D = B A^-1 as a transform of live points
        Ra, ta, Rb, tb = A[:, :, :3], A[:, :, 3], B[:, :, :3], B[:, :, 3]
        Rd = Rb @ np.transpose(Ra, (0, 2, 1))
        td = tb - np.einsum("nij,nj->ni", Rd, ta)
        ang = np.degrees(Rotation.from_matrix(Rd).magnitude())
        assert ang.max() <= 2.0 + 1e-6 and ang.max() > 0.5
        live = np.einsum("nij,nj->ni", Ra, p) + ta                     # each node's live position
        moved = np.einsum("nij,nj->ni", Rd, live) + td - live          # the step's translation there
        assert np.linalg.norm(moved, axis=1).max() <= 0.005 + 1e-9
    assert not np.array_equal(walk[1], walk[2])


def test_ping_pong_playback_steps_one_frame_at_a_time():
    import bench
    seq = [bench.ping_pong(k, 4) for k in range(13)]
    assert seq[:7] == [1, 2, 3, 2, 1, 0, 1]
    assert all(abs(a - b) == 1 for a, b in zip(seq[:-1], seq[1:]))
    assert all(bench.ping_pong(k, 1) == 0 for k in range(3))
    tr = bench.arrival_trace(3, 30.0, 1.0, seed=2)
    assert all(t0 <= t1 for (t0, _, _), (t1, _, _) in zip(tr[:-1], tr[1:]))
    for i in range(3):
        ks = [k for _, s, k in tr if s == i]
        assert ks == list(range(len(ks)))                         # each stream's arrivals in order
