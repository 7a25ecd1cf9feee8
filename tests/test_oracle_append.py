"""Pins of the append-candidate oracle (Sec. 6.2 live skinning and Eq. 7,
Sec. 6.3 compressive test and Eq. 8, Sec. 6.4 weight-sum test) against brute
force, closed forms and the definition of the largest stretch."""
import numpy as np
from scipy.spatial.transform import Rotation

from gen.scenes import Camera
from oracle import append as A
from oracle import fusion as F
from oracle import replica32 as R32
from oracle.quat import dq_from_rt


def _tables(R, t):
    r, d = dq_from_rt(R, t)
    return r, d


def test_live_skinning_is_the_brute_force_nearest_set_and_ratio_test():
    rng = np.random.default_rng(0)
    ref = rng.uniform(-0.1, 0.1, (60, 3)).astype(np.float32)
    live = (ref + rng.normal(0, 0.006, ref.shape)).astype(np.float32)
    q = rng.uniform(-0.1, 0.1, (500, 3)).astype(np.float32)
    q[7] = live[3]                          # on a node: key 0
    idx, keep = A.live_skinning(q, live, ref, 0.2)
    for i in range(q.shape[0]):
        d = [(float(np.sum((q[i].astype(np.float64) - live[j]) ** 2)), j) for j in range(live.shape[0])]
        want = [j for _, j in sorted(d)[:4]]
        assert idx[i].tolist() == want
        for k in range(1, 4):
            a, b = idx[i, 0], idx[i, k]
            ratio = np.linalg.norm(live[b].astype(np.float64) - live[a]) / np.linalg.norm(ref[b].astype(np.float64) - ref[a])
            if abs(ratio - 0.8) > 1e-5 and abs(ratio - 1.2) > 1e-5:
                assert keep[i, k] == (0.8 < ratio < 1.2)
    assert keep[:, 0].all() and idx[7, 0] == 3
    assert 0.05 < keep[:, 1:].mean() < 0.95          # both outcomes occur


def test_rigid_field_warps_back_exactly_and_does_not_stretch():
    rng = np.random.default_rng(1)
    n = 30
    ref = rng.uniform(-0.08, 0.08, (n, 3))
    Rm = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    tv = np.array([0.02, -0.01, 0.03])
    live = ref @ Rm.T + tv
    r, d = _tables(np.repeat(Rm[None], n, 0), np.repeat(tv[None], n, 0))
    x = rng.uniform(-0.06, 0.06, (200, 3)) @ Rm.T + tv
    nl = rng.normal(size=(200, 3))
    nl /= np.linalg.norm(nl, axis=1, keepdims=True)
    idx, keep = A.live_skinning(x.astype(np.float32), live.astype(np.float32), ref.astype(np.float32), 0.2)
    assert keep.all()                       # a rigid motion keeps every distance
    vr, nr = A.warp_back(x, nl, live, r, d, idx, keep, 0.025)
    assert np.max(np.abs(vr - (x - tv) @ Rm)) < 1e-12
    assert np.max(np.abs(nr - nl @ Rm)) < 1e-12
    s, Fm = A.stretch(x, live, r, d, idx, keep, 0.025)
    assert np.max(np.abs(s - 1.0)) < 1e-9
    assert np.max(np.abs(Fm - Rm.T[None])) < 1e-9


def _two_node_line(t1):
    """Nodes 0 and 1 on the x axis 6 cm apart, node 1 translated by t1 along
    x; nodes 2 and 3 half a metre away (weights ~e^-200)."""
    ref = np.array([[0.0, 0, 1], [0.06, 0, 1], [0.0, 0.5, 1], [0.0, -0.5, 1]])
    t = np.zeros((4, 3))
    t[1, 0] = t1
    live = ref + t
    r, d = _tables(np.repeat(np.eye(3)[None], 4, 0), t)
    return ref, live, r, d


def test_stretch_closed_form_on_a_line():
    """Translations along x only: x_ref(x) = x - w1(x) t1 on the axis, and
    d w1 / dx = w0 w1 (c1 - c0) / sigma^2; at the live midpoint w0 = w1 = 1/2,
    so the stretch is 1 - t1 (c1 - c0) / (4 sigma^2) along x and 1 across."""
    sig = 0.025
    for t1, compressive in ((-0.011, True), (-0.005, False), (0.008, False)):
        ref, live, r, d = _two_node_line(t1)
        mid = 0.5 * (live[0] + live[1])
        idx = np.array([[0, 1, 2, 3]])
        keep = np.array([[True, True, True, True]])
        s, Fm = A.stretch(mid[None], live, r, d, idx, keep, sig)
        gap = live[1, 0] - live[0, 0]
        want = 1.0 - t1 * gap / (4 * sig * sig)
        assert abs(Fm[0, 0, 0] - want) < 2e-3 * abs(want - 1.0) + 1e-9
        assert np.allclose(Fm[0, 1:, 1:], np.eye(2), atol=1e-9)
        assert abs(s[0] - max(abs(want), 1.0)) < 1e-3
        assert (s[0] > 1.2) == compressive
        vr, _ = A.warp_back(mid[None], None, live, r, d, idx, keep, sig)
        assert abs(vr[0, 0] - (mid[0] - 0.5 * t1)) < 1e-12


def test_stretch_is_the_largest_directional_stretch():
    rng = np.random.default_rng(2)
    n = 40
    ref = rng.uniform(-0.06, 0.06, (n, 3)) + [0, 0, 1.0]
    Rs = Rotation.from_rotvec(rng.normal(0, 0.15, (n, 3))).as_matrix()
    ts = rng.normal(0, 0.004, (n, 3))
    live = np.einsum("nij,nj->ni", Rs, ref) + ts
    r, d = _tables(Rs, ts)
    x = live[rng.choice(n, 25)] + rng.normal(0, 0.004, (25, 3))
    idx, keep = A.live_skinning(x.astype(np.float32), live.astype(np.float32), ref.astype(np.float32), 0.2)
    s, Fm = A.stretch(x, live, r, d, idx, keep, 0.025)
    dirs = rng.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    h = 1e-5
    for i in range(x.shape[0]):
        xp, _ = A.warp_back(x[i] + h * dirs, None, live, r, d, np.repeat(idx[i:i + 1], 400, 0),
                            np.repeat(keep[i:i + 1], 400, 0), 0.025)
        xm, _ = A.warp_back(x[i] - h * dirs, None, live, r, d, np.repeat(idx[i:i + 1], 400, 0),
                            np.repeat(keep[i:i + 1], 400, 0), 0.025)
        dd = np.linalg.norm(xp - xm, axis=1) / (2 * h)
        assert dd.max() <= s[i] * (1 + 2e-3)            # no direction stretches more
        assert dd.max() >= s[i] * (1 - 2e-2)            # and some direction nearly as much


def test_pipeline_candidates_weights_and_attributes():
    cam = Camera(width=24, height=18, fx=30.0, fy=30.0, cx=11.5, cy=8.5)
    ys, xs = np.mgrid[0:18, 0:24]
    depth = (1.0 + 0.01 * np.sin(xs / 3.0)).astype(np.float32)
    depth[2, 5] = 0.0                                     # a hole
    N32, ok = R32.normal_map(depth, cam, 0.03)
    V = R32.backproject(xs.ravel(), ys.ravel(), depth.ravel(), cam).astype(np.float64)
    rng = np.random.default_rng(3)
    ref = V[ok.ravel()][rng.choice(int(ok.sum()), 25, replace=False)]
    ref[0] += [0.0, 0.0, 0.3]                             # a node far behind the surface
    n = ref.shape[0]
    r, d = _tables(np.repeat(np.eye(3)[None], n, 0), np.zeros((n, 3)))
    match = np.full((18, 24), -1)
    match[::3, ::2] = 5                                   # fused pixels take no part
    ap = A.AppendParams(delta_nn=0.3)
    out = A.append_candidates(match, depth, N32, ok, cam, ref.astype(np.float32), ref.astype(np.float32), r, d, ap)
    cand = ok & (match < 0)
    assert np.array_equal(out["pixel"], np.flatnonzero(cand.ravel()))
    # weight sum by brute force
    Vc = V[out["pixel"]]
    S = np.array([sum(np.exp(-np.sum((Vc[i] - ref[j]) ** 2) / (2 * 0.025 ** 2))
                      for j, k in zip(out["idx"][i], out["keep"][i]) if k) for i in range(Vc.shape[0])])
    assert np.allclose(out["S"], S, rtol=1e-12)
    assert np.array_equal(out["near"], S >= 0.3) and 0 < out["near"].sum() < S.size
    # identity field: back at the depth vertex, no stretch, nothing compressive
    sel = out["near"]
    assert np.max(np.abs(out["v_ref"][sel] - Vc[sel])) < 1e-12
    assert np.max(np.abs(out["stretch"][sel] - 1.0)) < 1e-9 and not out["compressive"].any()
    assert np.array_equal(out["ok"], sel)
    ys_c, xs_c = np.divmod(out["pixel"], 24)
    assert np.allclose(out["radius"], F.depth_radius(depth.astype(np.float64), N32.astype(np.float64), cam)[ys_c, xs_c])
    assert np.allclose(out["conf"], F.depth_confidence(cam)[ys_c, xs_c])


def test_unstable_surfels_and_the_updated_array():
    conf = np.array([1.0, 12.0, 9.99, 10.0, 3.0, 50.0], np.float32)
    t_init = np.array([0, 0, 0, 0, 20, 0])
    gone = A.unstable(conf, t_init, 31, 10.0, 30)
    # below 10 and older than 30 frames: 0 and 2; 3 sits at the threshold, 4 is young
    assert gone.tolist() == [True, False, True, False, False, False]
    assert not A.unstable(conf, t_init, 30, 10.0, 30).any()        # exactly 30 frames: kept
    app = dict(ok=np.array([True, False, True]), v_ref=np.arange(9.0).reshape(3, 3),
               n_ref=-np.arange(9.0).reshape(3, 3), radius=np.array([0.1, 0.2, 0.3]), conf=np.array([0.5, 0.6, 0.7]))
    pos = np.arange(18.0).reshape(6, 3)
    out = A.update_surfels(pos, -pos, np.full(6, 0.01), conf, np.zeros(6, int), t_init, ~gone, app, 31)
    assert np.array_equal(out["pos"], np.concatenate([pos[[1, 3, 4, 5]], [[0, 1, 2], [6, 7, 8]]]))
    assert np.array_equal(out["nrm"][-2:], [[0, -1, -2], [-6, -7, -8]])
    assert out["radius"].tolist() == [0.01] * 4 + [0.1, 0.3]
    assert out["t_obs"].tolist() == [0, 0, 0, 0, 31, 31] and out["t_init"].tolist() == [0, 0, 20, 0, 31, 31]
    assert np.allclose(out["conf"], [12.0, 10.0, 3.0, 50.0, 0.5, 0.7])
