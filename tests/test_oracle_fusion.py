"""Pins of the fusion oracle (Sec. 5 depth-surfel attributes, Sec. 6.1 fusion,
Sec. 6.4 return to the reference frame) against closed forms and brute force."""
import numpy as np
from scipy.spatial.transform import Rotation

from gen.scenes import Camera
from oracle import fusion as F
from oracle import replica32 as R32
from oracle import warp
from oracle.quat import qmul


def _cam(W=16, H=12, f=20.0):
    return Camera(width=W, height=H, fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)


def test_depth_confidence_closed_form():
    cam = _cam()
    c = F.depth_confidence(cam)
    # at the principal point (between pixels here) the largest; 1 at its distance 0
    cam2 = Camera(width=17, height=13, fx=20.0, fy=20.0, cx=8.0, cy=6.0)
    c2 = F.depth_confidence(cam2)
    assert c2[6, 8] == 1.0
    assert np.isclose(c2[0, 0], np.exp(-1.0 / (2 * 0.6 ** 2)), rtol=1e-15)
    assert np.allclose(c, c[::-1, ::-1])          # symmetric about the centre
    assert np.all((c > 0) & (c <= 1))


def test_depth_radius_closed_form_and_clamp():
    cam = _cam()
    d = np.full((cam.height, cam.width), 1.5)
    for deg, expect_deg in ((0.0, 0.0), (60.0, 60.0), (80.0, 75.0), (89.0, 75.0)):
        a = np.deg2rad(deg)
        N = np.broadcast_to(np.array([np.sin(a), 0.0, -np.cos(a)]), d.shape + (3,))
        r = F.depth_radius(d, N, cam)
        want = np.sqrt(2.0) * 1.5 / (cam.fx * np.cos(np.deg2rad(expect_deg)))
        assert np.allclose(r, want, rtol=1e-14), deg


def test_subpixel_lies_in_its_depth_pixel():
    cam = _cam()
    rng = np.random.default_rng(0)
    v = np.stack([rng.uniform(-0.6, 0.6, 4000), rng.uniform(-0.45, 0.45, 4000), rng.uniform(0.8, 1.2, 4000)], 1)
    v32 = v.astype(np.float32)
    sx, sy, ins = F.subpixel(v32, cam)
    ux, uy, ins2 = R32.project(v32, cam)
    assert np.array_equal(ins, ins2)
    assert np.array_equal(sx[ins] // 4, ux[ins]) and np.array_equal(sy[ins] // 4, uy[ins])


def test_index_map_4x_is_the_per_subpixel_minimum():
    cam = _cam(8, 6, 10.0)
    rng = np.random.default_rng(1)
    n = 900
    v = np.stack([rng.uniform(-0.45, 0.45, n), rng.uniform(-0.3, 0.3, n), rng.uniform(0.9, 1.1, n)], 1)
    v32 = v.astype(np.float32)
    v32[4] = (0.01, 0.01, 0.5)            # nearest in its sub-pixel ...
    v32[5] = v32[4]                       # ... and an exact tie: the lower index wins
    valid = rng.random(n) > 0.1
    valid[4] = valid[5] = True
    I4 = F.index_map_4x(v32, cam, valid)
    sx, sy, ins = F.subpixel(v32, cam)
    want = np.full(I4.shape, -1)
    for i in range(n):                    # brute force in index order
        if not (ins[i] and valid[i]):
            continue
        j = want[sy[i], sx[i]]
        if j < 0 or (v32[i, 2], i) < (v32[j, 2], j):
            want[sy[i], sx[i]] = i
    assert np.array_equal(I4, want)
    assert I4[sy[4], sx[4]] == 4


def _brute_match(I4, v32, n32, conf, depth, N32, nvalid, cam, fp):
    H, W = cam.height, cam.width
    out = np.full((H, W), -1)
    f = np.float32
    for y in range(H):
        for x in range(W):
            if not nvalid[y, x]:
                continue
            d = f(depth[y, x])
            V = np.array([((f(x) - f(cam.cx)) / f(cam.fx)) * d, ((f(y) - f(cam.cy)) / f(cam.fy)) * d, d], f)
            best = None
            for s in I4[4 * y:4 * y + 4, 4 * x:4 * x + 4].ravel():
                if s < 0:
                    continue
                dv = v32[s] - V
                d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]
                dot = (n32[s, 0] * N32[y, x, 0] + n32[s, 1] * N32[y, x, 1]) + n32[s, 2] * N32[y, x, 2]
                if d2 <= f(fp.delta_distance) * f(fp.delta_distance) and dot >= f(fp.delta_normal):
                    key = (-conf[s], d2, s)
                    if best is None or key < best[0]:
                        best = (key, s)
            if best is not None:
                out[y, x] = best[1]
    return out


def test_match_selects_by_confidence_then_distance_then_index():
    cam = _cam(8, 6, 10.0)
    rng = np.random.default_rng(2)
    H, W = cam.height, cam.width
    depth = rng.uniform(0.95, 1.05, (H, W))
    depth[0, 0] = 0.0
    N32 = np.zeros((H, W, 3), np.float32)
    N32[..., 2] = -1.0
    nvalid = depth > 0
    nvalid[1, 1] = False
    ys, xs = np.mgrid[0:H, 0:W]
    Vd = np.stack([(xs - cam.cx) / cam.fx * depth, (ys - cam.cy) / cam.fy * depth, depth], -1)
    # 6 surfels near each pixel's depth vertex, spread over its sub-pixels
    n_per = 6
    base = np.repeat(Vd.reshape(-1, 3), n_per, axis=0)
    v = base + rng.normal(0, 4e-4, base.shape)
    v32 = v.astype(np.float32)
    n = np.tile(np.array([0, 0, -1.0]), (v.shape[0], 1)) + rng.normal(0, 0.3, (v.shape[0], 3))
    n32 = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    conf = rng.integers(1, 4, v.shape[0]).astype(np.float32)     # many equal confidences
    # constructed ties: two surfels at one point, equal confidence -> lower index
    v32[11] = v32[10]
    n32[11] = n32[10]
    conf[10] = conf[11] = 9.0
    fp = F.FusionParams()
    I4 = F.index_map_4x(v32, cam, np.ones(v.shape[0], bool))
    got = F.match(I4, v32, n32, conf, depth, N32, nvalid, cam, fp)
    want = _brute_match(I4, v32, n32, conf, depth, N32, nvalid, cam, fp)
    assert np.array_equal(got, want)
    assert got[0, 0] == -1 and got[1, 1] == -1
    assert np.count_nonzero(got >= 0) > 10
    chosen = got[got >= 0]
    assert np.unique(chosen).size == chosen.size


def test_fuse_weights_and_renormalised_normal():
    best = np.array([[1, -1], [-1, 0]])
    v = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 1.0], [2.0, 0.0, 1.0]])
    n = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    r = np.array([1.0, 2.0, 3.0])
    c = np.array([1.0, 3.0, 5.0])
    t = np.array([0, 0, 0])
    Vd = np.zeros((2, 2, 3))
    Vd[0, 0] = [3.0, 0.0, 1.0]
    Vd[1, 1] = [1.0, 1.0, 1.0]
    Nd = np.zeros((2, 2, 3))
    Nd[0, 0] = [0.0, 1.0, 0.0]
    Nd[1, 1] = [0.0, 0.0, -1.0]
    rd = np.array([[4.0, 0.0], [0.0, 1.0]])
    cd = np.array([[1.0, 0.0], [0.0, 1.0]])
    out = F.fuse(best, v, n, r, c, t, Vd, Nd, rd, cd, t_now=7)
    # surfel 1 (c 3) with the depth surfel at (0,0) (c 1)
    assert np.allclose(out["v"][1], [(3 * 1.0 + 3.0) / 4, 0.0, 1.0])
    assert np.allclose(out["n"][1], np.array([3.0, 1.0, 0.0]) / np.sqrt(10.0))
    assert out["r"][1] == (3 * 2.0 + 4.0) / 4 and out["c"][1] == 4.0 and out["t"][1] == 7
    # surfel 0 (c 1) with (1,1) (c 1): midpoints
    assert np.allclose(out["v"][0], [0.5, 0.5, 1.0]) and np.allclose(out["n"][0], [0, 0, -1])
    # surfel 2 untouched
    assert np.array_equal(out["v"][2], v[2]) and out["c"][2] == 5.0 and out["t"][2] == 0
    assert out["fused"].tolist() == [True, True, False]


def test_to_reference_inverts_the_blend():
    rng = np.random.default_rng(3)
    n_nodes, ns = 12, 500
    R = Rotation.from_rotvec(rng.normal(0, 0.2, (n_nodes, 3)))
    q = R.as_quat()[:, [3, 0, 1, 2]]
    q *= np.sign(q[:, :1])
    t = rng.normal(0, 0.05, (n_nodes, 3))
    d = 0.5 * qmul(np.concatenate([np.zeros((n_nodes, 1)), t], 1), q)
    idx = np.stack([rng.choice(n_nodes, 4, replace=False) for _ in range(ns)])
    w = rng.random((ns, 4))
    w /= w.sum(1, keepdims=True)
    b, _ = warp.blend(idx, w, q, d)
    v = rng.normal(0, 0.3, (ns, 3))
    nrm = rng.normal(0, 1, (ns, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    vl, nl, ok = warp.apply_blend(b, v, nrm)
    assert ok.all()
    vr, nr = F.to_reference(b, vl, nl)
    assert np.max(np.abs(vr - v)) < 1e-13 and np.max(np.abs(nr - nrm)) < 1e-13
    # one node: the closed form R^T (v' - t)
    b1, _ = warp.blend(np.zeros((1, 1), int), np.ones((1, 1)), q[:1], d[:1])
    vr1, _ = F.to_reference(b1, vl[:1], nl[:1])
    assert np.allclose(vr1[0], R[0].inv().apply(vl[0] - t[0]), atol=1e-13)
