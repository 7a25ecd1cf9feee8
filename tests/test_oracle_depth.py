"""Pins of the depth-map step: vertex map, normal map and its validity."""
import numpy as np

from gen.scenes import Camera, Sphere, ray_cast
from oracle import depth as D64
from oracle import replica32 as R32

CAM = Camera(64, 48, 60.0, 62.0, 31.5, 23.0)


def test_vertex_map_closed_form():
    rng = np.random.default_rng(0)
    d = rng.uniform(0.5, 2.0, size=(CAM.height, CAM.width)).astype(np.float32)
    V = D64.vertex_map(d, CAM)
    y, x = 17, 40
    dd = float(d[y, x])
    assert np.allclose(V[y, x], [(x - CAM.cx) * dd / CAM.fx, (y - CAM.cy) * dd / CAM.fy, dd], rtol=1e-15)
    V32 = R32.backproject(np.array([x]), np.array([y]), np.array([d[y, x]]), CAM)
    assert np.allclose(V32[0], V[y, x], rtol=1e-6)


def test_fronto_parallel_plane_normal_is_exact():
    d = np.full((CAM.height, CAM.width), 1.3, dtype=np.float32)
    N32, ok = R32.normal_map(d, CAM, 0.03)
    assert ok[1:-1, 1:-1].all() and not ok[0].any() and not ok[:, -1].any()
    assert np.array_equal(N32[ok], np.tile(np.float32([0, 0, -1]), (ok.sum(), 1)))
    N64 = D64.normal_map(d, CAM)
    assert np.allclose(N64[ok], [0, 0, -1], atol=0)


def test_tilted_plane_normal():
    # plane n.x = c with unit normal n facing the camera
    n = np.array([0.3, -0.2, -1.0])
    n /= np.linalg.norm(n)
    c = -1.0
    ys, xs = np.mgrid[0:CAM.height, 0:CAM.width].astype(np.float64)
    ray = np.stack([(xs - CAM.cx) / CAM.fx, (ys - CAM.cy) / CAM.fy, np.ones_like(xs)], -1)
    z = c / (ray @ n)
    d = z.astype(np.float32)
    N64 = D64.normal_map(d, CAM)
    N32, ok = R32.normal_map(d, CAM, 1.0)
    assert ok[1:-1, 1:-1].all()
    assert np.allclose(N64[ok], n, atol=1e-5)      # FP32 depth rounding only
    assert np.allclose(N32[ok], n, atol=1e-4)


def test_sphere_normal_converges_to_radial():
    errs = []
    for scale in (1, 2, 4):
        cam = Camera(64 * scale, 48 * scale, 60.0 * scale, 60.0 * scale, 32.0 * scale, 24.0 * scale)
        ys, xs = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
        sph = Sphere((0.0, 0.0, 1.5), 0.6)
        t, p, nrm, pid = ray_cast(cam, [sph], xs, ys)
        d = np.where(np.isfinite(t), t, 0).astype(np.float64)
        N = D64.normal_map(d, cam)
        ok = np.zeros_like(pid, dtype=bool)
        ok[1:-1, 1:-1] = (pid[1:-1, 1:-1] == 0) & (pid[2:, 1:-1] == 0) & (pid[:-2, 1:-1] == 0) \
            & (pid[1:-1, 2:] == 0) & (pid[1:-1, :-2] == 0)
        # stay away from the grazing rim
        with np.errstate(invalid="ignore"):
            ok &= np.einsum("...i,...i->...", nrm, -p / np.linalg.norm(p, axis=-1, keepdims=True)) > 0.5
        errs.append(np.max(np.linalg.norm(N[ok] - nrm[ok], axis=-1)))
    assert errs[0] < 5e-3
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3     # second order


def _validity_brute(d, gate):
    H, W = d.shape
    ok = np.zeros((H, W), bool)
    for y in range(1, H - 1):
        for x in range(1, W - 1):
            vals = [d[y, x], d[y - 1, x], d[y + 1, x], d[y, x - 1], d[y, x + 1]]
            if not all(np.isfinite(v) and v > 0 for v in vals):
                continue
            if any(abs(np.float32(v) - np.float32(d[y, x])) > np.float32(gate) for v in vals[1:]):
                continue
            ok[y, x] = True
    return ok


def test_normal_validity_rule_brute_force():
    rng = np.random.default_rng(5)
    d = rng.uniform(1.0, 1.02, size=(12, 14)).astype(np.float32)
    d[3, 4] = 0.0
    d[6, 6] = np.nan
    d[8, 2] = np.inf
    d[2, 10] = -1.0
    d[9, 9] = 1.5            # depth jump
    d[5, 11] = 1.0 + 0.03    # right at the gate
    _, ok = R32.normal_map(d, CAM, 0.03)
    assert np.array_equal(ok, _validity_brute(d, 0.03))


def test_replica_normals_match_fp64(scene_cache):
    s = scene_cache("c1")
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    N64 = D64.normal_map(s.depth, s.cam)
    assert ok.sum() > 0.8 * (s.depth > 0).sum()
    err = np.linalg.norm(N32[ok].astype(np.float64) - N64[ok], axis=1)
    assert err.max() < 1e-4
    # normals face the camera
    V = D64.vertex_map(s.depth, s.cam)
    assert np.all(np.sum(N64[ok] * V[ok], axis=1) <= 0)
