"""Pins of the index map and the correspondence gates (brute force)."""
import numpy as np

from gen.scenes import Camera
from oracle import replica32 as R32

CAM = Camera(16, 12, 14.0, 14.0, 7.5, 5.5)


def _brute_index_map(v, cam):
    v = v.astype(np.float32)
    best = {}
    for i, (x, y, z) in enumerate(v):
        if not z > 0:
            continue
        px = np.float32(cam.fx) * (x / z) + np.float32(cam.cx)
        py = np.float32(cam.fy) * (y / z) + np.float32(cam.cy)
        if not (np.isfinite(px) and np.isfinite(py)):
            continue
        ux = int(np.floor(px + np.float32(0.5)))
        uy = int(np.floor(py + np.float32(0.5)))
        if not (0 <= ux < cam.width and 0 <= uy < cam.height):
            continue
        key = (float(z), i)
        if (ux, uy) not in best or key < best[(ux, uy)]:
            best[(ux, uy)] = key
    I = -np.ones((cam.height, cam.width), dtype=np.int64)
    for (ux, uy), (_, i) in best.items():
        I[uy, ux] = i
    return I


def test_index_map_brute_force():
    rng = np.random.default_rng(3)
    n = 2000
    v = np.empty((n, 3), np.float32)
    v[:, 2] = rng.choice([0.8, 1.0, 1.2, -0.5], size=n)     # repeated z: exact ties
    v[:, 0] = rng.uniform(-0.8, 0.8, n) * v[:, 2]
    v[:, 1] = rng.uniform(-0.6, 0.6, n) * v[:, 2]
    v[5] = [0.0, 0.0, 0.0]
    v[6] = [np.nan, 0.0, 1.0]
    got = R32.index_map(v, CAM)
    assert np.array_equal(got, _brute_index_map(v, CAM))


def test_projection_rounds_half_up_at_pixel_boundary():
    # x/z chosen so that fx*(x/z)+cx lands exactly on k + 0.5
    cam = Camera(8, 8, 4.0, 4.0, 0.0, 0.0)
    v = np.array([[0.625, 0.375, 1.0]], np.float32)    # px = 2.5, py = 1.5
    ux, uy, ins = R32.project(v, cam)
    assert ins[0] and ux[0] == 3 and uy[0] == 2
    v = np.array([[-0.125, 0.0, 1.0]], np.float32)     # px = -0.5 -> pixel 0
    ux, uy, ins = R32.project(v, cam)
    assert ins[0] and ux[0] == 0
    v = np.array([[-0.1251, 0.0, 1.0]], np.float32)    # just outside
    _, _, ins = R32.project(v, cam)
    assert not ins[0]


def test_correspondence_gates_brute_force():
    rng = np.random.default_rng(4)
    cam = CAM
    depth = rng.uniform(0.9, 1.1, size=(cam.height, cam.width)).astype(np.float32)
    depth[4, 4] = 0
    N32, ok = R32.normal_map(depth, cam, 0.5)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    V = R32.backproject(xs, ys, depth, cam).reshape(-1, 3)
    n = V.shape[0]
    v = V + rng.normal(scale=0.02, size=V.shape).astype(np.float32)
    nv = N32.reshape(-1, 3) + rng.normal(scale=0.5, size=V.shape).astype(np.float32)
    I = R32.index_map(v, cam)
    m, ux, uy = R32.correspondence(v, nv, I, depth, N32, ok, cam, 0.03, 0.5)
    for i in range(n):
        _, _, ins = R32.project(v[i:i + 1], cam)
        exp = bool(ins[0]) and I[uy[i], ux[i]] == i and ok[uy[i], ux[i]]
        if exp:
            Vd = R32.backproject(np.array([ux[i]]), np.array([uy[i]]),
                                 np.array([depth[uy[i], ux[i]]]), cam)[0]
            dv = (v[i] - Vd).astype(np.float64)
            exp = (dv @ dv < 0.03 ** 2 * (1 + 1e-6)) and \
                float(nv[i].astype(np.float64) @ N32[uy[i], ux[i]]) > 0.5
            # decisions within FP32 rounding of the gates are not pinned here
            near = abs(dv @ dv - 0.03 ** 2) < 1e-7 or \
                abs(float(nv[i].astype(np.float64) @ N32[uy[i], ux[i]]) - 0.5) < 1e-6
            if near:
                continue
        assert bool(m[i]) == exp, i
