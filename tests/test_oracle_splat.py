"""Pins of the splat rendering and its pixel-driven pairs (Sec. 7: the live
surfels as opaque discs): reduction to the point rule at radius 0, the disc
coverage and occlusion by brute force, ties, the box cap, and the system of a
splat association against finite differences of its stacked residual."""
import numpy as np

from gen.scenes import Camera
from oracle import quat as Q
from oracle import replica32 as R32
from oracle import solve as S
from oracle.terms import arap_residuals


def _cam(W=24, H=18, f=100.0):
    return Camera(width=W, height=H, fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)


def _coverage64(v, n, r, cam, ux, uy):
    d = np.array([(ux - cam.cx) / cam.fx, (uy - cam.cy) / cam.fy, 1.0])
    nd = n @ d
    if nd == 0:
        return False, np.inf
    t = (n @ v) / nd
    return bool(t > 0 and np.sum((t * d - v) ** 2) <= r * r), t


def test_radius_zero_is_the_point_rule(scene_cache):
    s = scene_cache("tiny")
    v, n = s.surfel_pos.astype(np.float32), s.surfel_nrm.astype(np.float32)
    zero = np.zeros(v.shape[0], np.float32)
    I_s = R32.splat_index_map(v, n, zero, s.cam)
    assert np.array_equal(I_s, R32.index_map(v, s.cam))
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    k, ux, uy = R32.splat_pairs(v, n, I_s, s.depth, N32, ok, s.cam, s.params.corr_dist, s.params.corr_normal)
    m, px, py = R32.correspondence(v, n, I_s, s.depth, N32, ok, s.cam, s.params.corr_dist, s.params.corr_normal)
    got = np.full(I_s.shape, -1)
    got[uy, ux] = k
    want = np.full(I_s.shape, -1)
    want[py[m], px[m]] = np.flatnonzero(m)
    assert np.array_equal(got, want)


def test_disc_coverage_and_occlusion_by_brute_force():
    cam = _cam()
    rng = np.random.default_rng(4)
    ns = 60
    v = np.stack([rng.uniform(-0.08, 0.08, ns), rng.uniform(-0.06, 0.06, ns), rng.uniform(0.9, 1.1, ns)], 1)
    n = np.stack([rng.normal(0, 0.3, ns), rng.normal(0, 0.3, ns), -np.ones(ns)], 1)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    r = rng.uniform(0.004, 0.03, ns)
    v32, n32, r32 = v.astype(np.float32), n.astype(np.float32), r.astype(np.float32)
    I = R32.splat_index_map(v32, n32, r32, cam)
    ux0, uy0, inside = R32.project(v32, cam)
    near_tie = 0
    for y in range(cam.height):
        for x in range(cam.width):
            cands = []
            for i in range(ns):
                if not inside[i]:
                    continue
                h = min(4, int(np.ceil(cam.fx * r[i] / v[i, 2])))
                if abs(x - ux0[i]) > h or abs(y - uy0[i]) > h:
                    continue
                d = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
                t = (n[i] @ v[i]) / (n[i] @ d)
                e2 = np.sum((t * d - v[i]) ** 2)
                if abs(e2 - r[i] ** 2) < 1e-6 * r[i] ** 2:
                    near_tie += 1
                    break
                if t > 0 and e2 <= r[i] ** 2:
                    cands.append((t, i))
            else:
                want = min(cands)[1] if cands else -1
                if len(cands) > 1:
                    ts = sorted(c[0] for c in cands)
                    if ts[1] - ts[0] < 1e-6:
                        continue                        # depth near-tie: FP32 may order them either way
                assert I[y, x] == want, (x, y, I[y, x], want)
    assert near_tie < 10
    assert np.count_nonzero(I >= 0) > 100                # discs cover many pixels
    assert np.unique(I[I >= 0]).size > 20


def test_equal_discs_tie_to_the_lower_index_and_the_box_is_capped():
    cam = _cam()
    v = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.02, 0.0, 0.5]], np.float32)
    n = np.array([[0, 0, -1], [0, 0, -1], [0, 0, -1]], np.float32)
    r = np.array([0.02, 0.02, 0.5], np.float32)          # the third: 100 px radius, capped to a 9 x 9 box
    I = R32.splat_index_map(v[:2], n[:2], r[:2], cam)
    assert np.all(I[I >= 0] == 0) and np.count_nonzero(I == 0) > 4
    I3 = R32.splat_index_map(v, n, r, cam)
    ux, uy, _ = R32.project(v[2:], cam)
    assert np.count_nonzero(I3 == 2) == 81
    ys, xs = np.nonzero(I3 == 2)
    assert xs.min() == ux[0] - 4 and xs.max() == ux[0] + 4 and ys.min() == uy[0] - 4 and ys.max() == uy[0] + 4


def _frozen_pairs(pb, lin, R, t):
    ws = S.warp_surfels(pb, R, t)
    k, ux, uy = lin["corr_idx"], lin["pair_ux"], lin["pair_uy"]
    rd = np.sum(pb.N64[uy, ux] * (ws["v"][k] - pb.V64[uy, ux]), axis=1)
    ra = arap_residuals(pb.node_pos, R, t, pb.nbr).reshape(-1)
    return np.concatenate([rd, np.sqrt(pb.lambda_reg) * ra])


def test_splat_system_matches_fd_jacobian_with_several_pairs_per_surfel(scene_cache):
    s = scene_cache("tiny")
    from oracle import fusion as F
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    # radii of depth surfels at the reference (about 1.4 px): discs overlap
    ux, uy, inside = R32.project(s.surfel_pos.astype(np.float32), s.cam)
    rad = np.sqrt(2.0) * s.surfel_pos[:, 2] / (s.cam.fx * np.maximum(np.abs(s.surfel_nrm[:, 2]), np.cos(np.deg2rad(75))))
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params,
                        splat_radius=rad.astype(np.float32))
    R, t = Q.se3_to_rt(s.gt_se3)
    lin = S.linearize(pb, R, t)
    k = lin["corr_idx"]
    counts = np.bincount(k, minlength=pb.surfel_pos.shape[0])
    assert counts.max() >= 2 and (counts >= 2).sum() > 20           # surfels with several pairs
    assert np.unique(lin["pair_uy"] * s.cam.width + lin["pair_ux"]).size == k.size   # a pixel pairs once
    A, g = S.normal_equations(pb, lin)
    nn = pb.node_pos.shape[0]
    h = 1e-6

    def moved(kk, e):
        R2, t2 = R.copy(), t.copy()
        c = R[kk] @ pb.node_pos[kk].astype(np.float64) + t[kk]
        E = Q.exp_so3(e[:3][None])[0]
        R2[kk] = E @ R[kk]
        t2[kk] = E @ (t[kk] - c) + c + e[3:]
        return R2, t2

    r0 = _frozen_pairs(pb, lin, R, t)
    Jfd = np.zeros((r0.size, 6 * nn))
    for kk in range(nn):
        for c in range(6):
            e = np.zeros(6)
            e[c] = h
            Jfd[:, 6 * kk + c] = (_frozen_pairs(pb, lin, *moved(kk, e)) - _frozen_pairs(pb, lin, *moved(kk, -e))) / (2 * h)
    Hfd = Jfd.T @ Jfd + pb.damping * np.eye(6 * nn)
    Ad = A.toarray()
    assert np.linalg.norm(Ad - Hfd) <= 1e-6 * np.linalg.norm(Hfd)
    assert np.linalg.norm(g - Jfd.T @ r0) <= 1e-6 * np.linalg.norm(g)
    assert np.isclose(r0 @ r0, lin["e_data"] + pb.lambda_reg * lin["e_reg"], rtol=1e-12)
    # the pairs of the point rule are a subset size-wise: discs add pairs
    lin_pt = S.linearize(S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params), R, t)
    assert k.size > lin_pt["corr_idx"].size
