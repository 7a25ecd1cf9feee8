"""Depth-map fusion (Sec. 5, Sec. 6.1, Sec. 6.4) and the solver's visibility
filter (Sec. 7) on the GPU, through the C ABI, against the oracle.

The integer outputs (the solver's index and correspondence maps with the
filter, the fusion match map) are compared bit for bit with the FP32
decisions of the oracle, fed the GPU's own live surfels where the live
positions come from a non-identity warp. Fused attributes and the updated
reference surfels are compared within FP32 tolerances."""
import numpy as np
import pytest

from gpu_common import gpu_lib, stream_for
from oracle import fusion as F
from oracle import replica32 as R32
from oracle import solve as S
from oracle import warp
from oracle.quat import se3_to_rt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _attributes(ns, seed):
    rng = np.random.default_rng(seed)
    conf = rng.uniform(0.5, 20.0, ns).astype(np.float32)
    conf[::7] = 10.0                        # at the stable threshold exactly: not stable
    rad = rng.uniform(0.001, 0.004, ns).astype(np.float32)
    tob = rng.integers(0, 10, ns).astype(np.int32)
    return rad, conf, tob


@pytest.mark.parametrize("name,recent", [("c1", 2), ("c2", 2), ("c1", -1)])
def test_visibility_filter_maps_bit_exact(swgn, scene_cache, name, recent):
    s = scene_cache(name)
    ns = s.surfel_pos.shape[0]
    rad, conf, tob = _attributes(ns, 5)
    st = stream_for(swgn, s, debug_iter=0, gn_iters=1, visibility=1, stable_conf=10.0, recent_frames=recent)
    st.set_surfel_attributes(rad, conf, tob)
    st.set_frame_time(9)
    st.solve_frame(s.depth)
    I, Cm, live, N = st.last_maps()
    st.close()
    vis = S.visible_surfels(conf, tob, 9, 10.0, recent)
    assert 0 < vis.sum() < ns
    I_ref = R32.index_map(s.surfel_pos, s.cam, vis)     # identity state: live = reference exactly
    assert np.array_equal(I, I_ref)
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    m, ux, uy = R32.correspondence(s.surfel_pos, s.surfel_nrm, I_ref, s.depth, N32, ok, s.cam,
                                   s.params.corr_dist, s.params.corr_normal, vis)
    C_ref = np.full(I.shape, -1, np.int64)
    C_ref[uy[m], ux[m]] = np.flatnonzero(m)
    assert np.array_equal(Cm, C_ref)
    assert not np.isin(Cm, np.flatnonzero(~vis)).any()


def _fusion_reference(s, se3, live_pos, live_nrm, rad, conf, tob, t_now, fp):
    """The oracle's fusion on the GPU's live surfels (FP32 decisions), then the
    fused surfels back to the reference frame at the GPU's node state."""
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    valid = np.isfinite(live_pos[:, 0])
    I4 = F.index_map_4x(live_pos, s.cam, valid)
    best = F.match(I4, live_pos, live_nrm, conf, s.depth, N32, ok, s.cam, fp)
    ys, xs = np.mgrid[0:s.cam.height, 0:s.cam.width]
    Vd = R32.backproject(xs, ys, s.depth, s.cam).astype(np.float64)
    N64 = N32.astype(np.float64)
    cd = F.depth_confidence(s.cam)
    rd = F.depth_radius(s.depth.astype(np.float64), N64, s.cam)
    out = F.fuse(best, live_pos, live_nrm, rad, conf, tob, Vd, N64, rd, cd, t_now)
    pb = S.make_problem(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, s.params)
    R, t = se3_to_rt(np.asarray(se3, np.float64))
    r, d, _ = S.node_tables(pb.node_pos, R, t)
    b, _ = warp.blend(pb.idx, pb.w, r, d)
    f = out["fused"]
    vr, nr = F.to_reference(b[f], out["v"][f], out["n"][f])
    return best, ok, out, f, vr, nr


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_fusion_matches_oracle_after_a_solve(swgn, scene_cache, name):
    s = scene_cache(name)
    ns = s.surfel_pos.shape[0]
    rad, conf, tob = _attributes(ns, 6)
    st = stream_for(swgn, s, fusion_dist=0.004)      # 1 mm is Table 1's; wider here for more pairs
    st.set_surfel_attributes(rad, conf, tob)
    st.solve_frame(s.depth)
    se3 = st.node_se3()
    stats = st.fuse_frame(s.depth, t_now=12)
    match, live_pos, live_nrm = st.last_fusion()
    rad1, conf1, tob1 = st.surfel_attributes()
    pos1, nrm1 = st.reference_surfels()
    st.close()
    fp = F.FusionParams(delta_distance=0.004)
    best, ok, out, f, vr, nr = _fusion_reference(s, se3, live_pos, live_nrm, rad, conf, tob, 12, fp)
    assert np.array_equal(match, best)
    assert stats["n_fused"] == int(f.sum()) > 0
    assert stats["n_candidates"] == int(np.count_nonzero(ok & (best < 0)))
    # fused attributes (FP32 arithmetic against FP64)
    assert np.array_equal(tob1[f], np.full(f.sum(), 12)) and np.array_equal(tob1[~f], tob[~f])
    assert np.allclose(conf1[f], out["c"][f], rtol=2e-6)
    assert np.allclose(rad1[f], out["r"][f], rtol=2e-5)
    assert np.array_equal(conf1[~f], conf[~f]) and np.array_equal(rad1[~f], rad[~f])
    # fused surfels back in the reference frame; the others untouched
    assert np.max(np.abs(pos1[f] - vr)) < 2e-6
    assert np.max(np.abs(nrm1[f] - nr)) < 2e-5
    assert np.array_equal(pos1[~f], s.surfel_pos[~f].astype(np.float32))
    assert np.array_equal(nrm1[~f], s.surfel_nrm[~f].astype(np.float32))


def test_fusion_of_the_identical_frame():
    """Surfels cast from the depth itself at the identity warp: every pixel with
    a normal holds its own surfel at distance 0 and fuses into it; positions
    and normals stay where they are, confidence grows by the depth surfel's."""
    swgn = gpu_lib()
    from test_oracle_solve import exact_identity_problem
    cam, d, pos, nrm, nodes, params = exact_identity_problem()
    cfg = swgn.sw_config_default(width=cam.width, height=cam.height, fx=cam.fx, fy=cam.fy, cx=cam.cx,
                                 cy=cam.cy, gn_iters=1, pcg_iters=4, lambda_reg=params.lambda_reg,
                                 node_sigma=params.node_sigma, corr_dist=params.corr_dist,
                                 corr_normal=params.corr_normal, edge_gate=params.edge_gate,
                                 damping=params.damping)
    st = swgn.Stream(cfg)
    st.set_reference_surfels(pos, nrm)
    st.set_node_graph(nodes)
    stats = st.fuse_frame(d, t_now=3)
    match, live_pos, _ = st.last_fusion()
    rad1, conf1, tob1 = st.surfel_attributes()
    pos1, nrm1 = st.reference_surfels()
    st.close()
    N32, ok = R32.normal_map(d, cam, params.edge_gate)
    yy, xx = np.nonzero(ok)
    want = np.full(match.shape, -1)
    want[yy, xx] = np.arange(pos.shape[0])
    assert np.array_equal(live_pos, pos)
    assert np.array_equal(match, want)
    assert stats["n_fused"] == pos.shape[0] and stats["n_candidates"] == 0
    cd = F.depth_confidence(cam)[yy, xx]
    assert np.allclose(conf1, 1.0 + cd, rtol=1e-6) and np.all(tob1 == 3)
    assert np.max(np.abs(pos1 - pos)) < 1e-6 and np.max(np.abs(nrm1 - nrm)) < 1e-6
    rd = F.depth_radius(d.astype(np.float64), N32.astype(np.float64), cam)[yy, xx]
    assert np.allclose(rad1, cd * rd / (1.0 + cd), rtol=1e-5)


def test_solve_after_fusion_uses_the_updated_surfels(swgn, scene_cache):
    s = scene_cache("tiny")
    st = stream_for(swgn, s, fusion_dist=0.004)
    st.solve_frame(s.depth)
    before = st.reference_surfels()[0]
    stats = st.fuse_frame(s.depth, t_now=1)
    after = st.reference_surfels()[0]
    assert stats["n_fused"] > 0 and not np.array_equal(before, after)
    res = st.solve_frame(s.depth)
    st.close()
    assert all(np.isfinite(res["e_data"])) and res["n_corr"][-1] > 0
