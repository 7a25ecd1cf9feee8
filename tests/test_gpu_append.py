"""Append candidates after fusion (Sec. 6.2 - 6.4) on the GPU, through the C
ABI, against the oracle fed the GPU's own fusion match map and live node
positions.

The candidate set and every nearest-node and ratio decision have exact FP32
forms on both sides; the weight-sum and stretch decisions are FP32 on the GPU
and FP64 in the oracle, so the survivor sets must agree except for candidates
whose oracle value lies within a stated margin of its threshold. Reference
positions and normals of common survivors are compared within FP32
tolerances."""
import numpy as np
import pytest

from gen.scenes import random_node_motion
from gpu_common import gpu_lib, stream_for
from oracle import append as A
from oracle import replica32 as R32
from oracle import solve as S
from oracle.quat import se3_to_rt

pytestmark = pytest.mark.gpu

S_MARGIN = 1e-4           # relative, weight sum vs delta_nn (FP32 exp and key vs FP64)
STRETCH_MARGIN = 2e-3     # absolute, largest singular value vs 1 + eps (FP32 central differences)


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _oracle(s, st, se3, match):
    live = st.live_nodes()
    R, t = se3_to_rt(np.asarray(se3, np.float64))
    r, d, _ = S.node_tables(s.node_pos.astype(np.float32).astype(np.float64), R, t)
    N32, ok = R32.normal_map(s.depth, s.cam, s.params.edge_gate)
    ap = A.AppendParams(sigma=s.params.node_sigma, eps=0.2, delta_nn=0.3)
    return A.append_candidates(match, s.depth, N32, ok, s.cam, live, s.node_pos.astype(np.float32), r, d, ap)


def _compare(got, ref):
    assert got["n_candidates"] == ref["pixel"].size
    amb = (np.abs(ref["S"] - 0.3) < S_MARGIN * 0.3) | (ref["near"] & (np.abs(ref["stretch"] - 1.2) < STRETCH_MARGIN))
    want = set(ref["pixel"][ref["ok"]].tolist())
    have = set(got["pixel"].tolist())
    loose = set(ref["pixel"][amb].tolist())
    assert (want ^ have) <= loose, sorted(want ^ have)[:10]
    assert got["n_appended"] == got["n_written"] == len(have)
    assert np.all(np.diff(got["pixel"]) > 0)                      # row-major order
    assert abs(got["n_far"] - int((~ref["near"]).sum())) <= int(amb.sum())
    assert abs(got["n_compressive"] - int(ref["compressive"].sum())) <= int(amb.sum())
    both = np.array(sorted(want & have), dtype=np.int64)
    gi = np.searchsorted(got["pixel"], both)
    ri = np.searchsorted(ref["pixel"], both)
    assert np.max(np.abs(got["pos"][gi] - ref["v_ref"][ri])) < 1e-5
    assert np.max(np.abs(got["nrm"][gi] - ref["n_ref"][ri])) < 2e-5
    assert np.allclose(got["radius"][gi], ref["radius"][ri], rtol=1e-5)
    assert np.allclose(got["confidence"][gi], ref["conf"][ri], rtol=1e-5)
    return int(amb.sum())


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_append_after_a_solve_matches_oracle(swgn, scene_cache, name):
    s = scene_cache(name)
    st = stream_for(swgn, s)
    st.solve_frame(s.depth)
    se3 = st.node_se3()
    st.fuse_frame(s.depth, t_now=4)
    match = st.last_fusion()[0]
    got = st.append_candidates()
    ref = _oracle(s, st, se3, match)
    st.close()
    amb = _compare(got, ref)
    assert got["n_appended"] > 0
    print(f"{name}: {got['n_candidates']} candidates, {got['n_appended']} appended, {amb} near a threshold")


def test_append_drops_far_and_compressive_candidates(swgn, scene_cache):
    """An unsmoothed random field (20 deg, 3 cm per node) splits nearest sets
    (Eq. 7), pulls nodes away from the surface and compresses it (Eq. 8)."""
    s = scene_cache("tiny")
    se3 = random_node_motion(s.node_pos, 20.0, 0.03, np.random.default_rng(0), smooth_steps=0).astype(np.float32)
    st = stream_for(swgn, s, se3=se3)
    se3_gpu = st.node_se3()
    st.fuse_frame(s.depth, t_now=1)
    match = st.last_fusion()[0]
    got = st.append_candidates()
    ref = _oracle(s, st, se3_gpu, match)
    st.close()
    assert (~ref["near"]).sum() > 50 and ref["compressive"].sum() > 50
    assert (~ref["keep"][:, 1:]).sum() > 100
    _compare(got, ref)
    assert got["n_far"] > 0 and got["n_compressive"] > 0


def test_append_capacity_and_state(swgn, scene_cache):
    s = scene_cache("tiny")
    st = stream_for(swgn, s)
    with pytest.raises(swgn.SwError):
        st.append_candidates()                                      # no fusion yet
    st.solve_frame(s.depth)
    st.fuse_frame(s.depth, t_now=1)
    full = st.append_candidates()
    few = st.append_candidates(max_out=5)
    assert few["n_appended"] == full["n_appended"] and few["n_written"] == 5
    assert np.array_equal(few["pixel"], full["pixel"][:5]) and np.array_equal(few["pos"], full["pos"][:5])
    st.solve_frame(s.depth)                                         # a new frame replaces the fused one
    with pytest.raises(swgn.SwError):
        st.append_candidates()
    st.close()


def test_appended_surfels_join_the_model(swgn, scene_cache):
    """The geometry update round trip: survivors appended to the surfels
    (t_observed = t_now), the node graph rebuilt at the current transforms;
    the next solve of the same depth finds at least as many correspondences."""
    s = scene_cache("tiny")
    half = np.arange(s.surfel_pos.shape[0]) % 2 == 0
    st = swgn.Stream(swgn.config_for(s, gn_iters=2))
    st.set_reference_surfels(s.surfel_pos[half], s.surfel_nrm[half])
    st.set_node_graph(s.node_pos)
    r0 = st.solve_frame(s.depth)
    se3 = st.node_se3()
    st.fuse_frame(s.depth, t_now=1)
    got = st.append_candidates()
    assert got["n_appended"] > 0
    pos, nrm = st.reference_surfels()
    rad, conf, tob = st.surfel_attributes()
    st.set_reference_surfels(np.concatenate([pos, got["pos"]]), np.concatenate([nrm, got["nrm"]]))
    st.set_surfel_attributes(np.concatenate([rad, got["radius"]]), np.concatenate([conf, got["confidence"]]),
                             np.concatenate([tob, np.full(got["n_written"], 1, np.int32)]))
    st.set_node_graph(s.node_pos, se3)
    assert st.sizes()[0] == pos.shape[0] + got["n_written"]
    r1 = st.solve_frame(s.depth)
    st.close()
    assert r1["n_corr"][0] >= r0["n_corr"][-1]
    assert np.isfinite(r1["e_data"]).all()


def test_geometry_update_removes_appends_and_reskins(swgn, scene_cache):
    """sw_update_geometry: the long-unstable surfels go, the append survivors
    of the same fusion follow the kept ones, the node state is untouched and
    the new surfels are skinned as a fresh set would be (bit-exact nearest
    nodes); the next solve runs on the updated model."""
    from oracle import skin
    s = scene_cache("tiny")
    ns = s.surfel_pos.shape[0]
    rng = np.random.default_rng(8)
    conf = rng.uniform(1.0, 20.0, ns).astype(np.float32)
    t_init = rng.integers(0, 40, ns).astype(np.int32)
    st = stream_for(swgn, s, fusion_dist=0.004)
    st.set_surfel_attributes(None, conf, None, t_init)
    st.solve_frame(s.depth)
    se3 = st.node_se3()
    st.fuse_frame(s.depth, t_now=45)
    pos0, nrm0 = st.reference_surfels()
    rad0, conf0, tob0, ti0 = st.surfel_attributes(with_t_init=True)
    app = st.append_candidates()
    g = st.update_geometry()
    keep = ~A.unstable(conf0, ti0, 45, 10.0, 30)
    assert g["n_removed"] == int((~keep).sum()) > 0
    assert g["append"]["n_appended"] == app["n_appended"] > 0
    assert g["n_surfels"] == int(keep.sum()) + app["n_appended"] == st.sizes()[0]
    pos1, nrm1 = st.reference_surfels()
    rad1, conf1, tob1, ti1 = st.surfel_attributes(with_t_init=True)
    na = app["n_appended"]
    assert np.array_equal(pos1, np.concatenate([pos0[keep], app["pos"]]))
    assert np.array_equal(nrm1, np.concatenate([nrm0[keep], app["nrm"]]))
    assert np.array_equal(rad1, np.concatenate([rad0[keep], app["radius"]]))
    assert np.array_equal(conf1, np.concatenate([conf0[keep], app["confidence"]]))
    assert np.array_equal(tob1, np.concatenate([tob0[keep], np.full(na, 45, np.int32)]))
    assert np.array_equal(ti1, np.concatenate([ti0[keep], np.full(na, 45, np.int32)]))
    assert np.array_equal(st.node_se3(), se3)
    idx, _ = st.skinning()
    assert np.array_equal(idx, skin.knn_fp32(pos1, s.node_pos, 4))
    with pytest.raises(swgn.SwError):
        st.update_geometry()                                        # the fused frame is spent
    r = st.solve_frame(s.depth)
    st.close()
    assert r["n_corr"][0] > 0 and np.isfinite(r["e_data"]).all()


def test_empty_frame_fuses_nothing_and_an_update_that_would_empty_the_model_is_refused(swgn, scene_cache):
    """A depth frame without measurements: no pixel has a normal, so nothing
    fuses and nothing is a candidate. With every surfel unstable and old, an
    update would leave no surfel: it is refused and the model stays usable."""
    s = scene_cache("tiny")
    ns = s.surfel_pos.shape[0]
    st = stream_for(swgn, s)
    st.set_surfel_attributes(None, np.full(ns, 1.0, np.float32), None, np.zeros(ns, np.int32))
    pos0, _ = st.reference_surfels()
    empty = np.zeros_like(s.depth)
    f = st.fuse_frame(empty, t_now=100)
    assert f == {"n_fused": 0, "n_candidates": 0}
    match = st.last_fusion()[0]
    assert np.all(match == -1)
    a = st.append_candidates()
    assert a["n_candidates"] == a["n_appended"] == 0 and a["pixel"].size == 0
    assert np.array_equal(st.reference_surfels()[0], pos0)
    with pytest.raises(swgn.SwError):
        st.update_geometry()                                        # would remove all surfels, append none
    assert st.sizes()[0] == ns
    r = st.solve_frame(s.depth)
    st.close()
    assert r["n_corr"][0] > 0
