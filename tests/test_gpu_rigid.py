"""Rigid alignment before the non-rigid steps on the GPU: against the FP64
oracle (same readings), exact recovery of a rigidly moved surface, and the
same result alone and in a batch."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from gen.scenes import SolverParams
from gpu_common import gpu_lib, se3_errors, stream_for
from oracle import solve as S
from test_oracle_solve import _rigid_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_rigid_then_nonrigid_matches_the_oracle(swgn, scene_cache, name):
    s = scene_cache(name)
    params = SolverParams(**{**s.params.__dict__, "rigid_iters": 3})
    st = stream_for(swgn, s, rigid_iters=3)
    stats = st.solve_frame(s.depth)
    got = st.node_se3()
    st.close()
    want, tr = S.oracle_solve(s.cam, s.surfel_pos, s.surfel_nrm, s.node_pos, s.depth, params, linear="pcg")
    ang, dpos = se3_errors(got, want, s.node_pos)
    assert ang.max() < 1e-4 and dpos.max() < 1e-5, (ang.max(), dpos.max())
    assert np.allclose(stats["rigid_e"], tr["rigid"]["e"], rtol=1e-4)
    assert np.all(np.abs(np.array(stats["rigid_n"]) - np.array(tr["rigid"]["n_corr"])) <= 2)


def test_rigid_alignment_recovers_a_rigid_motion(swgn):
    cam, pos, nrm, nodes, depth, params, Rs, ts = _rigid_scene()
    cfg = swgn.sw_config_default(width=cam.width, height=cam.height, fx=cam.fx, fy=cam.fy, cx=cam.cx,
                                 cy=cam.cy, gn_iters=0, pcg_iters=10, lambda_reg=params.lambda_reg,
                                 node_sigma=params.node_sigma, corr_dist=params.corr_dist,
                                 corr_normal=params.corr_normal, edge_gate=params.edge_gate,
                                 damping=params.damping, rigid_iters=8)
    st = swgn.Stream(cfg)
    st.set_reference_surfels(pos, nrm)
    st.set_node_graph(nodes)
    stats = st.solve_frame(depth)
    se3 = st.node_se3().reshape(-1, 3, 4).astype(np.float64)
    st.close()
    ang = Rotation.from_matrix(se3[:, :, :3] @ Rs.T).magnitude()
    assert ang.max() < 2e-5, ang.max()
    assert np.max(np.abs(se3[:, :, 3] - ts)) < 2e-6
    assert stats["rigid_e"][-1] < 1e-6 * stats["rigid_e"][0]


def test_rigid_streams_alone_and_in_a_batch(swgn, scene_cache):
    scenes = [scene_cache("tiny"), scene_cache("c1"), scene_cache("random", 400)]
    cfgs = [dict(rigid_iters=2), {}, dict(rigid_iters=4, gn_iters=3)]
    want = []
    for sc, c in zip(scenes, cfgs):
        st = stream_for(swgn, sc, **c)
        st.solve_frame(sc.depth)
        want.append(st.node_se3())
        st.close()
    sts = [stream_for(swgn, sc, **c) for sc, c in zip(scenes, cfgs)]
    b = swgn.Batch()
    res, status = b.solve(sts, [sc.depth for sc in scenes])
    assert status == [swgn.SW_OK] * 3
    assert [len(r["rigid_e"]) for r in res] == [2, 0, 4]
    for st, w in zip(sts, want):
        assert np.array_equal(st.node_se3(), w)
        st.close()
    b.close()
