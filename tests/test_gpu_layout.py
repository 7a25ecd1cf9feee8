"""The segment layout built on the device at sw_set_node_graph (greedy cuts of
the sorted surfels into segments of at most 5 nodes and 232 surfels, packs of
whole segments, the block fold's entries, each surfel's node positions) against
the plain sequential walk over the same sorted surfels and block pattern
(sw_check_layout), element by element, on the workload scenes and on node sets
built to stress the cut: long runs of one node set (cuts inside a run, then
inside the run a merged segment reaches) and many short runs."""
import numpy as np
import pytest

from gpu_common import gpu_lib, stream_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _assert_same(st):
    d = st.check_layout()
    assert all(v == 0 for v in d.values()), d
    return st.layout()


@pytest.mark.parametrize("name,seed", [("tiny", None), ("c1", None), ("c2", None), ("random", 400),
                                       ("random", 401)])
def test_device_layout_matches_sequential_walk(swgn, scene_cache, name, seed):
    s = scene_cache(name, seed)
    st = stream_for(swgn, s)
    lay = _assert_same(st)
    st.close()
    ns = s.surfel_pos.shape[0]
    print(name, seed, lay, flush=True)
    assert -(-ns // 232) <= lay["packs"] <= lay["segments"] <= ns


def _cloud_stream(swgn, pos, nodes):
    cfg = swgn.sw_config_default(width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0, node_sigma=0.5)
    st = swgn.Stream(cfg)
    nrm = np.zeros_like(pos)
    nrm[:, 2] = -1.0
    st.set_reference_surfels(pos.astype(np.float32), nrm.astype(np.float32))
    st.set_node_graph(nodes.astype(np.float32))
    return st


@pytest.mark.parametrize("case", ["one_set", "few_nodes", "clustered", "many_sets", "whole_chunks", "large"])
def test_device_layout_on_constructed_node_sets(swgn, case):
    rng = np.random.default_rng({"one_set": 1, "few_nodes": 2, "clustered": 3, "many_sets": 4, "whole_chunks": 5,
                                 "large": 6}[case])
    if case == "one_set":
        # 9 nodes, every surfel beside node 0 and far from the rest but nodes 1-3:
        # one node set, one run of 5000 surfels, cut every 232
        nodes = np.array([[0, 0, 1], [0.1, 0, 1], [0, 0.1, 1], [0.1, 0.1, 1]] +
                         [[2 + k, 2, 1] for k in range(5)], np.float64)
        pos = np.array([0.02, 0.02, 1.0]) + rng.uniform(-0.004, 0.004, (5000, 3))
    elif case == "few_nodes":
        # 9 nodes on a line, surfels along it: few node sets, runs of hundreds
        nodes = np.stack([np.linspace(0, 1, 9), np.zeros(9), np.ones(9)], axis=1)
        pos = np.stack([rng.uniform(0, 1, 20000), rng.uniform(-0.01, 0.01, 20000), np.ones(20000)], axis=1)
    elif case == "clustered":
        # 12 nodes, surfels in clumps of uneven size: long and short runs mixed
        nodes = rng.uniform(0, 1, (12, 3))
        centers = rng.uniform(0, 1, (40, 3))
        sizes = rng.integers(1, 700, 40)
        pos = np.concatenate([c + rng.normal(0, 0.01, (n, 3)) for c, n in zip(centers, sizes)])
    elif case == "many_sets":
        # 400 nodes and 30000 surfels spread evenly: thousands of short runs
        nodes = rng.uniform(0, 1, (400, 3))
        pos = rng.uniform(0, 1, (30000, 3))
    elif case == "whole_chunks":
        # 32768 surfels: the segment chain is walked in exactly 32 chunks of 1024
        nodes = rng.uniform(0, 1, (300, 3))
        pos = rng.uniform(0, 1, (32768, 3))
    else:
        # 2M surfels and 4000 nodes: the chain over 245 chunks of 8192
        nodes = rng.uniform(0, 1, (4000, 3))
        pos = rng.uniform(0, 1, (2000000, 3))
    st = _cloud_stream(swgn, pos, nodes)
    lay = _assert_same(st)
    st.close()
    print(case, lay, flush=True)
    if case == "one_set":
        assert lay["node_sets"] == 1 and lay["segments"] == -(-5000 // 232)


def test_rebuilds_on_one_stream_equal_fresh_streams(swgn, scene_cache):
    """A node set rebuilt on a stream reuses the device memory of the last
    build (node-set arrays and temporaries); node sets of other sizes in turn
    must give the layout and the solve of a fresh stream, bit for bit."""
    s = scene_cache("c1")
    nodes = s.node_pos
    subsets = [nodes, nodes[: len(nodes) // 2], nodes, nodes[: (2 * len(nodes)) // 3]]
    st = swgn.Stream(swgn.config_for(s))
    st.set_reference_surfels(s.surfel_pos, s.surfel_nrm)
    for k, nd in enumerate(subsets):
        st.set_node_graph(nd)
        assert all(v == 0 for v in st.check_layout().values())
        st.solve_frame(s.depth)
        fresh = swgn.Stream(swgn.config_for(s))
        fresh.set_reference_surfels(s.surfel_pos, s.surfel_nrm)
        fresh.set_node_graph(nd)
        fresh.solve_frame(s.depth)
        assert st.layout() == fresh.layout()
        assert np.array_equal(st.node_se3(), fresh.node_se3()), k
        fresh.close()
    st.close()
