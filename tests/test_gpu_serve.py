"""Serving loop: frames of several streams arrive at different times and are
solved with continuous batching (admission by workspace footprint, one
Gauss-Newton iteration of every frame in flight per step). Every frame's
result must be the same as when its stream is solved alone."""
import time

import numpy as np
import pytest

from gpu_common import check_frame_against_oracle, gpu_lib, solve_with_captures, stream_for

pytestmark = pytest.mark.gpu

MIX = [("tiny", None), ("c1", None), ("random", 400), ("random", 402), ("random", 401)]


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _frames(scene, n, seed):
    """n depth frames of a stream: the scene's depth with seeded dropouts."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = scene.depth.copy()
        d[rng.random(d.shape) < 0.05] = 0.0
        out.append(d)
    return out


def _solo(swgn, scene, frames, **cfg):
    st = stream_for(swgn, scene, **cfg)
    stats = [st.solve_frame(f) for f in frames]
    se3 = st.node_se3()
    st.close()
    return se3, stats


def test_served_frames_equal_solo_solves(swgn, scene_cache):
    scenes = [scene_cache(n, s) for n, s in MIX]
    frames = [_frames(sc, 2, 10 + i) for i, sc in enumerate(scenes)]
    want = [_solo(swgn, sc, frames[i]) for i, sc in enumerate(scenes)]
    sv = swgn.Server(max_batch=8)
    sts = [stream_for(swgn, sc) for sc in scenes]
    for st in sts:
        sv.attach(st)
    tickets = []
    # the first frames back to back (submitting takes microseconds, a frame's
    # ten iterations about a millisecond: later ones join the first in
    # flight), the second ones staggered
    for k in range(2):
        for i, st in enumerate(sts):
            tickets.append((i, k, sv.submit(st, frames[i][k])))
            if k == 1:
                time.sleep(0.0005 * (i + 1))
    got = {}
    for i, k, t in tickets:
        stats, info = sv.poll(t, wait_ms=-1)
        assert info["status"] == swgn.SW_OK
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        got[(i, k)] = stats
    for i, st in enumerate(sts):
        assert np.array_equal(st.node_se3(), want[i][0]), f"stream {i}"
        for k in range(2):
            assert got[(i, k)]["n_corr"] == want[i][1][k]["n_corr"]
            assert got[(i, k)]["e_data"] == want[i][1][k]["e_data"]
    c = sv.counters()
    assert c["frames_done"] == 10 and c["pending"] == 0 and c["in_flight"] == 0
    assert c["max_in_flight"] >= 2
    sv.close()
    for st in sts:
        st.close()


def test_admission_by_workspace_budget(swgn, scene_cache):
    scenes = [scene_cache(n, s) for n, s in MIX[:4]]
    frames = [_frames(sc, 1, 30 + i) for i, sc in enumerate(scenes)]
    want = [_solo(swgn, sc, frames[i])[0] for i, sc in enumerate(scenes)]
    sts = [stream_for(swgn, sc) for sc in scenes]
    ws = [st.footprint()[1] for st in sts]
    budget = max(ws) + min(ws) + 4096     # the two largest never fit together
    sv = swgn.Server(max_batch=8, workspace_bytes=budget)
    for st in sts:
        sv.attach(st)
    tickets = [sv.submit(st, frames[i][0]) for i, st in enumerate(sts)]
    for t in tickets:
        _, info = sv.poll(t)
        assert info["status"] == swgn.SW_OK
    c = sv.counters()
    assert c["workspace_peak"] <= budget and c["frames_done"] == 4
    for i, st in enumerate(sts):
        assert np.array_equal(st.node_se3(), want[i])
    # a stream whose workspace exceeds the budget is refused
    small = swgn.Server(max_batch=2, workspace_bytes=min(ws) - 4096)
    big = stream_for(swgn, scenes[int(np.argmax(ws))])
    with pytest.raises(swgn.SwError) as e:
        small.attach(big)
    assert e.value.status == swgn.SW_EINVAL
    with pytest.raises(swgn.SwError) as e:      # attached to one server at a time
        small.attach(sts[0])
    assert e.value.status == swgn.SW_ESTATE
    big.close()
    small.close()
    sv.close()
    for st in sts:
        st.close()


def test_frames_of_one_stream_run_in_order_and_detach(swgn, scene_cache):
    sc = scene_cache("c1")
    frames = _frames(sc, 3, 50)
    want, _ = _solo(swgn, sc, frames)
    st = stream_for(swgn, sc)
    sv = swgn.Server(max_batch=4)
    sv.attach(st)
    with pytest.raises(swgn.SwError) as e:
        st.solve_frame(frames[0])
    assert e.value.status == swgn.SW_ESTATE
    tickets = [sv.submit(st, f) for f in frames]
    got = st.node_se3()           # waits for the stream's frames
    assert np.array_equal(got, want)
    for t in tickets:
        assert sv.poll(t, wait_ms=0)[1]["status"] == swgn.SW_OK
    sv.detach(st)
    st.solve_frame(frames[0])     # solves alone again with its own workspace
    sv.close()
    st.close()


def test_device_frames_and_a_failing_member(swgn, scene_cache):
    import torch
    scenes = [scene_cache(n, s) for n, s in MIX[:3]]
    dev = torch.device("cuda:0")
    depths = [torch.from_numpy(s.depth).to(dev) for s in scenes]
    torch.cuda.synchronize()
    sts = [stream_for(swgn, sc) for sc in scenes]
    nn = scenes[1].node_pos.shape[0]
    bad = np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (nn, 1))
    bad[3, 3] = np.nan
    sts[1].set_node_se3(bad)
    sv = swgn.Server(max_batch=4)
    for st in sts:
        sv.attach(st)
    tickets = [sv.submit(st, depths[i]) for i, st in enumerate(sts)]
    status = [sv.poll(t)[1]["status"] for t in tickets]
    assert status == [swgn.SW_OK, swgn.SW_ENUMERIC, swgn.SW_OK]
    assert np.array_equal(sts[1].node_se3(), bad, equal_nan=True)
    for i in (0, 2):
        want, _ = _solo(swgn, scenes[i], [scenes[i].depth])
        assert np.array_equal(sts[i].node_se3(), want)
    sv.close()
    for st in sts:
        st.close()


def test_served_frame_against_the_oracle(swgn, scene_cache):
    """A frame of a stream of the uneven-streams workload, served among frames
    of other streams, against the FP64 oracle. The served result equals the
    stream's solo solve bit for bit, so the solo run's per-iteration
    captures are the served frame's association; that association is checked
    against the replica and the transforms against the oracle's own
    association and, strictly, against the oracle on those correspondences."""
    scenes = [scene_cache(n, s) for n, s in [("random", 402), ("c1", None), ("tiny", None)]]
    s = scenes[0]
    solo, stats, caps = solve_with_captures(swgn, s)
    sv = swgn.Server(max_batch=4)
    sts = [stream_for(swgn, sc) for sc in scenes]
    for st in sts:
        sv.attach(st)
    tickets = []
    for i in (1, 0, 2):                    # staggered: the frame joins one in flight
        tickets.append((i, sv.submit(sts[i], scenes[i].depth)))
        time.sleep(0.0005)
    served = {}
    for i, t in tickets:
        st_i, info = sv.poll(t, wait_ms=-1)
        assert info["status"] == swgn.SW_OK
        served[i] = st_i
    got = sts[0].node_se3()
    sv.close()
    for st in sts:
        st.close()
    assert np.array_equal(got, solo)
    assert served[0]["n_corr"] == stats["n_corr"] and served[0]["e_data"] == stats["e_data"]
    check_frame_against_oracle(s, got, served[0], caps,
                               label=f"served frame {s.cam.width}x{s.cam.height}, {s.node_pos.shape[0]} nodes")
