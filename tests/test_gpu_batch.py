"""Batched solves: streams of uneven shapes solved together in one launch
per Gauss-Newton stage must end exactly where each ends when solved alone
(same kernels, same per-stream arithmetic and summation order), over several
frames, with uneven iteration counts, captures and a failing member."""
import numpy as np
import pytest

from gpu_common import check_frame_against_oracle, gpu_lib, stream_for

pytestmark = pytest.mark.gpu

MIX = [("tiny", None), ("c1", None), ("random", 400), ("random", 402), ("random", 401)]


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _scenes(scene_cache, names=MIX):
    return [scene_cache(n, s) for n, s in names]


def _solo(swgn, scenes, depths_per_frame, cfgs):
    out, stats = [], []
    for i, sc in enumerate(scenes):
        st = stream_for(swgn, sc, **cfgs[i])
        fr = []
        for depths in depths_per_frame:
            fr.append(st.solve_frame(depths[i]))
        out.append(st.node_se3())
        stats.append(fr)
        st.close()
    return out, stats


def _batched(swgn, scenes, depths_per_frame, cfgs, order=None):
    order = list(range(len(scenes))) if order is None else order
    sts = [stream_for(swgn, sc, **cfgs[i]) for i, sc in enumerate(scenes)]
    b = swgn.Batch()
    stats = [[] for _ in scenes]
    for depths in depths_per_frame:
        res, status = b.solve([sts[i] for i in order], [depths[i] for i in order])
        assert status == [swgn.SW_OK] * len(order)
        for k, i in enumerate(order):
            stats[i].append(res[k])
    out = [st.node_se3() for st in sts]
    for st in sts:
        st.close()
    b.close()
    return out, stats


def _assert_same(a_se3, a_stats, b_se3, b_stats):
    for i, (x, y) in enumerate(zip(a_se3, b_se3)):
        assert np.array_equal(x, y), f"stream {i}: node transforms differ"
    for i, (fa, fb) in enumerate(zip(a_stats, b_stats)):
        for sa, sb in zip(fa, fb):
            assert sa["n_corr"] == sb["n_corr"], f"stream {i}"
            assert sa["e_data"] == sb["e_data"] and sa["e_reg"] == sb["e_reg"], f"stream {i}"
            assert sa["pcg_resid"] == sb["pcg_resid"], f"stream {i}"


def test_batch_of_uneven_streams_equals_solo_runs(swgn, scene_cache):
    scenes = _scenes(scene_cache)
    shapes = {(s.cam.width, s.node_pos.shape[0]) for s in scenes}
    assert len(shapes) == len(scenes)          # image sizes and node counts differ
    frames = [[s.depth for s in scenes]]
    cfgs = [{} for _ in scenes]
    solo = _solo(swgn, scenes, frames, cfgs)
    bat = _batched(swgn, scenes, frames, cfgs, order=[3, 0, 4, 2, 1])
    _assert_same(*solo, *bat)
    assert all(st[0]["n_corr"][-1] > 0 for st in solo[1])


def test_batch_with_uneven_iteration_counts_and_two_frames(swgn, scene_cache):
    scenes = _scenes(scene_cache, MIX[:4])
    cfgs = [dict(gn_iters=3, pcg_iters=5), dict(gn_iters=10, pcg_iters=10), dict(gn_iters=0),
            dict(gn_iters=6, pcg_iters=0)]
    rng = np.random.default_rng(5)
    second = []
    for s in scenes:       # a second frame: the same depth with some pixels dropped
        d = s.depth.copy()
        d[rng.random(d.shape) < 0.1] = 0.0
        second.append(d)
    frames = [[s.depth for s in scenes], second]
    solo = _solo(swgn, scenes, frames, cfgs)
    bat = _batched(swgn, scenes, frames, cfgs)
    _assert_same(*solo, *bat)
    assert [len(f[0]["e_data"]) for f in bat[1]] == [3, 10, 0, 6]


def test_batch_from_device_depths_and_capture(swgn, scene_cache):
    import torch
    scenes = _scenes(scene_cache, MIX[:3])
    dev = torch.device("cuda:0")
    depths = [torch.from_numpy(s.depth).to(dev) for s in scenes]
    torch.cuda.synchronize()
    cfgs = [{}, dict(debug_iter=2), {}]
    solo_st = stream_for(swgn, scenes[1], debug_iter=2)
    solo_st.solve_frame(scenes[1].depth)
    want = solo_st.last_maps(), solo_st.last_system()
    solo_st.close()
    sts = [stream_for(swgn, sc, **cfgs[i]) for i, sc in enumerate(scenes)]
    b = swgn.Batch()
    b.solve(sts, depths)
    got = sts[1].last_maps(), sts[1].last_system()
    for w, g in zip(want[0] + want[1], got[0] + got[1]):
        assert np.array_equal(w, g, equal_nan=True)
    for st in sts:
        st.close()
    b.close()


def test_batch_arguments_and_a_failing_member(swgn, scene_cache):
    scenes = _scenes(scene_cache, MIX[:3])
    sts = [stream_for(swgn, sc) for sc in scenes]
    b = swgn.Batch()
    with pytest.raises(swgn.SwError) as e:
        b.solve([sts[0], sts[0]], [scenes[0].depth, scenes[0].depth])
    assert e.value.status == swgn.SW_EINVAL
    bare = swgn.Stream(swgn.config_for(scenes[0]))
    with pytest.raises(swgn.SwError) as e:
        b.solve([sts[0], bare], [scenes[0].depth, scenes[0].depth])
    assert e.value.status == swgn.SW_ESTATE
    bare.close()
    # one member with a non-finite node transform fails; the others are solved
    nn = scenes[1].node_pos.shape[0]
    bad = np.tile(np.eye(3, 4, dtype=np.float32).reshape(1, 12), (nn, 1))
    bad[5, 3] = np.nan
    sts[1].set_node_se3(bad)
    res, status = b.solve(sts, [s.depth for s in scenes], raise_numeric=False)
    assert status == [swgn.SW_OK, swgn.SW_ENUMERIC, swgn.SW_OK]
    assert np.array_equal(sts[1].node_se3(), bad, equal_nan=True)
    want, _ = _solo(swgn, [scenes[0], scenes[2]], [[scenes[0].depth, scenes[2].depth]], [{}, {}])
    assert np.array_equal(sts[0].node_se3(), want[0]) and np.array_equal(sts[2].node_se3(), want[1])
    for st in sts:
        st.close()
    b.close()


def test_graph_replays_equal_eager_launches(swgn, scene_cache):
    """The batch captured once as a HIP graph and replayed frame after frame
    (with host work between replays) ends exactly where launch-by-launch
    solves end; rebuilding a member's node graph forces a new capture."""
    scenes = _scenes(scene_cache, MIX[:3])
    rng = np.random.default_rng(9)
    frames = []
    for _ in range(3):
        fr = []
        for s in scenes:
            d = s.depth.copy()
            d[rng.random(d.shape) < 0.05] = 0.0
            fr.append(d)
        frames.append(fr)
    cfgs = [{}, dict(gn_iters=4, pcg_iters=7), {}]
    eager = _batched(swgn, scenes, frames, cfgs)
    sts = [stream_for(swgn, sc, **cfgs[i]) for i, sc in enumerate(scenes)]
    b = swgn.Batch(graph=True)
    got = [[] for _ in scenes]
    for fr in frames:
        res, status = b.solve(sts, fr)
        assert status == [swgn.SW_OK] * 3
        for i in range(3):
            got[i].append(res[i])
        _ = [st.node_se3() for st in sts]          # host work between replays
    _assert_same(eager[0], eager[1], [st.node_se3() for st in sts], got)
    # a rebuilt member: recaptured, and equal to a fresh eager solve
    sts[1].set_node_graph(scenes[1].node_pos)
    b.solve(sts, frames[0])
    ref = stream_for(swgn, scenes[1], **cfgs[1])
    ref.solve_frame(frames[0][1])
    assert np.array_equal(sts[1].node_se3(), ref.node_se3())
    ref.close()
    for st in sts:
        st.close()
    b.close()


def test_autotuned_tile_order_changes_no_result(swgn, scene_cache):
    """The autotuner only changes which workgroup takes which tile and how
    many rows or nodes a wave takes, never a reduction's shape: frames solved
    after tuning end exactly where untuned solves end."""
    scenes = _scenes(scene_cache, MIX[:4])
    frames = [[s.depth for s in scenes], [s.depth for s in scenes]]
    cfgs = [{} for _ in scenes]
    plain = _batched(swgn, scenes, frames, cfgs)
    sts = [stream_for(swgn, sc) for sc in scenes]
    b = swgn.Batch()
    res0, _ = b.solve(sts, frames[0])
    snap = [st.node_se3() for st in sts]
    variants = b.autotune(sts, reps=5)
    assert len(variants) == 12 and set(variants) <= {0, 1, 2, 3}
    for st, se3 in zip(sts, snap):       # the tuning replays leave the warp fields alone
        assert np.array_equal(st.node_se3(), se3)
    res1, _ = b.solve(sts, frames[1])
    _assert_same(plain[0], plain[1], [st.node_se3() for st in sts], [[a, c] for a, c in zip(res0, res1)])
    for st in sts:
        st.close()
    b.close()


def test_fused_and_split_pcg_schedules_agree_bit_for_bit(swgn, scene_cache):
    """One fused launch per PCG iteration (finish of i - 1 + products of i,
    columns' z and p formed in place) and a product + finish launch per
    iteration run the same operations: results are identical, with uneven
    PCG counts (a stream's last finish rides along with others' steps) and
    the 0 and 1 iteration cases."""
    scenes = _scenes(scene_cache, MIX[:4])
    cfgs = [dict(pcg_iters=7), dict(pcg_iters=10), dict(pcg_iters=1), dict(gn_iters=3, pcg_iters=0)]
    frames = [[s.depth for s in scenes]] * 2
    out = {}
    for mode in ("split", "fused"):
        sts = [stream_for(swgn, sc, **cfgs[i]) for i, sc in enumerate(scenes)]
        b = swgn.Batch(pcg=mode)
        stats = [[] for _ in scenes]
        for depths in frames:
            res, status = b.solve(sts, depths)
            assert status == [swgn.SW_OK] * len(sts), mode
            for i in range(len(sts)):
                stats[i].append(res[i])
        out[mode] = ([st.node_se3() for st in sts], stats)
        for st in sts:
            st.close()
        b.close()
    _assert_same(*out["split"], *out["fused"])
    solo = _solo(swgn, scenes, frames, cfgs)
    _assert_same(*solo, *out["split"])


def test_batched_uneven_member_against_the_oracle(swgn, scene_cache):
    """A member of uneven-stream shape (a random 640x480 or 320x240 scene of
    the uneven-streams workload) solved inside a batch of four different
    streams, against the FP64 oracle: its association at every iteration
    (captured inside the batch) bit for bit against the replica, its
    transforms against the oracle's own association and, strictly, against
    the oracle run on its correspondences."""
    scenes = _scenes(scene_cache, [("random", 400), ("tiny", None), ("c1", None), ("random", 402)])
    G = scenes[0].params.gn_iters

    def run(debug):
        sts = [stream_for(swgn, sc, **({"debug_iter": debug} if i == 0 and debug is not None else {}))
               for i, sc in enumerate(scenes)]
        b = swgn.Batch()
        res, status = b.solve(sts, [s.depth for s in scenes])
        assert status == [swgn.SW_OK] * len(sts)
        cap = None
        if debug is not None:
            I, Cm, live, N = sts[0].last_maps()
            cap = dict(I=I, C=Cm, N=N, live=live, nrm=sts[0].last_live_normals())
        se3 = sts[0].node_se3()
        for st in sts:
            st.close()
        b.close()
        return se3, res[0], cap

    got, stats, _ = run(None)
    caps = []
    for k in range(G):
        se3, _, cap = run(k)
        assert np.array_equal(se3, got), "a captured batch ended elsewhere"
        caps.append(cap)
    s = scenes[0]
    check_frame_against_oracle(s, got, stats, caps,
                               label=f"batched member {s.cam.width}x{s.cam.height}, {s.node_pos.shape[0]} nodes")
