"""The allocation-free solve (sw_solve_frame_noalloc): its frame workspace is
a static device array, not the stream's own. Through the C ABI its results
must equal sw_solve_frame's bit for bit (the same kernels on the same data),
on calls in a row of which a later one is smaller, and the stream's own
workspace must be in use again afterwards."""
import numpy as np
import pytest

from gpu_common import gpu_lib, stream_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swgn():
    return gpu_lib()


def _plain(swgn, s, frames):
    st = stream_for(swgn, s)
    out = []
    for d in frames:
        stats = st.solve_frame(d)
        out.append((st.node_se3(), stats))
    st.close()
    return out


def _same(a, b):
    assert np.array_equal(a[0], b[0])
    for k in ("e_data", "e_reg", "n_corr", "pcg_resid"):
        assert a[1][k] == b[1][k], k


def test_noalloc_equals_solve_frame_on_two_calls_the_second_smaller(swgn, scene_cache):
    import torch
    big, small = scene_cache("c1"), scene_cache("tiny")
    want_big = _plain(swgn, big, [big.depth])[0]
    want_small = _plain(swgn, small, [small.depth])[0]
    a = stream_for(swgn, big)
    b = stream_for(swgn, small)
    ra = a.solve_frame_noalloc(big.depth)
    got_a = a.node_se3()
    dev = torch.device("cuda:0")
    rb = b.solve_frame_noalloc(torch.from_numpy(small.depth).to(dev))     # device depth, smaller frame
    got_b = b.node_se3()
    _same((got_a, ra), want_big)
    _same((got_b, rb), want_small)
    a.close()
    b.close()


def test_stream_workspace_in_use_again_after_a_noalloc_call(swgn, scene_cache):
    s = scene_cache("tiny")
    rng = np.random.default_rng(3)
    d2 = s.depth.copy()
    d2[rng.random(d2.shape) < 0.05] = 0.0
    want = _plain(swgn, s, [s.depth, d2])
    st = stream_for(swgn, s)
    r1 = st.solve_frame_noalloc(s.depth)
    _same((st.node_se3(), r1), want[0])
    r2 = st.solve_frame(d2)                  # the stream's own workspace
    _same((st.node_se3(), r2), want[1])
    st.close()


def test_workspace_above_the_scratch_is_refused(swgn, scene_cache):
    s = scene_cache("tiny")
    st = swgn.Stream(swgn.config_for(s, width=2048, height=1536))     # ~88 MB of per-pixel maps
    st.set_reference_surfels(s.surfel_pos, s.surfel_nrm)
    st.set_node_graph(s.node_pos)
    assert st.footprint()[1] > 64 << 20
    with pytest.raises(swgn.SwError) as e:
        st.solve_frame_noalloc(np.zeros((1536, 2048), np.float32))
    assert e.value.status == swgn.SW_EINVAL
    st.close()
