"""The C-ABI library: loads, exports every declared symbol, validates
arguments on the host (no GPU call is made here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swgn.h")
LIB = os.path.join(ROOT, "paper_1904_13073_amd", "libswgn.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sw_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("sw_create_stream", "sw_set_reference_surfels", "sw_set_node_graph",
              "sw_solve_frame", "sw_get_node_se3", "sw_destroy_stream"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for n in declared_symbols():
        assert hasattr(lib, n), n
    from paper_1904_13073_amd import swgn
    assert sorted(swgn.EXPORTS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_defaults_and_status_strings():
    from paper_1904_13073_amd import swgn
    c = swgn.sw_config_default()
    assert (c.width, c.height, c.fx, c.cx, c.cy) == (640, 480, 570.0, 320.0, 240.0)
    assert c.gn_iters == 10 and c.pcg_iters == 10
    assert abs(c.node_sigma - 0.025) < 1e-9 and c.lambda_reg == 5.0
    assert c.debug_iter == -1 and c.dot_fp64 == 1
    L = swgn.lib()
    assert L.sw_status_string(0) == b"ok"
    assert L.sw_status_string(-5) == b"numerical failure"
    assert L.sw_last_error(None) == b"null stream"
    assert L.sw_destroy_stream(None) == 0
    assert L.sw_solve_frame(None, None, 0, None) == swgn.SW_EINVAL
    assert L.sw_get_sizes(None, None, None, None) == swgn.SW_EINVAL
    diff = (C.c_int64 * 9)()
    assert L.sw_check_layout(None, diff) == swgn.SW_EINVAL
    assert L.sw_get_layout(None, None) == swgn.SW_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("field,value", [
    ("width", 0), ("height", -3), ("fx", 0.0), ("fy", float("nan")), ("cx", float("inf")),
    ("gn_iters", 17), ("gn_iters", -1), ("pcg_iters", 5000), ("lambda_reg", -1.0),
    ("node_sigma", 0.0), ("corr_dist", 0.0), ("corr_normal", 1.5), ("edge_gate", -0.1),
    ("damping", float("nan")), ("jac_dtype", 7), ("debug_iter", -2), ("stage_timing", 2),
    ("rigid_iters", 17), ("rigid_iters", -1), ("visibility", 2), ("stable_conf", float("inf")),
    ("recent_frames", -2), ("fusion_dist", 0.0), ("fusion_normal", 1.5),
    ("warp_eps", 0.0), ("warp_eps", 1.0), ("append_nn", -0.1), ("append_nn", float("nan")), ("t_low_confid", -1), ("splat", 2),
])
def test_create_rejects_bad_config(field, value):
    from paper_1904_13073_amd import swgn
    c = swgn.sw_config_default(**{field: value})
    h = C.c_void_p()
    st = swgn.lib().sw_create_stream(C.byref(c), None, C.byref(h))
    assert st == swgn.SW_EINVAL and not h.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_batch_entry_points_validate_on_the_host():
    from paper_1904_13073_amd import swgn
    L = swgn.lib()
    h = C.c_void_p()
    assert L.sw_create_batch(None, 16, C.byref(h)) == swgn.SW_EINVAL and not h.value
    both = swgn.SW_BATCH_TIMING | swgn.SW_BATCH_GRAPH       # timing and graph replay exclude each other
    assert L.sw_create_batch(None, both, C.byref(h)) == swgn.SW_EINVAL and not h.value
    both = swgn.SW_BATCH_PCG_SPLIT | swgn.SW_BATCH_PCG_FUSED   # one PCG schedule or the other
    assert L.sw_create_batch(None, both, C.byref(h)) == swgn.SW_EINVAL and not h.value
    assert L.sw_create_batch(None, 0, None) == swgn.SW_EINVAL
    assert L.sw_destroy_batch(None) == 0
    assert L.sw_batch_last_error(None) == b"null batch"
    assert L.sw_solve_batch(None, None, 1, None, 0, None, None) == swgn.SW_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_server_entry_points_validate_on_the_host():
    from paper_1904_13073_amd import swgn
    L = swgn.lib()
    cfg = swgn.SwServerConfig()
    L.sw_server_config_default(C.byref(cfg))
    assert cfg.max_batch == 32 and cfg.workspace_bytes == 4 << 30
    h = C.c_void_p()
    for mb, ws in ((0, 1 << 20), (65, 1 << 20), (4, 100)):
        bad = swgn.SwServerConfig(max_batch=mb, workspace_bytes=ws)
        assert L.sw_create_server(C.byref(bad), None, C.byref(h)) == swgn.SW_EINVAL and not h.value
    assert L.sw_destroy_server(None) == 0
    assert L.sw_server_last_error(None) == b"null server"
    t = C.c_uint64()
    assert L.sw_server_submit(None, None, None, 0, C.byref(t)) == swgn.SW_EINVAL
    assert L.sw_server_poll(None, 1, 0, None, None) == swgn.SW_EINVAL
    assert L.sw_server_attach(None, None) == swgn.SW_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_fusion_entry_points_validate_on_the_host():
    from paper_1904_13073_amd import swgn
    L = swgn.lib()
    st = swgn.SwFusionStats()
    assert L.sw_fuse_frame(None, None, 0, 0, C.byref(st)) == swgn.SW_EINVAL
    assert L.sw_set_surfel_attributes(None, 1, None, None, None, None, 0) == swgn.SW_EINVAL
    assert L.sw_get_surfel_attributes(None, None, None, None, None) == swgn.SW_EINVAL
    assert L.sw_get_reference_surfels(None, None, None) == swgn.SW_EINVAL
    assert L.sw_set_frame_time(None, 3) == swgn.SW_EINVAL
    assert L.sw_get_last_fusion(None, None, None, None) == swgn.SW_EINVAL
    c = swgn.sw_config_default()
    assert c.visibility == 0 and c.recent_frames == 2 and abs(c.stable_conf - 10.0) < 1e-6
    assert abs(c.fusion_dist - 0.001) < 1e-9 and abs(c.fusion_normal - 0.85) < 1e-6
    assert abs(c.warp_eps - 0.2) < 1e-7 and abs(c.append_nn - 0.3) < 1e-7
    ast = swgn.SwAppendStats()
    assert L.sw_append_candidates(None, 0, 0, None, None, None, None, None, C.byref(ast)) == swgn.SW_EINVAL
    assert L.sw_get_live_nodes(None, None) == swgn.SW_EINVAL
    gst = swgn.SwGeometryStats()
    assert L.sw_update_geometry(None, C.byref(gst)) == swgn.SW_EINVAL
    assert c.t_low_confid == 30
