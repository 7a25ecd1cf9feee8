"""ctypes binding of the swgn C ABI (include/swgn.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Functions keep the C names; a failing status raises SwError with the stream's
last error message. Arrays are NumPy (host, on_device=0) or torch tensors on
the GPU (device, on_device=1); anything else with a `data_ptr()` is taken as
a device pointer.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from typing import Optional

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libswgn.so")

SW_OK, SW_EINVAL, SW_ESTATE, SW_ENOMEM, SW_EHIP, SW_ENUMERIC = 0, -1, -2, -3, -4, -5


class SwConfig(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("gn_iters", C.c_int32), ("pcg_iters", C.c_int32),
                ("lambda_reg", C.c_float), ("node_sigma", C.c_float), ("corr_dist", C.c_float),
                ("corr_normal", C.c_float), ("edge_gate", C.c_float), ("damping", C.c_float),
                ("jac_dtype", C.c_int32), ("dot_fp64", C.c_int32), ("debug_iter", C.c_int32),
                ("stage_timing", C.c_int32), ("rigid_iters", C.c_int32), ("visibility", C.c_int32),
                ("stable_conf", C.c_float), ("recent_frames", C.c_int32), ("fusion_dist", C.c_float),
                ("fusion_normal", C.c_float), ("warp_eps", C.c_float), ("append_nn", C.c_float),
                ("t_low_confid", C.c_int32), ("splat", C.c_int32)]


class SwFusionStats(C.Structure):
    _fields_ = [("n_fused", C.c_int32), ("n_candidates", C.c_int32)]


class SwAppendStats(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("n_far", C.c_int32), ("n_compressive", C.c_int32),
                ("n_appended", C.c_int32), ("n_written", C.c_int32)]


class SwGeometryStats(C.Structure):
    _fields_ = [("n_removed", C.c_int32), ("n_surfels", C.c_int32), ("append", SwAppendStats)]


class SwFrameStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("e_data", C.c_float * 16), ("e_reg", C.c_float * 16),
                ("n_corr", C.c_int32 * 16), ("pcg_resid", C.c_float * 16),
                ("stage_us", C.c_float * 12), ("alg_bytes", C.c_double), ("rigid_steps", C.c_int32),
                ("rigid_e", C.c_float * 16), ("rigid_n", C.c_int32 * 16)]

    def as_dict(self) -> dict:
        n, m = self.iters, self.rigid_steps
        return dict(iters=n, e_data=list(self.e_data[:n]), e_reg=list(self.e_reg[:n]),
                    n_corr=list(self.n_corr[:n]), pcg_resid=list(self.pcg_resid[:n]),
                    stage_us=list(self.stage_us[:12]), alg_bytes=self.alg_bytes,
                    rigid_e=list(self.rigid_e[:m]), rigid_n=list(self.rigid_n[:m]))


class SwServerConfig(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("reserved", C.c_int32), ("workspace_bytes", C.c_int64)]


class SwTicketInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


class SwServerInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("frames_done", C.c_int64), ("max_in_flight", C.c_int32),
                ("pending", C.c_int32), ("in_flight", C.c_int32), ("reserved", C.c_int32),
                ("workspace_bytes", C.c_int64), ("workspace_peak", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SwLayout(C.Structure):
    _fields_ = [("node_sets", C.c_int32), ("segments", C.c_int32), ("packs", C.c_int32),
                ("ell_width", C.c_int32), ("fold_entries", C.c_int64), ("gram_floats", C.c_int64)]


class SwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None

# Handles still open at interpreter exit are destroyed by an exit hook, which
# runs before the HIP runtime and any profiler tear down; servers first (they
# reference streams), then batches, then streams. After that hook, and while
# the interpreter finalises, a finalizer makes no library call at all: a HIP
# call into a runtime that is being torn down can crash the process.
_open = {"server": weakref.WeakSet(), "batch": weakref.WeakSet(), "stream": weakref.WeakSet()}
_exiting = False


def _no_more_calls() -> bool:
    return _exiting or sys.is_finalizing()


@atexit.register
def _close_open_handles():
    global _exiting
    for kind in ("server", "batch", "stream"):
        for obj in list(_open[kind]):
            try:
                obj.close()
            except Exception:
                pass
    _exiting = True

EXPORTS = ["sw_config_default", "sw_status_string", "sw_last_error", "sw_create_stream",
           "sw_destroy_stream", "sw_set_reference_surfels", "sw_set_node_graph", "sw_set_node_se3",
           "sw_solve_frame", "sw_solve_frame_noalloc", "sw_get_node_se3", "sw_get_sizes", "sw_get_skinning",
           "sw_get_node_graph", "sw_get_pattern", "sw_get_last_maps", "sw_get_last_live_normals",
           "sw_get_last_system",
           "sw_get_last_jacobian", "sw_create_batch", "sw_destroy_batch", "sw_batch_last_error",
           "sw_solve_batch", "sw_profile_stage", "sw_server_config_default", "sw_create_server",
           "sw_destroy_server", "sw_server_last_error", "sw_server_attach", "sw_server_detach",
           "sw_server_submit", "sw_server_poll", "sw_server_counters", "sw_get_footprint",
           "sw_batch_autotune", "sw_get_layout", "sw_check_layout", "sw_set_surfel_attributes", "sw_get_surfel_attributes",
           "sw_get_reference_surfels", "sw_set_frame_time", "sw_fuse_frame", "sw_get_last_fusion",
           "sw_append_candidates", "sw_get_live_nodes", "sw_update_geometry"]

SW_EPENDING = 1

SW_BATCH_TIMING = 1
SW_BATCH_GRAPH = 2
SW_BATCH_PCG_SPLIT = 4
SW_BATCH_PCG_FUSED = 8


def lib() -> C.CDLL:
    """The loaded library. Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"swgn HIP library missing at {_LIB_PATH}: build it with __graft_entry__.build()")
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64, fp, ip = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p
    sig = {
        "sw_config_default": (None, [C.POINTER(SwConfig)]),
        "sw_status_string": (C.c_char_p, [i32]),
        "sw_last_error": (C.c_char_p, [vp]),
        "sw_create_stream": (i32, [C.POINTER(SwConfig), vp, C.POINTER(vp)]),
        "sw_destroy_stream": (i32, [vp]),
        "sw_set_reference_surfels": (i32, [vp, i64, fp, fp, i32]),
        "sw_set_node_graph": (i32, [vp, i32, fp, fp, i32]),
        "sw_set_node_se3": (i32, [vp, fp, i32, i32]),
        "sw_solve_frame": (i32, [vp, fp, i32, C.POINTER(SwFrameStats)]),
        "sw_solve_frame_noalloc": (i32, [vp, fp, i32, C.POINTER(SwFrameStats)]),
        "sw_get_node_se3": (i32, [vp, fp, i32]),
        "sw_get_sizes": (i32, [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]),
        "sw_get_skinning": (i32, [vp, ip, fp]),
        "sw_get_node_graph": (i32, [vp, ip]),
        "sw_get_pattern": (i32, [vp, ip, ip]),
        "sw_get_last_maps": (i32, [vp, ip, ip, fp, fp]),
        "sw_get_last_live_normals": (i32, [vp, fp]),
        "sw_get_last_system": (i32, [vp, fp, fp, fp]),
        "sw_get_last_jacobian": (i32, [vp, fp, fp]),
        "sw_set_surfel_attributes": (i32, [vp, i64, fp, fp, ip, ip, i32]),
        "sw_get_surfel_attributes": (i32, [vp, fp, fp, ip, ip]),
        "sw_get_reference_surfels": (i32, [vp, fp, fp]),
        "sw_set_frame_time": (i32, [vp, i32]),
        "sw_fuse_frame": (i32, [vp, fp, i32, i32, C.POINTER(SwFusionStats)]),
        "sw_get_last_fusion": (i32, [vp, ip, fp, fp]),
        "sw_append_candidates": (i32, [vp, i32, i32, ip, fp, fp, fp, fp, C.POINTER(SwAppendStats)]),
        "sw_get_live_nodes": (i32, [vp, fp]),
        "sw_update_geometry": (i32, [vp, C.POINTER(SwGeometryStats)]),
        "sw_create_batch": (i32, [vp, i32, C.POINTER(vp)]),
        "sw_destroy_batch": (i32, [vp]),
        "sw_batch_last_error": (C.c_char_p, [vp]),
        "sw_solve_batch": (i32, [vp, C.POINTER(vp), i32, C.POINTER(vp), i32, C.POINTER(SwFrameStats),
                                 C.POINTER(i32)]),
        "sw_profile_stage": (i32, [vp, C.POINTER(vp), i32, i32, i32, i32, C.POINTER(C.c_float)]),
        "sw_server_config_default": (None, [C.POINTER(SwServerConfig)]),
        "sw_create_server": (i32, [C.POINTER(SwServerConfig), vp, C.POINTER(vp)]),
        "sw_destroy_server": (i32, [vp]),
        "sw_server_last_error": (C.c_char_p, [vp]),
        "sw_server_attach": (i32, [vp, vp]),
        "sw_server_detach": (i32, [vp, vp]),
        "sw_server_submit": (i32, [vp, vp, fp, i32, C.POINTER(C.c_uint64)]),
        "sw_server_poll": (i32, [vp, C.c_uint64, i32, C.POINTER(SwFrameStats), C.POINTER(SwTicketInfo)]),
        "sw_server_counters": (i32, [vp, C.POINTER(SwServerInfo)]),
        "sw_get_footprint": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "sw_batch_autotune": (i32, [vp, C.POINTER(vp), i32, i32, C.POINTER(i32)]),
        "sw_get_layout": (i32, [vp, C.POINTER(SwLayout)]),
        "sw_check_layout": (i32, [vp, C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(handle, st: int):
    if st != SW_OK:
        msg = lib().sw_last_error(handle).decode() if handle else ""
        name = lib().sw_status_string(st).decode()
        raise SwError(st, f"{name}: {msg}" if msg else name)


def _ptr(a, dtype):
    """(pointer, on_device, keepalive) for a host NumPy array or a device tensor."""
    if a is None:
        return None, 0, None
    if isinstance(a, np.ndarray):
        arr = np.ascontiguousarray(a, dtype=dtype)
        return arr.ctypes.data_as(C.c_void_p), 0, arr
    if hasattr(a, "data_ptr"):
        if hasattr(a, "is_contiguous") and not a.is_contiguous():
            raise ValueError("device tensor must be contiguous")
        if hasattr(a, "is_cuda") and not a.is_cuda:
            return _ptr(a.numpy(), dtype)
        return C.c_void_p(a.data_ptr()), 1, a
    return _ptr(np.asarray(a), dtype)


def sw_config_default(**overrides) -> SwConfig:
    c = SwConfig()
    lib().sw_config_default(C.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def sw_create_stream(cfg: SwConfig, hip_stream: Optional[int] = None):
    h = C.c_void_p()
    st = lib().sw_create_stream(C.byref(cfg), C.c_void_p(hip_stream) if hip_stream else None, C.byref(h))
    if st != SW_OK:
        raise SwError(st, lib().sw_status_string(st).decode())
    return h


def sw_destroy_stream(h):
    _check(None, lib().sw_destroy_stream(h))


def sw_set_reference_surfels(h, pos, nrm):
    p, dev, ka = _ptr(pos, np.float32)
    q, dev2, kb = _ptr(nrm, np.float32)
    if dev != dev2:
        raise ValueError("positions and normals must both be host or both device")
    n = ka.shape[0] if hasattr(ka, "shape") else len(ka)
    _check(h, lib().sw_set_reference_surfels(h, int(n), p, q, dev))


def sw_set_node_graph(h, node_pos, node_se3=None):
    p, dev, ka = _ptr(node_pos, np.float32)
    q, dev2, kb = _ptr(node_se3, np.float32)
    if node_se3 is not None and dev != dev2:
        raise ValueError("node positions and transforms must both be host or both device")
    _check(h, lib().sw_set_node_graph(h, int(ka.shape[0]), p, q, dev))


def sw_set_node_se3(h, se3):
    p, dev, ka = _ptr(se3, np.float32)
    _check(h, lib().sw_set_node_se3(h, p, int(ka.shape[0]), dev))


def sw_solve_frame(h, depth, with_stats: bool = True):
    p, dev, ka = _ptr(depth, np.float32)
    stats = SwFrameStats()
    _check(h, lib().sw_solve_frame(h, p, dev, C.byref(stats) if with_stats else None))
    return stats.as_dict() if with_stats else None


def sw_solve_frame_noalloc(h, depth, with_stats: bool = True):
    p, dev, ka = _ptr(depth, np.float32)
    stats = SwFrameStats()
    _check(h, lib().sw_solve_frame_noalloc(h, p, dev, C.byref(stats) if with_stats else None))
    return stats.as_dict() if with_stats else None


def sw_create_batch(hip_stream: Optional[int] = None, flags: int = 0):
    h = C.c_void_p()
    st = lib().sw_create_batch(C.c_void_p(hip_stream) if hip_stream else None, int(flags), C.byref(h))
    if st != SW_OK:
        raise SwError(st, lib().sw_status_string(st).decode())
    return h


def sw_destroy_batch(b):
    lib().sw_destroy_batch(b)


def sw_solve_batch(b, handles, depths, with_stats: bool = True, raise_numeric: bool = True):
    """Solve one frame per stream handle; returns (stats dicts or None, per-stream statuses)."""
    n = len(handles)
    if len(depths) != n:
        raise ValueError("one depth image per stream")
    ptrs, devs, keep = [], [], []
    for d in depths:
        p, dev, ka = _ptr(d, np.float32)
        ptrs.append(p)
        devs.append(dev)
        keep.append(ka)
    if len(set(devs)) > 1:
        raise ValueError("depths must be all host arrays or all device tensors")
    hs = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    ds = (C.c_void_p * n)(*[p.value for p in ptrs])
    stats = (SwFrameStats * n)()
    status = (C.c_int32 * n)()
    st = lib().sw_solve_batch(b, hs, n, ds, devs[0], stats if with_stats else None, status)
    if st != SW_OK and not (st == SW_ENUMERIC and not raise_numeric):
        msg = lib().sw_batch_last_error(b).decode()
        raise SwError(st, f"{lib().sw_status_string(st).decode()}: {msg}")
    return ([stats[i].as_dict() for i in range(n)] if with_stats else None), list(status)


class Batch:
    """A batch executor: solves one frame for each of several Streams per call."""

    def __init__(self, hip_stream: Optional[int] = None, timing: bool = False, graph: bool = False,
                 pcg: str = "auto"):
        """pcg: "auto" (chosen per batch shape), "split" (a product and a finish
        launch per PCG iteration) or "fused" (one fused step per iteration)."""
        modes = {"auto": 0, "split": SW_BATCH_PCG_SPLIT, "fused": SW_BATCH_PCG_FUSED}
        if pcg not in modes:
            raise ValueError(f"pcg must be one of {sorted(modes)}")
        self.h = sw_create_batch(hip_stream, (SW_BATCH_TIMING if timing else 0) | (SW_BATCH_GRAPH if graph else 0)
                                 | modes[pcg])
        _open["batch"].add(self)

    def close(self):
        if self.h:
            sw_destroy_batch(self.h)
            self.h = None

    def __del__(self, _stop=_no_more_calls):
        try:
            if _stop():
                return
            self.close()
        except Exception:
            pass

    def solve(self, streams, depths, with_stats: bool = True, raise_numeric: bool = True):
        return sw_solve_batch(self.h, [s.h for s in streams], depths, with_stats, raise_numeric)

    def autotune(self, streams, reps: int = 20):
        """Pick each stage's launch variant for this batch's shape bucket; returns the 12
        choices (bit 0: XCD-contiguous tile order, bit 1: 2 rows / nodes per wave or group,
        bit 2 of entry 5: fused PCG steps)."""
        n = len(streams)
        hs = (C.c_void_p * n)(*[s.h.value for s in streams])
        out = (C.c_int32 * 12)()
        st = lib().sw_batch_autotune(self.h, hs, n, int(reps), out)
        if st != SW_OK:
            raise SwError(st, f"{lib().sw_status_string(st).decode()}: {lib().sw_batch_last_error(self.h).decode()}")
        return list(out)

    def profile_stage(self, streams, stage: int, reps: int = 100, pcg_it: int = 0) -> float:
        """Mean microseconds per launch of one stage over these streams."""
        n = len(streams)
        hs = (C.c_void_p * n)(*[s.h.value for s in streams])
        us = C.c_float()
        st = lib().sw_profile_stage(self.h, hs, n, int(stage), int(pcg_it), int(reps), C.byref(us))
        if st != SW_OK:
            raise SwError(st, f"{lib().sw_status_string(st).decode()}: {lib().sw_batch_last_error(self.h).decode()}")
        return us.value


class Server:
    """Serving loop: attach Streams, submit frames as they arrive, poll tickets."""

    def __init__(self, max_batch: int = 32, workspace_bytes: int = 4 << 30, hip_stream: Optional[int] = None):
        cfg = SwServerConfig()
        lib().sw_server_config_default(C.byref(cfg))
        cfg.max_batch = int(max_batch)
        cfg.workspace_bytes = int(workspace_bytes)
        h = C.c_void_p()
        st = lib().sw_create_server(C.byref(cfg), C.c_void_p(hip_stream) if hip_stream else None, C.byref(h))
        if st != SW_OK:
            raise SwError(st, lib().sw_status_string(st).decode())
        self.h = h
        self._keep = {}
        _open["server"].add(self)

    def _check(self, st: int):
        if st != SW_OK:
            raise SwError(st, f"{lib().sw_status_string(st).decode()}: {lib().sw_server_last_error(self.h).decode()}")

    def close(self):
        if self.h:
            lib().sw_destroy_server(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self, _stop=_no_more_calls):
        try:
            if _stop():
                return
            self.close()
        except Exception:
            pass

    def attach(self, stream):
        self._check(lib().sw_server_attach(self.h, stream.h))

    def detach(self, stream):
        self._check(lib().sw_server_detach(self.h, stream.h))

    def submit(self, stream, depth) -> int:
        p, dev, ka = _ptr(depth, np.float32)
        t = C.c_uint64()
        self._check(lib().sw_server_submit(self.h, stream.h, p, dev, C.byref(t)))
        if dev:
            self._keep[t.value] = ka       # a device image must outlive its frame
        return t.value

    def poll(self, ticket: int, wait_ms: int = -1):
        """(stats dict, info dict) when the frame is done, None while it is pending."""
        stats, info = SwFrameStats(), SwTicketInfo()
        st = lib().sw_server_poll(self.h, C.c_uint64(ticket), int(wait_ms), C.byref(stats), C.byref(info))
        if st == SW_EPENDING:
            return None
        self._check(st)
        self._keep.pop(ticket, None)
        return stats.as_dict(), {"status": info.status, "t_submit": info.t_submit, "t_admit": info.t_admit,
                                 "t_done": info.t_done}

    def counters(self) -> dict:
        out = SwServerInfo()
        self._check(lib().sw_server_counters(self.h, C.byref(out)))
        return out.as_dict()


def sw_get_sizes(h):
    ns, nn, nb = C.c_int64(), C.c_int32(), C.c_int32()
    _check(h, lib().sw_get_sizes(h, C.byref(ns), C.byref(nn), C.byref(nb)))
    return ns.value, nn.value, nb.value


def sw_get_footprint(h):
    res, ws = C.c_int64(), C.c_int64()
    _check(h, lib().sw_get_footprint(h, C.byref(res), C.byref(ws)))
    return res.value, ws.value


def sw_get_node_se3(h) -> np.ndarray:
    _, nn, _ = sw_get_sizes(h)
    out = np.empty((nn, 12), np.float32)
    _check(h, lib().sw_get_node_se3(h, out.ctypes.data_as(C.c_void_p), nn))
    return out


def sw_get_skinning(h):
    ns, _, _ = sw_get_sizes(h)
    idx = np.empty((ns, 4), np.int32)
    w = np.empty((ns, 4), np.float32)
    _check(h, lib().sw_get_skinning(h, idx.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)))
    return idx, w


def sw_get_node_graph(h) -> np.ndarray:
    _, nn, _ = sw_get_sizes(h)
    out = np.empty((nn, 8), np.int32)
    _check(h, lib().sw_get_node_graph(h, out.ctypes.data_as(C.c_void_p)))
    return out


def sw_get_pattern(h):
    _, nn, nb = sw_get_sizes(h)
    rp = np.empty(nn + 1, np.int32)
    ci = np.empty(nb, np.int32)
    _check(h, lib().sw_get_pattern(h, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p)))
    return rp, ci


def sw_get_last_maps(h, width: int, height: int):
    ns, _, _ = sw_get_sizes(h)
    I = np.empty((height, width), np.int32)
    Cm = np.empty((height, width), np.int32)
    live = np.empty((ns, 3), np.float32)
    nrm = np.empty((3, height, width), np.float32)
    _check(h, lib().sw_get_last_maps(h, I.ctypes.data_as(C.c_void_p), Cm.ctypes.data_as(C.c_void_p),
                                     live.ctypes.data_as(C.c_void_p), nrm.ctypes.data_as(C.c_void_p)))
    return I, Cm, live, nrm


def sw_get_last_live_normals(h) -> np.ndarray:
    ns, _, _ = sw_get_sizes(h)
    out = np.empty((ns, 3), np.float32)
    _check(h, lib().sw_get_last_live_normals(h, out.ctypes.data_as(C.c_void_p)))
    return out


def sw_get_last_system(h):
    _, nn, nb = sw_get_sizes(h)
    blocks = np.empty((nb, 6, 6), np.float32)
    g = np.empty((nn, 6), np.float32)
    delta = np.empty((nn, 6), np.float32)
    _check(h, lib().sw_get_last_system(h, blocks.ctypes.data_as(C.c_void_p), g.ctypes.data_as(C.c_void_p),
                                       delta.ctypes.data_as(C.c_void_p)))
    return blocks, g, delta


def sw_get_last_jacobian(h):
    ns, _, _ = sw_get_sizes(h)
    r = np.empty(ns, np.float32)
    J = np.empty((ns, 4, 6), np.float32)
    _check(h, lib().sw_get_last_jacobian(h, r.ctypes.data_as(C.c_void_p), J.ctypes.data_as(C.c_void_p)))
    return r, J


def sw_set_surfel_attributes(h, radius=None, confidence=None, t_observed=None, t_init=None):
    ns, _, _ = sw_get_sizes(h)
    pr, dr, kr = _ptr(radius, np.float32)
    pc, dc, kc = _ptr(confidence, np.float32)
    pt, dt, kt = _ptr(t_observed, np.int32)
    pi, di, ki = _ptr(t_init, np.int32)
    devs = {d for d, p in ((dr, pr), (dc, pc), (dt, pt), (di, pi)) if p is not None}
    if len(devs) > 1:
        raise ValueError("attributes must all be host arrays or all device tensors")
    _check(h, lib().sw_set_surfel_attributes(h, ns, pr, pc, pt, pi, devs.pop() if devs else 0))


def sw_get_surfel_attributes(h, with_t_init: bool = False):
    """(radius, confidence, t_observed[, t_init]) in caller order."""
    ns, _, _ = sw_get_sizes(h)
    r = np.empty(ns, np.float32)
    c = np.empty(ns, np.float32)
    t = np.empty(ns, np.int32)
    ti = np.empty(ns, np.int32)
    _check(h, lib().sw_get_surfel_attributes(h, r.ctypes.data_as(C.c_void_p), c.ctypes.data_as(C.c_void_p),
                                             t.ctypes.data_as(C.c_void_p), ti.ctypes.data_as(C.c_void_p)))
    return (r, c, t, ti) if with_t_init else (r, c, t)


def sw_update_geometry(h) -> dict:
    st = SwGeometryStats()
    _check(h, lib().sw_update_geometry(h, C.byref(st)))
    out = {"n_removed": st.n_removed, "n_surfels": st.n_surfels}
    out["append"] = {f: getattr(st.append, f) for f, _ in st.append._fields_}
    return out


def sw_get_reference_surfels(h):
    ns, _, _ = sw_get_sizes(h)
    pos = np.empty((ns, 3), np.float32)
    nrm = np.empty((ns, 3), np.float32)
    _check(h, lib().sw_get_reference_surfels(h, pos.ctypes.data_as(C.c_void_p), nrm.ctypes.data_as(C.c_void_p)))
    return pos, nrm


def sw_set_frame_time(h, t_now: int):
    _check(h, lib().sw_set_frame_time(h, int(t_now)))


def sw_fuse_frame(h, depth, t_now: int):
    p, dev, ka = _ptr(depth, np.float32)
    st = SwFusionStats()
    _check(h, lib().sw_fuse_frame(h, p, dev, int(t_now), C.byref(st)))
    return dict(n_fused=st.n_fused, n_candidates=st.n_candidates)


def sw_get_last_fusion(h, width: int, height: int):
    ns, _, _ = sw_get_sizes(h)
    m = np.empty((height, width), np.int32)
    lv = np.empty((ns, 3), np.float32)
    ln = np.empty((ns, 3), np.float32)
    _check(h, lib().sw_get_last_fusion(h, m.ctypes.data_as(C.c_void_p), lv.ctypes.data_as(C.c_void_p),
                                       ln.ctypes.data_as(C.c_void_p)))
    return m, lv, ln


def sw_append_candidates(h, max_out: int):
    """Append candidates of the last fusion (host arrays of max_out entries):
    dict of pixel, pos, nrm, radius, confidence (the written ones) and the
    counts."""
    n = int(max_out)
    pix = np.empty(max(n, 1), np.int32)
    pos = np.empty((max(n, 1), 3), np.float32)
    nrm = np.empty((max(n, 1), 3), np.float32)
    rad = np.empty(max(n, 1), np.float32)
    conf = np.empty(max(n, 1), np.float32)
    st = SwAppendStats()
    _check(h, lib().sw_append_candidates(h, n, 0, pix.ctypes.data_as(C.c_void_p), pos.ctypes.data_as(C.c_void_p),
                                         nrm.ctypes.data_as(C.c_void_p), rad.ctypes.data_as(C.c_void_p),
                                         conf.ctypes.data_as(C.c_void_p), C.byref(st)))
    k = st.n_written
    out = {f: getattr(st, f) for f, _ in st._fields_}
    out.update(pixel=pix[:k].copy(), pos=pos[:k].copy(), nrm=nrm[:k].copy(), radius=rad[:k].copy(),
               confidence=conf[:k].copy())
    return out


def sw_get_live_nodes(h) -> np.ndarray:
    _, nn, _ = sw_get_sizes(h)
    out = np.empty((nn, 3), np.float32)
    _check(h, lib().sw_get_live_nodes(h, out.ctypes.data_as(C.c_void_p)))
    return out


class Stream:
    """One depth stream: owns a library handle (convenience over the functions above)."""

    def __init__(self, cfg: Optional[SwConfig] = None, hip_stream: Optional[int] = None, **overrides):
        self.cfg = cfg if cfg is not None else sw_config_default()
        for k, v in overrides.items():
            setattr(self.cfg, k, v)
        self.h = sw_create_stream(self.cfg, hip_stream)
        _open["stream"].add(self)

    def close(self):
        if self.h:
            sw_destroy_stream(self.h)
            self.h = None

    def __del__(self, _stop=_no_more_calls):
        try:
            if _stop():
                return
            self.close()
        except Exception:
            pass

    def set_reference_surfels(self, pos, nrm):
        sw_set_reference_surfels(self.h, pos, nrm)

    def set_node_graph(self, node_pos, node_se3=None):
        sw_set_node_graph(self.h, node_pos, node_se3)

    def set_node_se3(self, se3):
        sw_set_node_se3(self.h, se3)

    def solve_frame(self, depth, with_stats: bool = True):
        return sw_solve_frame(self.h, depth, with_stats)

    def solve_frame_noalloc(self, depth, with_stats: bool = True):
        return sw_solve_frame_noalloc(self.h, depth, with_stats)

    def node_se3(self) -> np.ndarray:
        return sw_get_node_se3(self.h)

    def sizes(self):
        return sw_get_sizes(self.h)

    def layout(self) -> dict:
        out = SwLayout()
        _check(self.h, lib().sw_get_layout(self.h, C.byref(out)))
        return {k: getattr(out, k) for k, _ in out._fields_}

    def check_layout(self) -> dict:
        """Differing element counts between the device's segment layout and
        the host's sequential walk over the same sorted surfels (all 0 when
        they agree)."""
        out = (C.c_int64 * 9)()
        _check(self.h, lib().sw_check_layout(self.h, out))
        names = ("seg_start", "mask", "off", "ent_ptr", "ent_sub", "ent_grad", "pack_start", "pack_seg", "pos4")
        return {k: int(v) for k, v in zip(names, out)}

    def footprint(self):
        """(resident bytes, workspace bytes of one frame in flight)."""
        return sw_get_footprint(self.h)

    def skinning(self):
        return sw_get_skinning(self.h)

    def node_graph(self):
        return sw_get_node_graph(self.h)

    def pattern(self):
        return sw_get_pattern(self.h)

    def last_maps(self):
        return sw_get_last_maps(self.h, self.cfg.width, self.cfg.height)

    def last_live_normals(self):
        return sw_get_last_live_normals(self.h)

    def last_system(self):
        return sw_get_last_system(self.h)

    def last_jacobian(self):
        return sw_get_last_jacobian(self.h)

    def set_surfel_attributes(self, radius=None, confidence=None, t_observed=None, t_init=None):
        sw_set_surfel_attributes(self.h, radius, confidence, t_observed, t_init)

    def surfel_attributes(self, with_t_init: bool = False):
        return sw_get_surfel_attributes(self.h, with_t_init)

    def update_geometry(self) -> dict:
        return sw_update_geometry(self.h)

    def reference_surfels(self):
        return sw_get_reference_surfels(self.h)

    def set_frame_time(self, t_now: int):
        sw_set_frame_time(self.h, t_now)

    def fuse_frame(self, depth, t_now: int):
        return sw_fuse_frame(self.h, depth, t_now)

    def last_fusion(self):
        return sw_get_last_fusion(self.h, self.cfg.width, self.cfg.height)

    def append_candidates(self, max_out: Optional[int] = None):
        return sw_append_candidates(self.h, self.cfg.width * self.cfg.height if max_out is None else max_out)

    def live_nodes(self) -> np.ndarray:
        return sw_get_live_nodes(self.h)


def config_for(scene, **overrides) -> SwConfig:
    """Config of a generated scene (camera and solver settings)."""
    p = scene.params
    c = sw_config_default(width=scene.cam.width, height=scene.cam.height, fx=scene.cam.fx,
                          fy=scene.cam.fy, cx=scene.cam.cx, cy=scene.cam.cy, gn_iters=p.gn_iters,
                          pcg_iters=p.pcg_iters, lambda_reg=p.lambda_reg, node_sigma=p.node_sigma,
                          corr_dist=p.corr_dist, corr_normal=p.corr_normal, edge_gate=p.edge_gate,
                          damping=p.damping, rigid_iters=getattr(p, "rigid_iters", 0))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c
