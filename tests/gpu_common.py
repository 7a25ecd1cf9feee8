"""Helpers shared by the GPU tests (no solver arithmetic)."""
import numpy as np
import pytest


def gpu_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X")
    from paper_1904_13073_amd import swgn
    swgn.lib()      # fails loudly if the HIP library is missing
    return swgn


def stream_for(swgn, scene, se3=None, **cfg):
    st = swgn.Stream(swgn.config_for(scene, **cfg))
    st.set_reference_surfels(scene.surfel_pos, scene.surfel_nrm)
    st.set_node_graph(scene.node_pos, None if se3 is None else np.asarray(se3, np.float32))
    return st


def se3_errors(a, b, node_pos):
    """Rotation angle of Ra Rb^T (rad) and distance of the warped node positions (m).

    The angle comes from the quaternion of the nearest rotation (accurate for
    small angles; the trace formula loses ~3e-4 rad to FP32 rounding)."""
    from scipy.spatial.transform import Rotation
    A = np.asarray(a, np.float64).reshape(-1, 3, 4)
    B = np.asarray(b, np.float64).reshape(-1, 3, 4)
    Ra, ta, Rb, tb = A[:, :, :3], A[:, :, 3], B[:, :, :3], B[:, :, 3]
    ang = Rotation.from_matrix(Ra @ np.transpose(Rb, (0, 2, 1))).magnitude()
    p = np.asarray(node_pos, np.float64)
    d = np.linalg.norm(np.einsum("nij,nj->ni", Ra, p) + ta - np.einsum("nij,nj->ni", Rb, p) - tb, axis=1)
    return ang, d


def expected_pattern(idx, nbr, nn):
    """Upper block pattern as a plain definition: every node pair sharing a
    surfel, every graph edge, every diagonal."""
    pairs = set((k, k) for k in range(nn))
    for t in np.unique(np.sort(idx, axis=1), axis=0):
        for a in range(4):
            for b in range(a + 1, 4):
                pairs.add((int(t[a]), int(t[b])))
    for j in range(nn):
        for m in nbr[j]:
            pairs.add((min(j, int(m)), max(j, int(m))))
    rows = [[] for _ in range(nn)]
    for a, b in pairs:
        rows[a].append(b)
    row_ptr = np.zeros(nn + 1, np.int64)
    cols = []
    for k in range(nn):
        cs = sorted(rows[k])
        cols.extend(cs)
        row_ptr[k + 1] = row_ptr[k] + len(cs)
    return row_ptr, np.asarray(cols)


def solve_with_maps(swgn, scene, **cfg):
    """One frame solve of a fresh stream, plus the correspondence map of each
    Gauss-Newton iteration (one captured rerun per iteration, each checked to
    end where the solve did: capturing does not change a solve)."""
    st = stream_for(swgn, scene, **cfg)
    stats = st.solve_frame(scene.depth)
    got = st.node_se3()
    st.close()
    maps = []
    for k in range(cfg.get("gn_iters", scene.params.gn_iters)):
        st = stream_for(swgn, scene, debug_iter=k, **cfg)
        st.solve_frame(scene.depth)
        maps.append(st.last_maps()[1])
        assert np.array_equal(st.node_se3(), got), "a captured solve ended elsewhere"
        st.close()
    return got, stats, maps


def map_flips(maps, trace):
    """Pixels where each iteration's correspondence map differs from the
    oracle's own association (a correspondence that moved by a pixel counts
    twice)."""
    return [int(np.count_nonzero(m != trace["lin"][k]["corr_map"])) for k, m in enumerate(maps)]
