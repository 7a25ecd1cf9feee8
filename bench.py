"""Benchmark: Gauss-Newton frame solves per second on the 640x480 workload.

One step = one whole frame solve (10 GN x 10 PCG iterations over ~250k
surfels and ~1.8k nodes: depth normals, warp + index map, correspondence +
Jacobians, assembly, block-Jacobi + PCG + node update), with the depth frame
and all stream state resident in HBM. Prints one JSON line.

Beside the headline (the plain single stream) it measures the uneven-streams
workload (16 random streams, 320x240 or 640x480, 300-4000 nodes) solved as
batches against the same streams solved one by one, and the serving workload
(48 such streams, Poisson 30 Hz arrivals, each frame a fresh small step of
the stream's motion) served with continuous batching against a plain FIFO of
single-stream solves. Scenes are generated before the GPU is touched, in a
pool of worker processes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# stage_us slots 0..8 (slot 3 holds the fused PCG steps)
KERNELS = ["depth_prep", "warp_zbuf", "corr_jac", "pcg_step", "pcg_init", "pcg_spmv", "pcg_update",
           "node_update", "asm_fold"]
STAGE_ID = {k: i for i, k in enumerate(KERNELS)}
STAGE_ID["pcg_step"] = 13


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=16,
                    help="streams of the uneven-streams workload (random scenes, seeds 400 + s) solved together "
                         "in the batched leg (0 = skip)")
    ap.add_argument("--serve-streams", type=int, default=48,
                    help="streams of the serving workload (random scenes, seeds 500 + s) (0 = skip)")
    ap.add_argument("--serve-hz", type=float, default=30.0, help="Poisson frame rate of each served stream")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="length of the arrival trace")
    ap.add_argument("--serve-frames", type=int, default=4,
                    help="depth frames rendered per served stream (a walk of fresh motion steps, played "
                         "back and forth)")
    ap.add_argument("--workers", type=int, default=16, help="scene-generation worker processes")
    ap.add_argument("--counters", action="store_true",
                    help="short fixed run for hardware-counter passes: 2 plain frames, 2 batched frames of "
                         "the --batch uneven streams and three 256 MiB device copies (the byte-counter "
                         "calibration); prints no JSON")
    ap.add_argument("--cpu-one-thread", type=int, default=1,
                    help="also time the CPU oracle on one thread (0 = all cores only)")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def kernel_bytes(ns, nn, nb, npx, lay):
    """Algorithmic bytes per launch of each kernel (fp32): the data each kernel
    must move at minimum, node tables counted once. `lay` = the stream's work
    layout (segments, fold entries, Gram floats)."""
    return {
        # depth in, normal map out, index-map reset
        "depth_prep": 28.0 * npx,
        # per surfel: position 12, node ids 16, weights 16, index 4; atomic 8
        "warp_zbuf": 56.0 * ns + 32.0 * nn,
        # per surfel: position + normal 24, node ids 16, weights 16, index 4,
        # index map 8, normal map 16, node positions 2; the segments' Gram
        # sub-blocks, J^T r and r^T r out; Jacobian rows stay on chip
        "corr_jac": 86.0 * ns + 48.0 * nn + 4.0 * lay["gram_floats"],
        # fused PCG step: the finish of one iteration for every node and the
        # products of the next (blocks once; per node the FP64 inverse, six
        # vectors in and six out: z, p_prev, u, v, r, x / x, r, z, p, u, v)
        "pcg_step": 144.0 * nb + 288.0 * nn + 12 * 24.0 * nn,
        # per entry: sub-block 144 and its two offsets 8; per diagonal block its
        # J^T r pieces (24 per entry, counted once per node); blocks out (upper
        # and both explicit-row copies), gradient out; the start of PCG: FP64
        # inverse and r, z, p, x out
        "asm_fold": 152.0 * lay["fold_entries"] + 24.0 * nn * 4 + 144.0 * (2 * nb - nn) + 144.0 * nn + 28.0 * nn
                    + 288.0 * nn + 4 * 24.0 * nn,
        # diagonal blocks and gradient in; FP64 inverses and r, z, p, x out
        "pcg_init": 144.0 * nn + 24.0 * nn + 288.0 * nn + 4 * 24.0 * nn,
        # upper blocks once (each is used for a row and, transposed, a column),
        # z and p_prev in, u = A z and v = A p_prev out
        "pcg_spmv": 144.0 * nb + 4 * 24.0 * nn,
        # PCG finish: z, p_prev, u, v, r, x and the inverses in; x, r, z, p out
        "pcg_update": 6 * 24.0 * nn + 288.0 * nn + 4 * 24.0 * nn,
        # twist in; node state and tables out; index map reset
        "node_update": 24.0 * nn + 32.0 * nn + 96.0 * nn + 8.0 * npx,
    }


def replay_us(bx, streams, pcg_iters, reps=200):
    """Mean time per launch of every replayable stage, each launched `reps`
    times back to back between two HIP events on the solve's stream."""
    out = {}
    for k in KERNELS:
        if k in ("depth_prep", "node_update") or (k == "pcg_step" and pcg_iters < 2):
            continue
        pit = min(1, max(0, pcg_iters - 1)) if k in ("pcg_spmv", "pcg_update", "pcg_step") else 0
        out[k] = bx.profile_stage(streams, STAGE_ID[k], reps=reps, pcg_it=pit)
    return out


def launches_per_frame(G, P, fused):
    """Launches of each kernel per frame: one fused step per PCG iteration
    after the first products, or a product and a finish launch; the start of
    PCG rides on the fold and the node update on the last finish (its own
    launch only without PCG)."""
    import numpy as np
    return np.array([1, G, G, G * P if fused else 0, 0, G if fused else G * P, 0 if fused else G * P,
                     0 if P > 0 else G, G], dtype=float)


def stage_roofline(per_frame_us, launches, kb, replay, scale=1.0, streams=1):
    """Achieved GB/s of every replayed kernel (algorithmic bytes x scale / mean
    time per launch) and the roofline entry of the kernel with the largest
    share of the frame."""
    import numpy as np
    rates = {k: scale * kb[k] / (us * 1e-6) / 1e9 for k, us in replay.items() if us > 0}
    share = {k: per_frame_us[i] for i, k in enumerate(KERNELS) if k in replay and launches[i] > 0}
    name = max(share, key=share.get)
    achieved = rates[name]
    traffic = measured_traffic(name, streams)
    roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": scale * kb[name], "avg_launch_us": round(float(replay[name]), 3),
            "launches_per_frame": int(launches[KERNELS.index(name)])}
    if traffic is not None:
        # the bytes the kernel moves beyond L2 (counters) per launch time, beside the algorithmic rate
        roof["traffic_gbs"] = round(traffic / (replay[name] * 1e-6) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_gbs"] / HBM_PEAK_GBS, 4)
    return roof, {k: round(v, 1) for k, v in rates.items()}


def device_copy_gbs(torch, dev, mib=1024, reps=10):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of `mib` MiB (read + write bytes) timed with events over `reps` copies."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbs, 1)


def ping_pong(k, w):
    """Frame of the k-th arrival of a stream with w rendered frames, played
    1, 2, ..., w - 1, w - 2, ..., 0, 1, ... (frame 0 is solved before the
    trace): every arrival is one fresh motion step from the previous one."""
    if w <= 1:
        return 0
    period = 2 * (w - 1)
    q = (k + 1) % period
    return q if q < w else period - q


def arrival_trace(n_streams, hz, seconds, seed=0):
    """Poisson arrivals: (time, stream, arrival index of that stream) triples,
    exponential gaps of mean 1/hz per stream."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ev = []
    for i in range(n_streams):
        t = rng.exponential(1.0 / hz)
        k = 0
        while t < seconds:
            ev.append((t, i, k))
            t += rng.exponential(1.0 / hz)
            k += 1
    ev.sort()
    return ev


def run_served(swgn, sts, frames, trace, max_batch, closed_seconds=0.0):
    """Open loop: frames submitted at their arrival times; latency = done - submit.
    Closed loop (closed_seconds > 0): every stream resubmits as soon as its frame
    is done, for that long; gives the saturated throughput. frames[i] is
    stream i's list of device depth frames."""
    import threading
    sv = swgn.Server(max_batch=max_batch)
    for st in sts:
        sv.attach(st)
    tickets = []
    lock = threading.Lock()
    t0 = time.perf_counter()

    def submit_all():
        for t, i, k in trace:
            d = t - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tk = sv.submit(sts[i], frames[i][ping_pong(k, len(frames[i]))])
            with lock:
                tickets.append(tk)

    th = threading.Thread(target=submit_all)
    th.start()
    infos = []
    k = 0
    while True:
        with lock:
            tk = tickets[k] if k < len(tickets) else None
        if tk is None:
            if not th.is_alive() and k >= len(tickets):
                break
            time.sleep(0.0002)
            continue
        infos.append(sv.poll(tk, wait_ms=-1)[1])
        k += 1
    th.join()
    lat = [1000.0 * (i["t_done"] - i["t_submit"]) for i in infos]
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    ok = all(i["status"] == swgn.SW_OK for i in infos)
    out = {"frames": len(infos), "frames_per_s": round(len(infos) / span, 2),
           "latency_ms": {"p50": round(percentile(lat, 0.5), 3), "p99": round(percentile(lat, 0.99), 3)},
           "max_in_flight": sv.counters()["max_in_flight"], "all_ok": ok}
    if closed_seconds > 0:
        nxt = [len(trace) + i for i in range(len(sts))]
        live = {sv.submit(st, frames[i][ping_pong(nxt[i], len(frames[i]))]): i for i, st in enumerate(sts)}
        done, lat2 = 0, []
        c0 = time.perf_counter()
        first = None
        last = None
        while live:
            for tk in list(live):
                r = sv.poll(tk, wait_ms=0)
                if r is None:
                    continue
                i = live.pop(tk)
                info = r[1]
                first = info["t_submit"] if first is None else min(first, info["t_submit"])
                last = info["t_done"] if last is None else max(last, info["t_done"])
                done += 1
                lat2.append(1000.0 * (info["t_done"] - info["t_submit"]))
                if time.perf_counter() - c0 < closed_seconds:
                    nxt[i] += 1
                    live[sv.submit(sts[i], frames[i][ping_pong(nxt[i], len(frames[i]))])] = i
            time.sleep(0.0001)
        out["saturated"] = {"frames": done, "frames_per_s": round(done / (last - first), 2),
                            "latency_ms": {"p50": round(percentile(lat2, 0.5), 3),
                                           "p99": round(percentile(lat2, 0.99), 3)}}
    sv.close()
    return out


def run_plain_fifo(sts, frames, trace):
    """The same arrivals served one frame at a time in arrival order by plain
    single-stream solves; latency = completion - arrival."""
    lat = []
    t0 = time.perf_counter()
    for t, i, k in trace:
        d = t - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        sts[i].solve_frame(frames[i][ping_pong(k, len(frames[i]))], with_stats=False)
        lat.append(1000.0 * ((time.perf_counter() - t0) - t))
    span = time.perf_counter() - t0 - trace[0][0]
    return {"frames": len(lat), "frames_per_s": round(len(lat) / span, 2),
            "latency_ms": {"p50": round(percentile(lat, 0.5), 3), "p99": round(percentile(lat, 0.99), 3)}}


# the sources compiled into the frame-solve kernels (a change to any of them
# invalidates the committed HBM-traffic counts)
SOLVE_SOURCES = ("frame.hip", "assemble.hip", "solve.hip", "swgn_frame.h", "swgn_impl.h", "swgn_launch.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_1904_13073_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, streams):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (keyed by the launch's workload: 1 = the plain 640x480
    stream, uneven16 = the batch of 16 uneven streams), or None when there is
    none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_640x480.md")
    if not os.path.exists(path):
        return None
    src, table = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and parts[0] == "sources":
                src = parts[1]
            elif len(parts) == 4 and parts[0] == "traffic":
                table[(parts[1], parts[2])] = float(parts[3])
    if src != kernel_source_hash():
        return None
    name = {"corr_jac": "corr_gram", "pcg_update": "pcg_finish"}.get(kernel, kernel)
    return table.get((name, str(streams)))


def host_cpu():
    """The host's logical CPU count and CPU model (lscpu)."""
    import subprocess
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return os.cpu_count(), model


def cpu_baseline(c1, c2, one_thread=True):
    """The FP64 oracle as it stands, timed on this host. The dense mode is the
    reference: normal equations as a dense 6N x 6N matrix, SciPy/LAPACK
    Cholesky. On the 160x120 workload the whole frame (depth preparation and
    all 5 Gauss-Newton iterations) is timed, median of 3, on all BLAS threads
    and on one; on the 640x480 workload one dense Gauss-Newton iteration is
    timed (all threads, and one thread) and scaled to the frame's 10, the
    value reported. The sparse mode (SciPy sparse J^T J, FP64 block-Jacobi
    PCG x 10) is the second figure: 2 of the 10 iterations timed, scaled.
    Skinning and the node graph are setup (as on the GPU) and not timed."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import solve as S
    from oracle.quat import se3_to_rt

    def setup(sc):
        p = sc.params
        pb = S.make_problem(sc.cam, sc.surfel_pos, sc.surfel_nrm, sc.node_pos, sc.depth, p)
        return pb

    def prep(sc, pb):
        t0 = time.perf_counter()
        pb2 = S.make_problem(sc.cam, sc.surfel_pos, sc.surfel_nrm, sc.node_pos, sc.depth, sc.params,
                             idx=pb.idx, w=pb.w, nbr=pb.nbr)
        return pb2, time.perf_counter() - t0

    def gn_iterations(sc, pb, n, linear):
        R, t = se3_to_rt(S.identity_se3(sc.node_pos.shape[0]))
        t0 = time.perf_counter()
        for _ in range(n):
            lin = S.linearize(pb, R, t)
            A, g = S.normal_equations(pb, lin)
            delta = S.solve_cholesky(A, g) if linear == "chol" else S.solve_pcg(A, g, sc.params.pcg_iters)
            R, t = S.update_nodes(pb.node_pos, R, t, delta)
        return (time.perf_counter() - t0) / n

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    pb1, pb2 = setup(c1), setup(c2)

    def c1_frame():
        pb, tp = prep(c1, pb1)
        return tp + c1.params.gn_iters * gn_iterations(c1, pb, c1.params.gn_iters, "chol")

    def c2_frame(linear, n):
        pb, tp = prep(c2, pb2)
        return tp + c2.params.gn_iters * gn_iterations(c2, pb, n, linear), tp

    c1_all = sorted(c1_frame() for _ in range(3))[1]
    c2_all, c2_prep = c2_frame("chol", 1)
    out1 = {}
    if one_thread:
        with threadpool_limits(limits=1):
            out1["c1_frame_s"] = round(sorted(c1_frame() for _ in range(3))[1], 3)
            out1["c2_frame_s"] = round(c2_frame("chol", 1)[0], 3)
    sparse_s, _ = c2_frame("pcg", 2)
    nproc, model = host_cpu()
    return {"value": round(1.0 / c2_all, 5), "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"640x480 workload: depth preparation + 1 of {c2.params.gn_iters} dense Gauss-Newton "
                      f"iterations (6N x 6N FP64 normal equations, LAPACK Cholesky) timed on {threads} BLAS "
                      f"threads, scaled to one frame ({c2_all:.2f} s/frame); skinning excluded as setup",
            "host": {"nproc": nproc, "cpu_model": model},
            "dense": {"c2_frame_s": {"all_threads": round(c2_all, 3), "one_thread": out1.get("c2_frame_s")},
                      "c1_frame_s_median_of_3": {"all_threads": round(c1_all, 3),
                                                 "one_thread": out1.get("c1_frame_s")}},
            "sparse_pcg": {"c2_frame_s": round(sparse_s, 3),
                           "note": "second figure: SciPy sparse J^T J, FP64 block-Jacobi PCG x10, 2 of 10 "
                                   "Gauss-Newton iterations timed on all threads, scaled"}}


def _generate_one(job):
    """One scene (and, for a served stream, its rendered frames) in a worker."""
    from gen.scenes import make_scene, stream_frames
    kind, seed, nframes = job
    sc = make_scene(kind, seed)
    frames = stream_frames(sc, nframes, seed) if nframes > 1 else None
    return sc, frames


def generate(jobs, workers):
    """Scenes of every leg, generated in a pool of forked workers before the
    GPU is touched; results in job order."""
    import multiprocessing as mp
    n = max(1, min(workers, len(jobs), os.cpu_count() or 1))
    if n == 1:
        out = []
        for j in jobs:
            out.append(_generate_one(j))
            print(f"[bench] scenes generated: {len(out)} of {len(jobs)}", file=sys.stderr, flush=True)
        return out
    out = []
    pool = mp.get_context("fork").Pool(n)
    for r in pool.imap(_generate_one, jobs, chunksize=1):
        out.append(r)
        if len(out) % 8 == 0 or len(out) == len(jobs):
            print(f"[bench] scenes generated: {len(out)} of {len(jobs)}", file=sys.stderr, flush=True)
    pool.close()                      # workers leave on their own (no signal to them)
    pool.join()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: a depth stream's solve is not split across GPUs "
              "(streams shard across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    B = max(0, min(args.batch, 64))
    S = 0 if args.counters else max(0, min(args.serve_streams, 64))
    cpu = not (args.no_cpu_baseline or args.counters)
    jobs = [("c2", None, 0)] + ([("c1", None, 0)] if cpu else [])
    jobs += [("random", 400 + k, 0) for k in range(B)]
    jobs += [("random", 500 + k, args.serve_frames) for k in range(S)]
    t0 = time.perf_counter()
    res = generate(jobs, args.workers)
    print(f"[bench] {len(jobs)} scenes generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    scene = res[0][0]
    c1 = res[1][0] if cpu else None
    off = 2 if cpu else 1
    bscenes = [r[0] for r in res[off:off + B]]
    sstreams = res[off + B:]

    import numpy as np
    import torch

    from paper_1904_13073_amd import swgn

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    p = scene.params
    ns, nn = scene.surfel_pos.shape[0], scene.node_pos.shape[0]
    print(f"[bench] 640x480 workload: {ns} surfels, {nn} nodes, {p.gn_iters} GN x {p.pcg_iters} PCG",
          file=sys.stderr, flush=True)
    hip_stream = torch.cuda.current_stream().cuda_stream

    def stream_of(sc, **over):
        st = swgn.Stream(swgn.config_for(sc, **over), hip_stream=hip_stream)
        st.set_reference_surfels(torch.from_numpy(sc.surfel_pos).to(dev), torch.from_numpy(sc.surfel_nrm).to(dev))
        st.set_node_graph(torch.from_numpy(sc.node_pos).to(dev))
        return st

    def make_stream(**over):
        return stream_of(scene, **over)

    depth = torch.from_numpy(scene.depth).to(dev)
    bdepths = [torch.from_numpy(sc.depth).to(dev) for sc in bscenes]
    if args.counters:
        one = make_stream()
        for _ in range(2):
            one.solve_frame(depth, with_stats=False)
        one.close()
        if B > 0:
            sts = [stream_of(sc) for sc in bscenes]
            bx = swgn.Batch(hip_stream=hip_stream)
            for _ in range(2):
                bx.solve(sts, bdepths, with_stats=False)
            bx.close()
            for t in sts:
                t.close()
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] counters run done: {ns} surfels, batch {B}, copy 256 MiB x3", file=sys.stderr, flush=True)
        return
    st = make_stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        st.solve_frame(depth, with_stats=False)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        st.solve_frame(depth, with_stats=False)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fps = args.steps / elapsed
    _, _, nb = st.sizes()
    lay = st.layout()
    st.close()
    print(f"[bench] {args.steps} frames in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # per-kernel times: HIP events around every launch on the solve's stream
    tst = make_stream(stage_timing=1)
    reps = max(5, min(50, args.steps))
    tot = np.zeros(len(KERNELS))
    stats = None
    for _ in range(reps):
        stats = tst.solve_frame(depth)
        tot += np.array(stats["stage_us"][:len(KERNELS)])
    per_frame_us = tot / reps
    G, Pi = p.gn_iters, p.pcg_iters
    fused = bool(per_frame_us[KERNELS.index("pcg_step")] > 0)    # the schedule the plain solve took
    launches = launches_per_frame(G, Pi, fused)
    kb = kernel_bytes(ns, nn, nb, scene.cam.width * scene.cam.height, lay)
    px = swgn.Batch(hip_stream=hip_stream)
    replay = replay_us(px, [tst], Pi)
    px.close()
    tst.close()
    roofline, rates = stage_roofline(per_frame_us, launches, kb, replay)
    copy_gbs = device_copy_gbs(torch, dev)
    roofline["achievable_copy_gbs"] = copy_gbs
    roofline["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    # depth-map fusion after the frame's solve (one call: depth preprocessing,
    # the 4x super-sampled index map, match and fuse; it ends in a sync)
    fst = make_stream()
    fst.solve_frame(depth, with_stats=False)
    fst.fuse_frame(depth, t_now=1)
    torch.cuda.synchronize()
    flat = []
    for k in range(max(5, min(50, args.steps))):
        a = time.perf_counter()
        fstats = fst.fuse_frame(depth, t_now=2 + k)
        flat.append(time.perf_counter() - a)
    # the geometry update after a fusion (removal, appending, compaction and
    # re-skinning of every surfel): each timed call follows an untimed fusion
    fst.close()
    glat = []
    gstats = None
    for k in range(3):
        gst = make_stream()
        gst.solve_frame(depth, with_stats=False)
        gst.fuse_frame(depth, t_now=1)
        torch.cuda.synchronize()
        a = time.perf_counter()
        gstats = gst.update_geometry()
        glat.append(time.perf_counter() - a)
        gst.close()
    fusion = {"us_per_frame": {"p50": round(1e6 * percentile(flat, 0.5), 1),
                               "mean": round(1e6 * float(np.mean(flat)), 1)},
              "n_fused": fstats["n_fused"], "n_candidates": fstats["n_candidates"],
              "geometry_update_ms": {"p50": round(1e3 * percentile(glat, 0.5), 3),
                                     "surfels_after": gstats["n_surfels"],
                                     "appended": gstats["append"]["n_appended"],
                                     "removed": gstats["n_removed"]}}
    print(f"[bench] fusion: {fusion}", file=sys.stderr, flush=True)

    # the same frame with the surfels rendered as opaque disc splats of their
    # depth-surfel radii (pairs per pixel; a surfel may hold several)
    nzc = np.maximum(np.abs(scene.surfel_nrm[:, 2]), np.cos(np.deg2rad(75.0)))
    rad = (np.sqrt(2.0) * scene.surfel_pos[:, 2] / (scene.cam.fx * nzc)).astype(np.float32)
    sst = make_stream(splat=1)
    sst.set_surfel_attributes(rad)
    sres = sst.solve_frame(depth)
    torch.cuda.synchronize()
    a = time.perf_counter()
    nsp = max(5, args.steps // 10)
    for _ in range(nsp):
        sst.solve_frame(depth, with_stats=False)
    torch.cuda.synchronize()
    splat = {"value": round(nsp / (time.perf_counter() - a), 2), "unit": "frames/s",
             "pairs_last_iteration": sres["n_corr"][-1], "point_rule_correspondences": stats["n_corr"][-1]}
    sst.close()
    print(f"[bench] splats: {splat}", file=sys.stderr, flush=True)

    batched = None
    if B > 0:
        batched = run_batched(swgn, torch, bscenes, bdepths, stream_of, hip_stream, args, copy_gbs)
        print(f"[bench] batched x{B}: {batched['value']} frames/s, plain {batched['plain_same_streams']['value']}",
              file=sys.stderr, flush=True)

    served = None
    if S > 0:
        served = run_serving(swgn, torch, dev, sstreams, stream_of, args)

    out = {
        "metric": "GN frame solves/s at 640x480 ~2k nodes; p50/p99 solve latency, served vs plain",
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "640x480 depth (f=570), 3 spheres + bumpy plane, plain single stream",
                   "surfels": ns, "nodes": nn, "blocks": nb, "node_sets": lay["node_sets"],
                   "segments": lay["segments"], "packs": lay["packs"], "gn_iters": p.gn_iters,
                   "pcg_iters": p.pcg_iters, "mode": "plain"},
        "latency_ms": {"p50": round(1000 * percentile(lat, 0.5), 4),
                       "p99": round(1000 * percentile(lat, 0.99), 4)},
        "pcg_schedule": "fused" if fused else "split",
        "kernel_us_per_frame": {k: round(float(v), 2) for k, v in zip(KERNELS, per_frame_us)},
        "kernel_us_per_launch": {k: round(v, 3) for k, v in replay.items()},
        "roofline": roofline,
        "kernel_gbs": rates,
        "n_corr": stats["n_corr"][-1],
        "fusion": fusion,
        "splat": splat,
    }
    if batched is not None:
        out["batched"] = batched
    if served is not None:
        out["served"] = served
    if cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(c1, scene, one_thread=bool(args.cpu_one_thread))
    print(json.dumps(out), flush=True)


def run_batched(swgn, torch, scenes, depths, stream_of, hip_stream, args, copy_gbs):
    """The uneven-streams workload: all streams solved per call in one launch
    per stage (autotuned), against the same streams solved one at a time."""
    import numpy as np
    B = len(scenes)
    sts = [stream_of(sc) for sc in scenes]
    snap = [t.node_se3() for t in sts]
    bx = swgn.Batch(hip_stream=hip_stream)
    torch.cuda.synchronize()
    for _ in range(max(2, args.warmup // 2)):
        bx.solve(sts, depths, with_stats=False)
    orders = bx.autotune(sts, reps=10)      # tile order per stage for this batch shape
    bx.solve(sts, depths, with_stats=False)
    torch.cuda.synchronize()
    nbs = max(5, args.steps // B)
    blat = []
    t0 = time.perf_counter()
    for _ in range(nbs):
        a = time.perf_counter()
        bx.solve(sts, depths, with_stats=False)
        blat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    bel = time.perf_counter() - t0
    # the same streams, one plain solve each
    plat = []
    t0 = time.perf_counter()
    for _ in range(nbs):
        for t, d in zip(sts, depths):
            a = time.perf_counter()
            t.solve_frame(d, with_stats=False)
            plat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    pel = time.perf_counter() - t0
    # one frame from the same start: batched members against solo solves
    for t, s0 in zip(sts, snap):
        t.set_node_se3(s0)
    bx.solve(sts, depths, with_stats=False)
    in_batch = [t.node_se3() for t in sts]
    for t, s0, d in zip(sts, snap, depths):
        t.set_node_se3(s0)
        t.solve_frame(d, with_stats=False)
    same = all(np.array_equal(a, t.node_se3()) for a, t in zip(in_batch, sts))
    bx.close()
    # per-stage times and replays with a timing batch
    tb = swgn.Batch(hip_stream=hip_stream, timing=True)
    tb.solve(sts, depths, with_stats=False)
    tb.autotune(sts, reps=10)
    btot = np.zeros(len(KERNELS))
    breps = 3
    for _ in range(breps):
        res, _ = tb.solve(sts, depths)
        btot += np.array(res[0]["stage_us"][:len(KERNELS)])
    Pi = max(sc.params.pcg_iters for sc in scenes)
    G = max(sc.params.gn_iters for sc in scenes)
    b_replay = replay_us(tb, sts, Pi, reps=50)
    tb.close()
    kb = {}
    for t, sc in zip(sts, scenes):
        ns_, nn_, nb_ = t.sizes()
        k1 = kernel_bytes(ns_, nn_, nb_, sc.cam.width * sc.cam.height, t.layout())
        for k, v in k1.items():
            kb[k] = kb.get(k, 0.0) + v
    shapes = [(sc.cam.width, sc.cam.height, int(sc.node_pos.shape[0]), int(sc.surfel_pos.shape[0])) for sc in scenes]
    for t in sts:
        t.close()
    b_fused = bool(orders[5] & 4)
    b_roof, b_rates = stage_roofline(btot / breps, launches_per_frame(G, Pi, b_fused), kb, b_replay,
                                     streams=f"uneven{B}")
    b_roof["achievable_copy_gbs"] = copy_gbs
    b_roof["frac_of_copy"] = round(b_roof["achieved"] / copy_gbs, 4)
    return {"streams": B, "value": round(B * nbs / bel, 2), "unit": "frames/s",
            "workload": f"{B} uneven streams (random scenes, seeds 400-{399 + B}): 320x240 or 640x480, "
                        f"300-4000 node targets, 4k-300k surfels, motion <=8 deg / 2 cm, 10 GN x 10 PCG",
            "shapes_wh_nodes_surfels": shapes,
            "ms_per_batch": round(1000.0 * bel / nbs, 3),
            "latency_ms": {"p50": round(1000 * percentile(blat, 0.5), 4),
                           "p99": round(1000 * percentile(blat, 0.99), 4)},
            "plain_same_streams": {"value": round(B * nbs / pel, 2), "unit": "frames/s",
                                   "latency_ms": {"p50": round(1000 * percentile(plat, 0.5), 4),
                                                  "p99": round(1000 * percentile(plat, 0.99), 4)}},
            "kernel_us_per_batch_frame": {k: round(float(v), 2) for k, v in zip(KERNELS, btot / breps)},
            "kernel_us_per_launch": {k: round(v, 3) for k, v in b_replay.items()},
            "kernel_gbs": b_rates, "roofline": b_roof, "identical_to_solo": bool(same),
            "pcg_schedule": "fused" if b_fused else "split",
            "launch_variant": {k: ("xcd" if orders[STAGE_ID[k]] & 1 else "linear") +
                               ("+wide" if orders[STAGE_ID[k]] & 2 else "")
                               for k in KERNELS if k not in ("depth_prep", "node_update")
                               and STAGE_ID[k] < len(orders)}}


def run_serving(swgn, torch, dev, streams, stream_of, args):
    """The serving workload: each stream's frames arrive as a Poisson process
    and step its motion; served with continuous batching and, on fresh copies
    of the same streams, by a plain FIFO of single-stream solves."""
    S = len(streams)
    trace = arrival_trace(S, args.serve_hz, args.serve_seconds)
    frames = [[torch.from_numpy(f).to(dev) for f in fr] for _, fr in streams]
    torch.cuda.synchronize()

    def fresh():
        sts = [stream_of(sc) for sc, _ in streams]
        for st, fr in zip(sts, frames):
            st.solve_frame(fr[0], with_stats=False)     # the stream's first frame (not timed)
        torch.cuda.synchronize()
        return sts

    sts = fresh()
    plain = run_plain_fifo(sts, frames, trace)
    for t in sts:
        t.close()
    print(f"[bench] plain FIFO: {plain}", file=sys.stderr, flush=True)
    sts = fresh()
    srv = run_served(swgn, sts, frames, trace, max_batch=S, closed_seconds=2.0)
    for t in sts:
        t.close()
    print(f"[bench] served: {srv}", file=sys.stderr, flush=True)
    sizes = [sc.cam.width for sc, _ in streams]
    return {"streams": S, "hz_per_stream": args.serve_hz, "trace_seconds": args.serve_seconds,
            "offered_frames_per_s": round(len(trace) / args.serve_seconds, 1),
            "workload": f"{S} streams (random scenes, seeds 500-{499 + S}; {sizes.count(640)} at 640x480, "
                        f"{sizes.count(320)} at 320x240), Poisson {args.serve_hz:g} Hz each for "
                        f"{args.serve_seconds:g} s (shortened from 60 s); {args.serve_frames} depth frames "
                        f"rendered per stream along a walk of fresh <=2 deg / 5 mm motion steps, played back "
                        f"and forth, every arrival one step from the previous; solves start from the "
                        f"stream's previous solution",
            "served": srv, "plain_fifo": plain}


if __name__ == "__main__":
    main()
