"""Benchmark: LOD octree build throughput on one MI355X.

Default workload: the 100M-point aerial scene (1 x 1 km: 70% terrain, 20% box
buildings, 10% Gaussian vegetation; float32 xyz + uint8 RGBA), leaf cap
50 000, 128^3 voxel grid per inner node, colour-filtered (cell average).  One
step = one complete lod_build of the whole cloud (bounding box, both
partition passes, node enumeration, leaf and inner voxels, output tables)
plus lod_tree_free, with the input already resident in HBM.

Beside it, on the same box and in the same run:
  batched: 512 independent chunks (lognormal sizes, median 1M, sigma 0.5,
           clipped 10k-20M; terrain + buildings tiles) built by one
           lod_build_batch call, against lod_build on each chunk in turn,
           both with the input resident in HBM;
  served:  Poisson arrivals at 200 requests/s of chunks from host memory
           (lognormal sizes, median 2M, sigma 1.0, clipped 50k-50M; prefixes
           of 50M-point tiles of the same generator) through lod_submit /
           lod_poll, reporting throughput and p50/p99 latency (completion
           minus scheduled arrival, including queueing and the host-to-device
           copy), against the same requests built one by one; and a stream of
           many small requests (50k points at 20 000 requests/s), where the
           server's batching of queued requests into one build matters most;
  full precision: the plain build again with a full-precision record (input
           coordinates of the cell's accepted sample, voxel colour) for every
           voxel of the lower levels;
  weighted: the same cloud with the neighbourhood-weighted average.

Prints one JSON line with the throughput (points/s), the roofline of the
dominant kernel (algorithmic bytes per launch over its average duration,
measured with HIP events on the build stream), the CPU oracle timed on a
bounded sample of the same workload, and the batched and served results.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points/s LOD build (color-filtered, 100M pts), batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "aerial100m": dict(n=100_000_000, gen="aerial", seed=2,
                       desc="aerial 1x1 km: 70% terrain, 20% on 200 box buildings, 10% in 2000 Gaussian blobs"),
    "terrain1m": dict(n=1_000_000, gen="terrain", seed=1, desc="terrain heightfield 100x100 m"),
}
SAMPLING = {"average": 0, "first": 1, "random": 2, "weighted": 3}


def stage_bytes(stage: str, n: int, ids: bool) -> float:
    """Bytes one launch of a stage moves when every array it touches is read
    or written once: 16-byte records, and 4-byte ids when carried.  From 64M
    points on, the first insert also writes each record's 2-byte cell of the
    second partition, which the second count reads instead of the records."""
    idb = 4 if ids else 0
    dig = 2.0 if n >= (64 << 20) else 0.0
    return {
        "bbox": 16.0 * n,
        "count0": 16.0 * n,
        "scatter0": (16.0 + idb + 16.0 + idb + dig) * n,
        "count1": (dig if dig else 16.0) * n,
        "scatter1": (16.0 + idb + 16.0 + idb) * n,
        "leaf_voxels": (16.0 + idb) * n,
    }.get(stage, 0.0)


def method_bytes_per_point(sampling: int, voxels: int, n: int) -> float:
    """Bytes per point the method itself must move (each record pass once):
    AVERAGE 16 (bounding box) + 16 (count) + 32 (insert) + 16 (leaf points
    read) + 16 per voxel (written, then read by the parent level); the pick
    modes add 8 B of ids per point and 8 B of ids per voxel."""
    vn = voxels / max(n, 1)
    if sampling in (1, 2):
        return 80.0 + 8.0 + 24.0 * vn
    return 80.0 + 16.0 * vn


# Library kernels and the build stages (HIP-event brackets) that time their
# main launches.
KERNEL_STAGES = {
    "k_part_scatter": ["scatter0", "scatter1"],
    "k_part_count": ["count0", "count1"],
    "k_leaf_voxels": ["leaf_voxels"],
    "k_bbox": ["bbox"],
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_aerial100m.json")


def measured_traffic(kernel: str, workload: str, sampling: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (calibrated on a plain copy), or None when
    those counters were taken on other kernel sources or another workload."""
    import hashlib
    if workload != "aerial100m" or sampling != 0 or not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    per = [rec["hbm_bytes_per_launch"].get(s) for s in KERNEL_STAGES[kernel]]
    if any(v is None for v in per):
        return None
    return round(sum(per) / len(per), 1)


def params_plain(lod, args, sampling):
    return lod.make_params(leaf_cap=args.leaf_cap, max_level=args.max_level, sampling=sampling)


def run_batched(lod, torch, num_chunks: int, reps: int, params):
    """One lod_build_batch over all chunks (median of `reps`) against
    lod_build per chunk, input resident in HBM in both cases."""
    import synth
    sizes = synth.chunk_sizes(num_chunks, seed=4)
    total = int(sizes.sum())
    print(f"[bench] batched: generating {num_chunks} chunks, {total} points", file=sys.stderr, flush=True)
    host = torch.empty(total * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    _, offs = synth.batch_chunks(sizes, seed=4, out=pts)
    dev = host.to("cuda:0")
    del host, pts
    stream = torch.cuda.current_stream()

    def batch(p):
        trees = lod.lod_build_batch(dev, offs, params=p, stream=stream)
        nodes = sum(t.view().num_nodes for t in trees)
        voxels = sum(t.view().num_voxels for t in trees)
        for t in trees:
            t.free()
        return nodes, voxels

    def timed(p):
        batch(p)  # warm-up (allocations)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = batch(p)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), res

    from paper_2302_14801_amd import autotune
    t0 = time.perf_counter()
    tuned, tune_info = autotune.tune_batch(dev, offs, params, stream=stream)
    tune_info["tuning_s"] = round(time.perf_counter() - t0, 3)
    print(f"[bench] batched: tuned plan {tune_info['plan']}", file=sys.stderr, flush=True)
    t_default, _ = timed(params)
    t_batch, (nodes, voxels) = timed(tuned)
    print(f"[bench] batched: {1e3 * t_batch:.2f} ms per batch; plain builds next", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(num_chunks):
        t = lod.lod_build(dev[int(offs[i]) * 16:int(offs[i + 1]) * 16], params=params, stream=stream)
        t.free()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    del dev
    torch.cuda.empty_cache()
    return {"workload": f"{num_chunks} chunks, lognormal sizes (median 1M, sigma 0.5, clipped 10k-20M), "
                        "terrain+buildings tiles with their own bounding boxes; input resident in HBM",
            "chunks": num_chunks, "points": total, "nodes": nodes, "voxels": voxels,
            "batched_points_per_s": round(total / t_batch, 1), "batched_ms": round(1e3 * t_batch, 3),
            "untuned_points_per_s": round(total / t_default, 1), "autotune": tune_info,
            "plain_points_per_s": round(total / t_plain, 1), "plain_ms": round(1e3 * t_plain, 3),
            "batched_over_plain": round(t_plain / t_batch, 3), "reps": reps}


def run_served(lod, torch, num_requests: int, rate: float, params, budget: int, inflight: int,
               pool_tiles: int, keep: int, fixed_size: int = 0):
    """Open-loop Poisson client of the request server, then the same requests
    built one by one (host to device copy + lod_build each).  Sizes are
    lognormal (median 2M, sigma 1.0, clipped 50k-50M), or all fixed_size."""
    import synth
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / rate, num_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    if fixed_size:
        sizes = np.full(num_requests, fixed_size, np.int64)
    else:
        sizes = synth.chunk_sizes(num_requests, seed=5, median=2e6, sigma=1.0, lo=50_000, hi=50_000_000)
    tile_n = int(min(50_000_000, sizes.max()))
    print(f"[bench] served: generating {pool_tiles} tiles of {tile_n} points", file=sys.stderr, flush=True)
    tiles = []
    for k in range(pool_tiles):
        h = torch.empty(tile_n * 16, dtype=torch.uint8, pin_memory=True)
        synth.serve_tile(tile_n, seed=5000 + k, out=h.numpy().view(synth.POINT_DTYPE))
        tiles.append(h.numpy().view(synth.POINT_DTYPE))
    reqs = [tiles[r % pool_tiles][:int(sizes[r])] for r in range(num_requests)]
    total = int(sizes.sum())

    srv = lod.Server(budget, inflight, params=params)
    # warm-up: one request of each of a few sizes
    for r in range(min(4, num_requests)):
        tk = srv.submit(reqs[r])
        while srv.poll(tk) is None:
            time.sleep(0.0005)
    resident, lat, build_done = [], np.zeros(num_requests), np.zeros(num_requests)
    pending = {}
    print(f"[bench] served: {num_requests} requests at {rate}/s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    nxt = 0
    while nxt < num_requests or pending:
        now = time.perf_counter() - t0
        while nxt < num_requests and arrivals[nxt] <= now:
            pending[srv.submit(reqs[nxt])] = nxt
            nxt += 1
        # the oldest tickets first (the server takes requests in order), a
        # bounded number per sweep so that a long queue does not slow the client
        for tk in list(pending)[:256]:
            t = srv.poll(tk)
            if t is not None:
                i = pending.pop(tk)
                done = time.perf_counter() - t0
                lat[i] = done - arrivals[i]
                build_done[i] = done
                resident.append(t)
                while len(resident) > keep:
                    resident.pop(0).free()
        if nxt < num_requests and not pending:
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
        else:
            time.sleep(0.0002)
    t_served = build_done.max() - arrivals[0]
    for t in resident:
        t.free()
    resident.clear()
    # the same requests all at once (closed loop): the server's throughput
    print("[bench] served: saturated", file=sys.stderr, flush=True)
    s0 = time.perf_counter()
    pending = {srv.submit(reqs[r]): r for r in range(num_requests)}
    while pending:
        for tk in list(pending)[:256]:
            t = srv.poll(tk)
            if t is not None:
                pending.pop(tk)
                resident.append(t)
                while len(resident) > keep:
                    resident.pop(0).free()
        time.sleep(0.0002)
    t_sat = time.perf_counter() - s0
    for t in resident:
        t.free()
    srv.destroy()
    # the same requests one by one
    print("[bench] served: plain sequential builds", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    dbuf = torch.empty(tile_n * 16, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for r in range(num_requests):
        n = int(sizes[r])
        src = torch.from_numpy(reqs[r].view(np.uint8).reshape(-1))
        dbuf[:n * 16].copy_(src, non_blocking=True)
        t = lod.lod_build(dbuf[:n * 16], params=params, stream=stream)
        t.free()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - p0
    del dbuf, tiles, reqs
    torch.cuda.empty_cache()
    size_desc = f"{fixed_size} points each" if fixed_size else "lognormal sizes (median 2M, sigma 1.0, clipped 50k-50M)"
    return {"workload": f"{num_requests} requests, Poisson arrivals at {rate:g}/s, {size_desc}, "
                        f"prefixes of {pool_tiles} pinned host tiles of {tile_n} points; "
                        f"budget {budget >> 30} GiB, {inflight} in flight, newest {keep} trees kept",
            "requests": num_requests, "points": total,
            "served_points_per_s": round(total / t_served, 1),
            "p50_latency_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_latency_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "max_latency_ms": round(1e3 * float(lat.max()), 3),
            "offered_points_per_s": round(total / (arrivals[-1] - arrivals[0]), 1),
            "saturated_points_per_s": round(total / t_sat, 1), "saturated_s": round(t_sat, 3),
            "plain_points_per_s": round(total / t_plain, 1), "plain_s": round(t_plain, 3)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pts, sample: int, args, sampling: int) -> dict:
    """The CPU oracle (single-threaded C) on the first `sample` points of the
    same cloud, pinned to one core, median of args.cpu_reps builds."""
    import oracle
    core = min(os.sched_getaffinity(0))
    saved = os.sched_getaffinity(0)
    times = []
    print(f"[bench] CPU oracle on the first {sample} points, core {core}, {args.cpu_reps} builds",
          file=sys.stderr, flush=True)
    try:
        os.sched_setaffinity(0, {core})
        for r in range(max(1, args.cpu_reps)):
            c0 = time.perf_counter()
            oracle.build(pts[:sample], leaf_cap=args.leaf_cap, max_level=args.max_level, sampling=sampling)
            times.append(time.perf_counter() - c0)
            print(f"[bench] CPU oracle build {r}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    finally:
        os.sched_setaffinity(0, saved)
    med = float(np.median(times))
    whole = "the whole" if sample == len(pts) else f"the first {sample} points of the same"
    return {"value": round(sample / med, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{whole} {args.workload} cloud ({sample} points); single-threaded C oracle pinned to core "
                      f"{core} of {os.cpu_count()} ({cpu_model()}), build only, median of {len(times)}: "
                      + ", ".join(f"{t:.2f}" for t in times) + " s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="aerial100m", choices=sorted(WORKLOADS))
    ap.add_argument("--sampling", default="average", choices=sorted(SAMPLING))
    ap.add_argument("--leaf-cap", type=int, default=50000)
    ap.add_argument("--max-level", type=int, default=12)
    ap.add_argument("--cpu-sample", type=int, default=100_000_000,
                    help="points of the workload the CPU oracle builds (0 = skip)")
    ap.add_argument("--cpu-reps", type=int, default=3, help="CPU oracle builds (the median is reported)")
    ap.add_argument("--profile-copy", action="store_true",
                    help="run one plain device copy of the input first (known bytes, for counter calibration)")
    ap.add_argument("--batch-chunks", type=int, default=512, help="chunks of the batched run (0 = skip)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=400, help="requests of the served run (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-tiles", type=int, default=4)
    ap.add_argument("--serve-small-requests", type=int, default=4000,
                    help="requests of the served run of many small requests (0 = skip)")
    ap.add_argument("--serve-small-rate", type=float, default=20000.0)
    ap.add_argument("--serve-small-points", type=int, default=50_000)
    ap.add_argument("--full-precision-steps", type=int, default=5,
                    help="builds of the same cloud with full-precision lower levels (0 = skip)")
    ap.add_argument("--weighted-steps", type=int, default=3,
                    help="builds of the same cloud with the neighbourhood-weighted average (0 = skip)")
    ap.add_argument("--chunked-steps", type=int, default=2,
                    help="chunked builds of the same cloud from host memory (0 = skip)")
    ap.add_argument("--chunk-points", type=int, default=10_000_000, help="chunk size of the chunked build")
    ap.add_argument("--chunked-forms", default="both", choices=["both", "resident", "streaming"],
                    help="forms of the chunked build to time: cloud resident on the device, or streaming")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this builder has no multi-GPU path "
              "(the chunks of a batch are independent and would be assigned to GPUs by size). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2302_14801_amd as lod
    import synth

    wl = WORKLOADS[args.workload]
    n = wl["n"]
    sampling = SAMPLING[args.sampling]
    ids = sampling in (1, 2)  # pick modes carry point ids through the partition
    print(f"[bench] generating {n} points ({args.workload})", file=sys.stderr, flush=True)
    host = torch.empty(n * 16, dtype=torch.uint8, pin_memory=True)
    pts = host.numpy().view(synth.POINT_DTYPE)
    getattr(synth, wl["gen"])(n, seed=wl["seed"], out=pts)
    dev = host.to("cuda:0", non_blocking=False)
    stream = torch.cuda.current_stream()
    params = lod.make_params(leaf_cap=args.leaf_cap, max_level=args.max_level, sampling=sampling, timing=True)

    def step():
        t = lod.lod_build(dev, params=params, stream=stream)
        tm = t.timings()
        v = t.view()
        info = (v.num_nodes, v.num_voxels)
        t.free()
        return tm, info

    if args.profile_copy:
        cp = torch.empty_like(dev)
        cp.copy_(dev)
        torch.cuda.synchronize()
        del cp
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stages, infos = [], []
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tm, info = step()
        stages.append(tm)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed

    avg = {k: float(np.mean([s[k] for s in stages])) for k in stages[0]}
    single = ["bbox", "count0", "scatter0", "count1", "scatter1", "leaf_voxels"]
    kernels = {}
    for kname, stg in KERNEL_STAGES.items():
        t_ms = sum(avg[s] for s in stg)
        alg = sum(stage_bytes(s, n, ids) for s in stg)
        gbs = alg / (t_ms * 1e-3) / 1e9
        kernels[kname] = {"launches": len(stg), "ms_per_step": round(t_ms, 4), "avg_launch_ms": round(t_ms / len(stg), 4),
                          "algorithmic_bytes_per_launch": alg / len(stg), "achieved_GBps": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kd["frac"], "traffic": measured_traffic(dom, args.workload, sampling),
                "algorithmic_bytes_per_launch": kd["algorithmic_bytes_per_launch"],
                "avg_launch_ms": kd["avg_launch_ms"]}
    whole_alg = sum(stage_bytes(k, n, ids) for k in single)
    nodes, voxels = infos[-1]
    # the whole build against the method's own bytes (each record pass once)
    mb = method_bytes_per_point(sampling, voxels, n)
    whole_gbs = mb * n / (ms_per_step * 1e-3) / 1e9
    whole_roofline = {"bound": "hbm", "bytes_per_point": round(mb, 2), "voxels_per_point": round(voxels / n, 4),
                      "achieved": round(whole_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(whole_gbs / HBM_PEAK_GBS, 4), "ms_per_step": round(ms_per_step, 4),
                      "target_frac": 0.6, "ms_at_target": round(mb * n / (0.6 * HBM_PEAK_GBS * 1e9) * 1e3, 4)}

    def variant(steps, **kw):
        """The same cloud built `steps` times with other parameters (one warm-up)."""
        pv = lod.make_params(leaf_cap=args.leaf_cap, max_level=args.max_level, timing=True, **kw)

        def vstep():
            t = lod.lod_build(dev, params=pv, stream=stream)
            tm = t.timings()
            t.free()
            return tm

        vstep()
        torch.cuda.synchronize()
        v0 = time.perf_counter()
        vtm = [vstep() for _ in range(steps)]
        torch.cuda.synchronize()
        vms = 1e3 * (time.perf_counter() - v0) / steps
        return {"ms_per_build": round(vms, 4), "points_per_s": round(n / (vms * 1e-3), 1),
                "vs_plain": round(vms / ms_per_step, 3), "steps": steps,
                "leaf_voxels_ms": round(float(np.mean([t["leaf_voxels"] for t in vtm])), 4),
                "levels_ms": round(float(np.mean([t["levels"] for t in vtm])), 4)}

    # same cloud and parameters, plus a full-precision record (accepted
    # sample's coordinates, voxel colour) for every voxel
    full = variant(args.full_precision_steps, sampling=sampling, full_precision=True) \
        if args.full_precision_steps > 0 else None
    # the neighbourhood-weighted average on the same cloud
    weighted = variant(args.weighted_steps, sampling=3) if args.weighted_steps > 0 else None

    # the same cloud from pinned host memory, built in chunks and merged
    # (the out-of-core scheme), beside a host -> device copy plus the in-core build
    chunked = None
    if args.chunked_steps > 0:
        print(f"[bench] chunked build, {args.chunk_points} points per chunk", file=sys.stderr, flush=True)
        def cstep(pc):
            t = lod.lod_build_chunked(pts, args.chunk_points, params=pc, stream=stream)
            v = t.view()
            info = (v.num_nodes, v.num_voxels)
            t.free()
            return info

        def ctime(low_memory):
            pc = lod.make_params(leaf_cap=args.leaf_cap, max_level=args.max_level, sampling=sampling,
                                 low_memory=low_memory)
            cstep(pc)
            c0 = time.perf_counter()
            info = [cstep(pc) for _ in range(args.chunked_steps)]
            return 1e3 * (time.perf_counter() - c0) / args.chunked_steps, info[-1]

        cms, cinfo = ctime(False) if args.chunked_forms != "streaming" else (None, infos[-1])
        sms, sinfo = ctime(True) if args.chunked_forms != "resident" else (None, infos[-1])
        h0 = time.perf_counter()
        for _ in range(args.chunked_steps):
            d2 = host.to("cuda:0", non_blocking=False)
            t = lod.lod_build(d2, params=params, stream=stream)
            t.free()
            del d2
        torch.cuda.synchronize()
        hms = 1e3 * (time.perf_counter() - h0) / args.chunked_steps
        rnd = (lambda v: None if v is None else round(v, 2))
        chunked = {"chunk_points": args.chunk_points, "ms_per_build": rnd(cms),
                   "points_per_s": None if cms is None else round(n / (cms * 1e-3), 1), "steps": args.chunked_steps,
                   "in_core_from_host_ms": round(hms, 2), "same_nodes_and_voxels": cinfo == infos[-1] == sinfo,
                   "streaming_ms_per_build": rnd(sms),
                   "note": "host input: one upload that also gives the cube, each piece sorted by cell on the GPU "
                           "(its counts give the split level), chunk builds from the sorted pieces, the merge above "
                           "the chunk roots; streaming (low-memory flag): the sorted pieces kept in host memory and "
                           "chunks uploaded batch by batch"}

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(pts, min(args.cpu_sample, n), args, sampling)

    del dev
    torch.cuda.empty_cache()
    batched = served = served_small = None
    if args.batch_chunks > 0:
        batched = run_batched(lod, torch, args.batch_chunks, args.batch_reps, params_plain(lod, args, sampling))
    if args.serve_requests > 0:
        served = run_served(lod, torch, args.serve_requests, args.serve_rate, params_plain(lod, args, sampling),
                            192 << 30, 4, args.serve_tiles, 256)
    if args.serve_small_requests > 0:
        served_small = run_served(lod, torch, args.serve_small_requests, args.serve_small_rate,
                                  params_plain(lod, args, sampling), 192 << 30, 4, args.serve_tiles, 256,
                                  fixed_size=args.serve_small_points)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"plain build, {wl['desc']}", "points": n, "leaf_cap": args.leaf_cap,
                   "max_level": args.max_level, "grid": 128, "sampling": args.sampling,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages_ms": {k: round(v, 4) for k, v in avg.items()},
        "kernels": kernels,
        "whole_build_roofline": whole_roofline,
        "whole_build_stage_GBps": round(whole_alg / (ms_per_step * 1e-3) / 1e9, 1),
        "nodes": nodes,
        "voxels": voxels,
        "full_precision": full,
        "weighted": weighted,
        "chunked": chunked,
        "batched": batched,
        "served": served,
        "served_small": served_small,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
