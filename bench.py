#!/usr/bin/env python3
"""Throughput of the boundary-aware normal estimator on one MI355X.

Default workload: plain single-frame launches on 1920x1080 binary32 depth
(fx=fy=1050, principal point at the centre, alpha=2, REL mask tau=4).  To
measure HBM rather than the 256 MB last-level cache, every step processes the
next frame of a ring of distinct device buffers (>= 1 GiB of traffic per
pass).  One step = one launch of the whole per-pixel path (stencil gather,
validity, normal, boundary mask, normalisation, stores, per-frame counts)
over one frame.  The launches of one pass over the ring are captured in a
HIP graph and replayed, so that Python's per-call overhead does not starve
the GPU.

`--workload batch` runs the 256-frame mixed batch (64x 320x240, 96x 640x480,
64x 1280x720, 32x 1920x1080) as one step.

Prints one JSON line.  Also reports the FP64 CPU oracle, timed on the host
cores on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_PIXEL = 17          # 4 B depth in, 12 B normal + 1 B code out
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E, AMD published peak
# Unpacked binary32 VALU instructions: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one operation each: packed FP32 is not used, FMA contraction is off, and
# the fused multiply-adds that pair removal's sequence names are one
# instruction, so one operation, each).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def alu_ops_per_pixel(method: str, scales: int = 0) -> int:
    """Binary32 operations per pixel of the definition (products, sums,
    compares and class tests; the normalisation's reciprocal square root and
    its three products), counted on the path where every pair passes."""
    if method == "four_pair":
        return 34
    if method == "pair_removal":
        return 95
    return 16 * scales + 14   # multiscale: 16 per scale, 14 for the rest
KERNEL_SOURCES = ["bn_device.h", "bn_tiles.h", "bn_kernels.hip", "bn_batch.hip"]
ADJOINT_SOURCES = ["bn_device.h", "bn_adjoint.hip", "bn_stack.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _gen(job):
    """One host frame of the run (a process-pool job)."""
    from synth import scenes
    kind, a = job
    if kind == "1080":
        return scenes.frame_1920x1080(seed=a)
    if kind == "640":
        return scenes.frame_640x480(seed=a)
    H, W, seed = a
    return scenes.sized_frame(H, W, seed)


def generate_inputs(args) -> dict:
    """Every host frame the run uses, generated before anything touches the
    GPU: the process pool forks, and a process that has initialised HIP must
    not fork.  The pool is shut down (its workers joined) before returning."""
    import concurrent.futures as cf
    from synth import scenes
    jobs = {}
    if args.workload == "batch":
        jobs["batch"] = [("sized", (H, W, 1000 + i))
                         for i, (H, W) in enumerate(scenes.batch_shapes())]
    elif args.workload == "plain640":
        jobs["plain640"] = [("640", 1 + i) for i in range(8)]
    else:
        nd = min(args.distinct, args.ring)
        if not args.no_batch and not args.no_serve:
            # the slowest job (4096x3072) first, so the pool stays busy
            jobs["serve"] = [("sized", (H, W, 3000 + k))
                             for k, (H, W) in enumerate(scenes.SERVE_SIZES)]
        jobs["plain"] = [("1080", 2 + i) for i in range(nd)]
        if not args.no_batch:
            jobs["batch"] = [("sized", (H, W, 1000 + i))
                             for i, (H, W) in enumerate(scenes.batch_shapes())]
        if not args.quick:
            jobs["plain640"] = [("640", 1 + i) for i in range(8)]
            jobs["diff"] = [("640", 2000 + i) for i in range(16)]
    flat = [j for js in jobs.values() for j in js]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(16, int(cores or 1), len(flat)))
    kind = "threads" if getattr(args, "gen_threads", False) else "processes"
    log(f"generating {len(flat)} host frames ({', '.join(f'{k}: {len(v)}' for k, v in jobs.items())}) "
        f"on {workers} {kind}, before any GPU use")
    t0 = time.perf_counter()
    pool = cf.ThreadPoolExecutor if kind == "threads" else cf.ProcessPoolExecutor
    with pool(max_workers=workers) as ex:
        out = list(ex.map(_gen, flat, chunksize=1))
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    res, i = {}, 0
    for k, js in jobs.items():
        res[k] = out[i:i + len(js)]
        i += len(js)
    return res


def kernel_hash(sources=None) -> str:
    """The measured kernels' sources (the forward kernels' by default) and the
    flags they are compiled with."""
    from paper_2209_08241_amd.build import HIPCC_FLAGS
    h = hashlib.sha256()
    h.update(" ".join(HIPCC_FLAGS).encode())
    for name in (KERNEL_SOURCES if sources is None else sources):
        p = os.path.join(ROOT, "paper_2209_08241_amd", "csrc", name)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, launch_pixels: int, sources=None, variant=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload in this tile shape (variant name; None for kernels without
    a choice of shape), if it was taken on the current kernel sources; else
    None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("kernel_hash") != kernel_hash(sources):
        return None
    if variant and rec.get("variant") != variant:
        rec = rec.get("other_tile_shapes", {}).get(variant)
        if rec is None:
            return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(frames, alpha, mode, tau, budget_s):
    """The oracle as it stands, single thread, on frames until budget_s."""
    import oracle
    t0 = time.perf_counter()
    px = 0
    n = 0
    while True:
        s = frames[n % len(frames)]
        oracle.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, alpha, mode, tau)
        px += s.depth.size
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": px / el / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} frames ({', '.join(sorted(set(f'{f.depth.shape[1]}x{f.depth.shape[0]}' for f in frames)))}), "
                      f"{el:.1f} s, single thread, FP64 normals + binary32 mask"}


def cpu_threads(frames, alpha, mode, tau, budget_s):
    """The same oracle on every host core: each frame's rows split into one
    band per thread (ctypes releases the GIL during the call)."""
    import concurrent.futures as cf
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores or 1), 16))
    o = oracle.default()
    t0 = time.perf_counter()
    px = n = 0
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        while True:
            s = frames[n % len(frames)]
            H = s.depth.shape[0]
            bands = [(H * k // cores, H * (k + 1) // cores) for k in range(cores)]
            list(ex.map(lambda b: o.normals_f32_rows(s.depth, s.fx, s.fy, s.cx, s.cy, alpha,
                                                     mode, tau, b[0], b[1]), bands))
            px += s.depth.size
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    return {"value": px / el / 1e6, "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} frames, {el:.1f} s, rows split over {cores} threads"}


class Ring:
    """A ring of distinct device frame buffers, one plain launch per step."""

    def __init__(self, torch, bn, scs, ring):
        dev = torch.device("cuda:0")
        H, W = scs[0].depth.shape
        self.torch, self.bn, self.scs, self.ring = torch, bn, scs, ring
        self.H, self.W = H, W
        self.depth = [torch.from_numpy(scs[i % len(scs)].depth).to(dev) for i in range(ring)]
        self.normals = [torch.empty((H, W, 3), dtype=torch.float32, device=dev)
                        for _ in range(ring)]
        self.masks = [torch.empty((H, W), dtype=torch.uint8, device=dev) for _ in range(ring)]
        self.stats = bn.new_stats(ring, device=dev)

    def launch(self, i, kw, stream=None):
        j = i % self.ring
        s0 = self.scs[0]
        self.bn.estimate_normals(self.depth[j], s0.fx, s0.fy, s0.cx, s0.cy,
                                 normals=self.normals[j], mask=self.masks[j],
                                 stats=self.stats[j], stream=stream, **kw)

    def time(self, kw, steps, warmup, eager=False, hot=False, min_passes=10):
        """ms per launch over `steps` launches (graph replay of one pass over
        the ring unless eager; hot: the same buffer every launch).  A graph
        run times whole passes over the ring, at least min_passes of them, so
        that the timed window spans milliseconds whatever `steps` asks."""
        torch = self.torch
        ring = 1 if hot else self.ring
        stream = torch.cuda.Stream()
        graph = None
        if not eager:
            with torch.cuda.stream(stream):
                for i in range(ring):
                    self.launch(i, kw, stream)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                for i in range(ring):
                    self.launch(i, kw, torch.cuda.current_stream())
            torch.cuda.synchronize()
            steps = max(-(-steps // ring), min_passes) * ring
            warmup = max(-(-warmup // ring), 1) * ring

        def run(n):
            if graph is not None:
                for _ in range(n // ring):
                    graph.replay()
            else:
                for i in range(n):
                    self.launch(i % ring, kw, stream)

        with torch.cuda.stream(stream):
            run(warmup)
        torch.cuda.synchronize()
        self.stats.fill_(-1)   # every launch stores its frame's counts over this
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            start.record(stream)
            run(steps)
            end.record(stream)
        end.synchronize()
        torch.cuda.synchronize()
        return start.elapsed_time(end) / steps, steps, warmup, graph is not None

    def single_launch_us(self, kw, reps=30):
        """Latency of one eager launch, synchronised, median of reps."""
        import numpy as np
        torch = self.torch
        stream = torch.cuda.Stream()
        out = []
        for r in range(reps + 3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                self.launch(r, kw, stream)
            stream.synchronize()
            out.append(time.perf_counter() - t0)
        return 1e6 * float(np.median(out[3:]))


def parity_check(ring, kw, alpha, mode, tau, method="four_pair", scales=0):
    """The benchmarked configuration against the oracle on frame 0."""
    import numpy as np
    import oracle
    torch = ring.torch
    ring.launch(0, kw)
    torch.cuda.synchronize()
    s0 = ring.scs[0]
    ref = oracle.variant_f32(s0.depth, s0.fx, s0.fy, s0.cx, s0.cy, alpha, mode, tau,
                             method=method, scales=scales)
    ok_mask = bool(np.array_equal(ring.masks[0].cpu().numpy(), ref["mask"]))
    err = float(np.abs(ring.normals[0].cpu().numpy().astype(np.float64) - ref["normals"]).max())
    log(f"parity frame 0 ({method}): mask equal={ok_mask}, max normal error={err:.2e}")
    if not ok_mask or err > 1e-5:
        raise SystemExit(f"benchmark configuration ({method}) disagrees with the oracle")
    return ref


def roofline(px, ms, traffic=None):
    achieved = BYTES_PER_PIXEL * px / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}


def alu_roofline(px, ms, ops_per_pixel):
    """The same launch against the vector ALUs: algorithmic operations per
    second over the unpacked binary32 issue rate."""
    achieved = ops_per_pixel * px / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
            "frac": achieved / ALU_PEAK_TOPS, "ops_per_pixel": ops_per_pixel}


def roofline_from_rate(mpix_s):
    """HBM roofline of a pixel rate (17 algorithmic bytes per pixel)."""
    achieved = BYTES_PER_PIXEL * mpix_s * 1e6 / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}


def achievable_rates(torch, bn, reps=5):
    """HBM rates of plain streaming kernels on this GPU: torch's device copy,
    the library's 16-byte non-temporal copy (2 GiB moved each), and the
    estimator's traffic shape without its arithmetic (168 Mpixel)."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            fn()
        end.record()
        end.synchronize()
        return start.elapsed_time(end) / reps
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"torch_copy_GBs": 2 * n * 4 / (timed(lambda: dst.copy_(src)) * 1e-3) / 1e9,
           "stream_copy_GBs": 2 * n * 4 / (timed(lambda: bn.stream_copy(dst, src)) * 1e-3) / 1e9}
    del src, dst
    px = 160 << 20
    depth = torch.ones(px, dtype=torch.float32, device="cuda")
    normals = torch.empty(3 * px, dtype=torch.float32, device="cuda")
    mask = torch.empty(px, dtype=torch.uint8, device="cuda")
    ms = timed(lambda: bn.stream_pattern(depth, normals, mask))
    out["pattern_GBs"] = BYTES_PER_PIXEL * px / (ms * 1e-3) / 1e9
    out["what"] = ("GB/s of read + write bytes: torch copy_ and bn_stream_copy of 1 GiB; "
                   "bn_stream_pattern = 4 B in + 13 B out per pixel through the kernels' LDS "
                   "staging, no arithmetic, 168 Mpixel; valu_tops: bn_alu_probe, unpacked "
                   "binary32 multiplies per second (8192 workgroups x 256 threads x 8 "
                   "independent chains x 4096 steps)")
    del depth, normals, mask
    acc = torch.empty(8192 * 256, dtype=torch.float32, device="cuda")
    lane_ops = 8192 * 256 * 8 * 4096
    out["valu_tops"] = lane_ops / (timed(lambda: bn.alu_probe(acc, 4096)) * 1e-3) / 1e12
    out["valu_peak_tops"] = ALU_PEAK_TOPS
    del acc
    torch.cuda.empty_cache()
    return out


def graph_ring_ms(torch, launch, n, passes=10):
    """ms per call of launch(i, stream), i = 0..n-1, captured in one graph and
    replayed `passes` times after one untimed replay."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for i in range(n):
            launch(i, stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for i in range(n):
            launch(i, torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        graph.replay()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(passes):
            graph.replay()
        end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / (passes * n)


def launch_breakdown(torch, bn, ring, kw):
    """Per-launch times on the same graph-replayed ring: the launch floor (a
    16-byte device copy), the estimator's traffic shape without arithmetic
    or counts, and the estimator without its counts."""
    dev = ring.depth[0].device
    n = ring.ring
    a16 = [torch.empty(4, device=dev) for _ in range(n)]
    b16 = [torch.zeros(4, device=dev) for _ in range(n)]
    s0 = ring.scs[0]
    return {
        "launch_floor_us": 1e3 * graph_ring_ms(
            torch, lambda i, st: bn.stream_copy(a16[i], b16[i], stream=st), n),
        "traffic_pattern_us": 1e3 * graph_ring_ms(
            torch, lambda i, st: bn.stream_pattern(ring.depth[i], ring.normals[i], ring.masks[i],
                                                   stream=st), n),
        "without_counts_us": 1e3 * graph_ring_ms(
            torch, lambda i, st: bn.estimate_normals(ring.depth[i], s0.fx, s0.fy, s0.cx, s0.cy,
                                                     normals=ring.normals[i], mask=ring.masks[i],
                                                     want_stats=False, stream=st, **kw), n),
        "what": ("per launch, graph-replayed over the same ring: a 16-byte bn_stream_copy (the "
                 "launch floor), bn_stream_pattern on the frame buffers (4 B in, 13 B out per "
                 "pixel through the same LDS staging and stores, no arithmetic, no counts), the "
                 "estimator without its counts; us_per_frame is the estimator with them"),
    }


def run_plain640(args, torch, bn, inputs):
    """The small plain configuration: 640x480, a ring of 256 buffers (1.6 GB,
    beyond the last-level cache), one launch per frame, the autotuner's tile
    shape."""
    scs640 = inputs["plain640"]
    r640 = Ring(torch, bn, scs640, 256)
    if args.variant:
        v640, from640 = args.variant, "--variant"
    elif args.no_autotune:
        v640, from640 = bn.default_variant(480, 640, "four_pair", args.alpha, 0), "library default"
    else:
        v640 = bn.autotune_plain(480, 640, args.alpha, args.mode, args.tau)[0]
        from640 = "autotuner"
    # variant 0 takes the autotuner's entry for this size when there is one
    kw640 = dict(alpha=args.alpha, mode=args.mode, tau=args.tau, variant=args.variant)
    parity_check(r640, kw640, args.alpha, args.mode, args.tau)
    ms640, steps640, warm640, _ = r640.time(kw640, 2560, 256)
    px640 = 640 * 480
    log(f"plain 640x480: {ms640 * 1e3:.2f} us per frame")
    brk = launch_breakdown(torch, bn, r640, kw640)
    log(f"plain 640x480 breakdown: floor {brk['launch_floor_us']:.2f} us, traffic pattern "
        f"{brk['traffic_pattern_us']:.2f} us, without counts {brk['without_counts_us']:.2f} us")
    del r640
    name640 = dict(bn.variants())[v640]
    return {"workload": "plain 640x480, one launch per frame, ring of 256 buffers (8 distinct "
                        "scenes, seeds 1..8)",
            "value": px640 / (ms640 * 1e-3) / 1e6, "unit": "Mpix/s", "ms_per_step": ms640,
            "us_per_frame": ms640 * 1e3, "steps": steps640, "warmup": warm640,
            "variant": name640,
            "variant_from": from640,
            "launch_breakdown": brk,
            "roofline": roofline(px640, ms640, load_traffic("plain640", px640,
                                                            variant=name640))}


def run_plain(args, torch, bn, inputs):
    ring_n = args.ring
    scs = inputs["plain"]
    ndistinct = len(scs)
    ring = Ring(torch, bn, scs, ring_n)
    H, W = ring.H, ring.W
    px = H * W
    tuned = None
    if args.variant == 0 and not args.no_autotune:
        # the autotuner's choice of tile shape for this frame size, taken by
        # variant 0 (the library's choice) from here on
        tv, tus = bn.autotune_plain(H, W, args.alpha, args.mode, args.tau)
        tuned = {"variant": dict(bn.variants())[tv], "autotune_us": tus}
        log(f"autotuned plain {W}x{H}: {tuned['variant']} ({tus:.2f} us in its own ring)")
    kw = dict(alpha=args.alpha, mode=args.mode, tau=args.tau, variant=args.variant)
    ref = parity_check(ring, kw, args.alpha, args.mode, args.tau)
    ms_step, steps, warm, graphed = ring.time(kw, args.steps, args.warmup, eager=args.eager)
    st = ring.stats.cpu().numpy()
    want = [int(c) for c in ref["counts"]] + [0]
    if st[0].tolist() != want:
        raise SystemExit(f"per-frame counts wrong after timing: {st[0].tolist()} != {want}")
    used = (tuned["variant"] if tuned else
            dict(bn.variants())[args.variant or
                                bn.default_variant(H, W, "four_pair", args.alpha, 0)])
    traffic = load_traffic("plain1080", px, variant=used)
    extra = {}
    if not args.quick:
        hot_ms, _, _, _ = ring.time(kw, args.steps // 4, args.warmup // 4, hot=True,
                                    min_passes=100)
        extra["hot_cache"] = {"value": px / (hot_ms * 1e-3) / 1e6, "unit": "Mpix/s",
                              "note": "one frame buffer relaunched: the 256 MB last-level "
                                      "cache holds it, not an HBM figure"}
        extra["single_launch_us"] = ring.single_launch_us(kw)
        extra["launch_breakdown"] = launch_breakdown(torch, bn, ring, kw)
        log("plain {}x{} breakdown: floor {:.2f} us, traffic pattern {:.2f} us, without counts "
            "{:.2f} us".format(W, H, *(extra["launch_breakdown"][k] for k in
                                       ("launch_floor_us", "traffic_pattern_us",
                                        "without_counts_us"))))
        methods = []
        for name, alpha, K in (("pair_removal", args.alpha, 0), ("multiscale", 1, 3),
                               ("multiscale", 3, 3)):
            mkw = dict(alpha=alpha, mode=args.mode, tau=args.tau, method=name, scales=K)
            mv = (bn.autotune_plain(H, W, alpha, args.mode, args.tau, method=name, scales=K)[0]
                  if not args.no_autotune else bn.default_variant(H, W, name, alpha, K))
            parity_check(ring, mkw, alpha, args.mode, args.tau, name, K)
            mms, msteps, _, _ = ring.time(mkw, args.steps // 2, args.warmup // 2, min_passes=5)
            methods.append({"method": name, "alpha": alpha, "scales": K, "steps": msteps,
                            "variant": dict(bn.variants())[mv],
                            "roofline_traffic_workload": f"{name}_a{alpha}_k{K}_1080",
                            "ms_per_step": mms, "value": px / (mms * 1e-3) / 1e6,
                            "unit": "Mpix/s",
                            "roofline": roofline(px, mms,
                                                 load_traffic(f"{name}_a{alpha}_k{K}_1080", px,
                                                              variant=dict(bn.variants())[mv])),
                            "alu_roofline": alu_roofline(px, mms, alu_ops_per_pixel(name, K))})
            log(f"{name}: {methods[-1]['value']:.0f} Mpix/s")
        extra["methods"] = methods
        extra["plain640"] = run_plain640(args, torch, bn, inputs)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle for {args.cpu_seconds} s (one thread)")
        cpu = cpu_baseline(scs, args.alpha, args.mode, args.tau, args.cpu_seconds)
        if not args.quick:
            log(f"timing the oracle for {args.cpu_seconds} s (all host cores)")
            extra["cpu_oracle_all_cores"] = cpu_threads(scs, args.alpha, args.mode, args.tau,
                                                        args.cpu_seconds)
    out = {
        "metric": "normals Mpix/s (plain single-frame launches)",
        "value": px / (ms_step * 1e-3) / 1e6,
        "unit": "Mpix/s",
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms_step,
        "config": {"workload": "plain 1920x1080, one launch per frame, ring of "
                               f"{ring_n} frame buffers ({ndistinct} distinct scenes)",
                   "frame": "1920x1080", "fx": 1050.0, "alpha": args.alpha,
                   "mask": args.mode, "tau": args.tau, "method": "four_pair",
                   "launch": "hip graph replay" if graphed else "eager",
                   "variant": used,
                   "variant_from": ("autotuner" if tuned else "--variant" if args.variant
                                    else "library default")},
        "roofline": roofline(px, ms_step, traffic),
        "alu_roofline": alu_roofline(px, ms_step, alu_ops_per_pixel("four_pair")),
        "cpu_baseline": cpu,
    }
    out.update(extra)
    return out


def run_batch(args, torch, bn, inputs):
    """The 256-frame mixed batch, one graph launch over all tiles per step."""
    frames_h = inputs["batch"]
    dev = torch.device("cuda:0")
    frames = [bn.BatchFrame(torch.from_numpy(s.depth).to(dev), s.fx, s.fy, s.cx, s.cy)
              for s in frames_h]
    plan = bn.BatchPlan(frames, alpha=args.alpha, mode=args.mode, tau=args.tau)
    stream = torch.cuda.Stream()
    # the autotuner's grid shape for this plan (it runs the plan to time it)
    shape, shape_us = plan.autotune(stream) if not args.no_autotune else (0, 0.0)
    shape_name = ("flat, 1 tile per workgroup" if shape == 0 else
                  f"flat, {-shape} tiles per workgroup" if shape < 0 else
                  f"{shape} persistent workgroups per CU")
    log(f"autotuned batch grid: {shape_name} ({shape_us:.1f} us)")
    info = plan.info()
    px = info["pixels"]
    with torch.cuda.stream(stream):
        for _ in range(max(args.batch_warmup, 1)):
            plan.run(stream)
    torch.cuda.synchronize()
    # correctness of the benchmarked configuration: a sample of frames
    import numpy as np
    import oracle
    for k in (0, 100, 200, 255):
        s, fr = frames_h[k], frames[k]
        ref = oracle.normals_f32(s.depth, s.fx, s.fy, s.cx, s.cy, args.alpha, args.mode, args.tau)
        ok = bool(np.array_equal(fr.mask.cpu().numpy(), ref["mask"]))
        err = float(np.abs(fr.normals.cpu().numpy().astype(np.float64) - ref["normals"]).max())
        if not ok or err > 1e-5:
            raise SystemExit(f"batched frame {k} disagrees with the oracle")
    log("batched parity sample ok")
    for fr in frames:
        fr.stats.fill_(-1)   # every run stores each frame's counts over this
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    steps = args.batch_steps
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(steps):
            plan.run(stream)
        end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end) / steps
    ref0 = oracle.normals_f32(frames_h[0].depth, frames_h[0].fx, frames_h[0].fy,
                              frames_h[0].cx, frames_h[0].cy, args.alpha, args.mode, args.tau)
    got0 = frames[0].stats.cpu().tolist()
    if got0 != [int(c) for c in ref0["counts"]] + [0]:
        raise SystemExit("batched counts wrong after timing")
    plan.close()
    plain = None
    if not args.quick:
        plain = plain_launches(args, torch, bn, frames, stream, px)
    return {
        "workload": "256 frames: 64x 320x240, 96x 640x480, 64x 1280x720, 32x 1920x1080 "
                    "(seeds 1000..1255, fx=fy=525*W/640), one graph launch over all tiles",
        "pixels": px, "tiles": info["tiles"], "workgroups": info["workgroups"],
        "grid_shape": shape_name,
        "grid_shape_from": "library default" if args.no_autotune else "autotuner",
        "value": px / (ms * 1e-3) / 1e6, "unit": "Mpix/s", "ms_per_step": ms, "steps": steps,
        "roofline": roofline(px, ms, load_traffic("batch256", px)),
        "same_frames_plain_launches": plain,
    }


def plain_launches(args, torch, bn, frames, stream, px):
    """The same 256 frames as 256 bn_estimate_normals launches on one stream:
    eager (one host call per frame) and replayed from a HIP graph."""
    kw = dict(alpha=args.alpha, mode=args.mode, tau=args.tau)

    def one_pass(st):
        for fr in frames:
            bn.estimate_normals(fr.depth, fr.fx, fr.fy, fr.cx, fr.cy, normals=fr.normals,
                                mask=fr.mask, stats=fr.stats, stream=st, **kw)

    res = {}
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    reps = max(args.batch_steps // 10, 3)
    with torch.cuda.stream(stream):
        one_pass(stream)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(reps):
            one_pass(stream)
        end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end) / reps
    res["eager"] = {"value": px / (ms * 1e-3) / 1e6, "unit": "Mpix/s", "ms_per_pass": ms,
                    "roofline_frac": roofline(px, ms)["frac"]}
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        one_pass(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        graph.replay()
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(reps):
            graph.replay()
        end.record(stream)
    end.synchronize()
    ms = start.elapsed_time(end) / reps
    res["graph"] = {"value": px / (ms * 1e-3) / 1e6, "unit": "Mpix/s", "ms_per_pass": ms,
                    "roofline_frac": roofline(px, ms)["frac"]}
    log(f"same frames as plain launches: eager {res['eager']['value']:.0f}, "
        f"graph {res['graph']['value']:.0f} Mpix/s")
    del graph
    return res


SETS = 6   # buffer sets the differentiation timings cycle over


def run_diff(args, torch, bn, inputs):
    """Differentiation: 16 x 640x480 frames (seeds 2000..2015) as one stack.
    The adjoint kernel over the stack (one launch), the forward over the
    stack, the adjoint as 16 single-frame launches for comparison, and one
    full step (forward, cosine loss against the normals of the noise-free
    depth, backward through the adjoint)."""
    import numpy as np
    import oracle
    scs = inputs["diff"]
    dev = torch.device("cuda:0")
    n, H, W = len(scs), 480, 640
    px = H * W
    intr = [(s.fx, s.fy, s.cx, s.cy) for s in scs]
    depth = torch.from_numpy(np.stack([s.depth for s in scs])).to(dev)
    clean = torch.from_numpy(np.stack([s.depth_clean for s in scs]).astype(np.float32)).to(dev)
    kw = dict(alpha=args.alpha, mode=args.mode, tau=args.tau)
    t_n, t_m, _ = bn.estimate_normals_stack(clean, intr, want_stats=False, **kw)
    gen = torch.Generator(device=dev).manual_seed(5)
    grads = torch.randn((n, H, W, 3), device=dev, generator=gen)
    gd = torch.empty((n, H, W), device=dev)
    # the benchmarked adjoint against the oracle's on frame 0 (codes frozen)
    s0 = scs[0]
    bn.normals_vjp_stack(depth, intr, grads, grad_depth=gd, **kw)
    torch.cuda.synchronize()
    codes = oracle.normals_f32(s0.depth, s0.fx, s0.fy, s0.cx, s0.cy, args.alpha, args.mode,
                               args.tau)["mask"]
    ref = oracle.normals_vjp_f64(s0.depth.astype(np.float64), s0.fx, s0.fy, s0.cx, s0.cy,
                                 args.alpha, codes, grads[0].cpu().numpy().astype(np.float64))
    got = gd[0].cpu().numpy().astype(np.float64)
    scale = np.abs(ref).max()
    if not np.all(np.abs(got - ref) <= 1e-4 * scale + 1e-3 * np.abs(ref)):
        raise SystemExit("benchmarked adjoint disagrees with the oracle")
    log("adjoint parity frame 0 ok")
    stream = torch.cuda.Stream()

    def timed_graph(fn, reps=20, calls=2 * SETS):
        """us per call of fn(stream, buffer set): `calls` calls captured in
        one graph, cycling over the buffer sets, replayed back to back (one
        call per graph would time the graph launch as well)."""
        with torch.cuda.stream(stream):
            fn(stream, 0)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for c in range(calls):
                fn(torch.cuda.current_stream(), c % SETS)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            start.record(stream)
            for _ in range(reps):
                g.replay()
            end.record(stream)
        end.synchronize()
        return start.elapsed_time(end) * 1e3 / (reps * calls)

    adj_bytes = 20                      # depth 4 B + cotangent 12 B in, gradient 4 B out
    fwd_bytes = 17                      # depth 4 B in, normal 12 B + code 1 B out
    # SETS copies of every buffer (160 MB a set), used in turn, so that the
    # 256 MB last-level cache cannot hold what a call reads and writes
    D = [depth] + [depth.clone() for _ in range(SETS - 1)]
    G = [grads] + [grads.clone() for _ in range(SETS - 1)]
    GD = [gd] + [torch.empty_like(gd) for _ in range(SETS - 1)]
    NRM = [torch.empty((n, H, W, 3), device=dev) for _ in range(SETS)]
    MSK = [torch.empty((n, H, W), dtype=torch.uint8, device=dev) for _ in range(SETS)]
    us_adj = timed_graph(lambda st, i: bn.normals_vjp_stack(D[i], intr, G[i], grad_depth=GD[i],
                                                            stream=st, **kw))
    us_fwd = timed_graph(lambda st, i: bn.estimate_normals_stack(D[i], intr, normals=NRM[i],
                                                                 mask=MSK[i], want_stats=False,
                                                                 stream=st, **kw))

    def per_frame(st, i):
        for k, s in enumerate(scs):
            bn.normals_vjp(D[i][k], s.fx, s.fy, s.cx, s.cy, G[i][k], grad_depth=GD[i][k],
                           stream=st, **kw)

    us_adj_frames = timed_graph(per_frame, reps=5)

    def rl(bpp, us, traffic=None):
        a = bpp * n * px / (us * 1e-6) / 1e9
        return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": a / HBM_PEAK_GBS, "bytes_per_pixel": bpp, "traffic": traffic}

    def step():
        x = depth.clone().requires_grad_(True)
        nn_, mm = bn.normals_with_grad_stack(x, intr, **kw)
        loss = bn.cosine_loss(nn_, t_n, mm, t_m)
        loss.backward()
        return loss.detach()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nstep = 20
    for _ in range(nstep):
        last = step()
    float(last)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / nstep
    log(f"stack of 16: adjoint {us_adj:.1f} us, forward {us_fwd:.1f} us, 16 single-frame "
        f"adjoints {us_adj_frames:.1f} us; step {ms_step:.3f} ms")
    return {"workload": "16 x 640x480 (seeds 2000..2015) as one stack [16, 480, 640] with "
                        "per-frame intrinsics; kernels graph-replayed, 12 calls a graph over "
                        f"{SETS} distinct sets of buffers; full step = stacked "
                        "forward + cosine loss vs the noise-free depth's normals + stacked "
                        "backward, eager, one host synchronisation per step",
            "adjoint_us_per_stack": us_adj, "adjoint_us_per_frame": us_adj / n,
            "adjoint_mpix_s": n * px / us_adj,
            "adjoint_roofline": rl(adj_bytes, us_adj,
                                   load_traffic("adjoint_stack16", n * px, ADJOINT_SOURCES)),
            "forward_us_per_stack": us_fwd, "forward_mpix_s": n * px / us_fwd,
            "forward_roofline": rl(fwd_bytes, us_fwd),
            "adjoint_single_frame_launches_us": us_adj_frames,
            "step_ms": ms_step, "step_mpix_s": n * px / (ms_step * 1e3)}


class _PoolFrame:
    """A device depth frame offered to the server (no outputs of its own)."""

    def __init__(self, depth, fx, fy, cx, cy):
        self.depth, self.fx, self.fy, self.cx, self.cy = depth, fx, fy, cx, cy

    def _c(self):
        import paper_2209_08241_amd as bn
        H, W = self.depth.shape
        return bn.Frame(self.depth.data_ptr(), H, W, self.depth.stride(0), self.fx, self.fy,
                        self.cx, self.cy, 0, 0, 0)


def run_serve(args, torch, bn, inputs, capacity_mpix_s):
    """Poisson request streams over the serving sizes at fractions of the
    batched capacity measured in the same run; device-resident inputs."""
    import numpy as np
    frames_h = inputs["serve"]
    # 16 device copies of each frame, each depth scaled by its own factor in
    # [0.98, 1.02], so that requests read 1 GB of distinct depth (more than
    # the 256 MB last-level cache holds); outputs live in the server's slots
    gen = torch.Generator(device="cuda").manual_seed(3000)
    pool = []
    for s in frames_h:
        d = torch.from_numpy(s.depth).cuda()
        for _ in range(16):
            f = 1.0 + 0.02 * (2.0 * float(torch.rand((), device="cuda", generator=gen)) - 1.0)
            pool.append(_PoolFrame(d * f, s.fx, s.fy, s.cx, s.cy))
    mean_px = float(np.mean([s.depth.size for s in frames_h]))
    cap_hz = capacity_mpix_s * 1e6 / mean_px
    out = []
    with bn.Server(args.serve_budget_gib << 30, max_batch=args.serve_max_batch,
                   max_batches_in_flight=args.serve_in_flight, alpha=args.alpha, mode=args.mode,
                   tau=args.tau) as srv:
        srv.run_poisson(pool, cap_hz * 0.3, 2000, seed=2999)      # warm-up
        for load in (0.5, 0.9):
            rate = cap_hz * load
            r = srv.run_poisson(pool, rate, args.serve_requests, seed=3000)
            lat = r["latency_s"]
            st = srv.stats()
            out.append({"load": load, "rate_hz": rate, "requests": args.serve_requests,
                        "p50_us": 1e6 * float(np.median(lat)),
                        "p99_us": 1e6 * float(np.quantile(lat, 0.99)),
                        "mean_us": 1e6 * float(np.mean(lat)),
                        "mpix_s": r["pixels"] / r["wall_s"] / 1e6,
                        "launches_total": st["batches"], "largest_launch": st["max_batch_seen"]})
            log(f"serve load {load}: {rate:.0f} req/s p50 {out[-1]['p50_us']:.0f} us "
                f"p99 {out[-1]['p99_us']:.0f} us")
        # saturation: every request arrives at once, so the scheduler always
        # has a backlog and the served rate is the server's capacity
        b0 = srv.stats()["batches"]
        r = srv.run_poisson(pool, 1e12, args.serve_requests // 4, seed=3100)
        mpix = r["pixels"] / r["wall_s"] / 1e6
        launches = srv.stats()["batches"] - b0
        sat = {"requests": args.serve_requests // 4, "mpix_s": mpix,
               "roofline": roofline_from_rate(mpix), "launches": launches,
               "mean_batch": (args.serve_requests // 4) / max(launches, 1)}
        log(f"serve saturated: {mpix:.0f} Mpix/s ({sat['roofline']['frac']:.1%} of HBM), "
            f"{sat['mean_batch']:.1f} requests per launch")
    return {"workload": "Poisson arrivals, sizes uniform over 320x240, 640x480, 1280x720, "
                        "1920x1080, 4096x3072 (fx=525*W/640, seeds 3000..3004; 16 depth-scaled "
                        "device copies of each, 1 GB of distinct input), device-resident "
                        "inputs, continuous batching, HBM budget "
                        f"{args.serve_budget_gib} GiB",
            "mean_request_mpix": mean_px / 1e6, "capacity_req_s": cap_hz, "rates": out,
            "saturated": sat}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3200)
    ap.add_argument("--warmup", type=int, default=320)
    ap.add_argument("--workload", default="plain1080", choices=["plain1080", "batch", "plain640"])
    ap.add_argument("--no-batch", action="store_true", help="skip the batched comparison")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-warmup", type=int, default=10)
    ap.add_argument("--ring", type=int, default=32)
    ap.add_argument("--distinct", type=int, default=8)
    ap.add_argument("--alpha", type=int, default=2)
    ap.add_argument("--mode", default="rel")
    ap.add_argument("--tau", type=float, default=4.0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--eager", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    ap.add_argument("--serve-max-batch", type=int, default=16,
                    help="requests per launch (16 = the small-list limit: one kernel per launch)")
    ap.add_argument("--serve-in-flight", type=int, default=2)
    ap.add_argument("--quick", action="store_true",
                    help="headline numbers only (no methods, latency, copy or multi-core oracle)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="the library's default tile and grid shapes (for runs under a profiler, "
                         "whose per-dispatch overhead would decide the autotuner's timings)")
    ap.add_argument("--gen-threads", action="store_true",
                    help="generate the host frames on threads instead of processes (for runs "
                         "under a profiler, which may initialise the GPU before the program "
                         "starts: nothing may fork then)")
    ap.add_argument("--calibration-mib", type=int, default=0,
                    help="first run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # host frames first: nothing below this line may fork
    inputs = generate_inputs(args)

    import torch
    import paper_2209_08241_amd as bn

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    bn.lib()
    if args.calibration_mib:
        n = args.calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "plain640":
        p = run_plain640(args, torch, bn, inputs)
        out = {"metric": "normals Mpix/s (plain single-frame launches)", "value": p["value"],
               "unit": "Mpix/s", "steps": p["steps"], "warmup": p["warmup"],
               "ms_per_step": p["ms_per_step"],
               "config": {"workload": p["workload"], "frame": "640x480", "fx": 525.0,
                          "alpha": args.alpha, "mask": args.mode, "tau": args.tau,
                          "variant": p["variant"], "variant_from": p["variant_from"]},
               "roofline": p["roofline"], "launch_breakdown": p["launch_breakdown"],
               "cpu_baseline": None}
    elif args.workload == "batch":
        b = run_batch(args, torch, bn, inputs)
        out = {"metric": "normals Mpix/s (batched launch)", "value": b["value"],
               "unit": "Mpix/s", "steps": b["steps"], "warmup": args.batch_warmup,
               "ms_per_step": b["ms_per_step"],
               "config": {"workload": b["workload"], "alpha": args.alpha, "mask": args.mode,
                          "tau": args.tau, "pixels": b["pixels"]},
               "roofline": b["roofline"], "cpu_baseline": None}
        if not args.no_cpu_baseline:
            sample = [inputs["batch"][i] for i in (0, 64, 160, 224)]
            out["cpu_baseline"] = cpu_baseline(sample, args.alpha, args.mode, args.tau,
                                               args.cpu_seconds)
    else:
        out = run_plain(args, torch, bn, inputs)
        if not args.no_batch:
            b = run_batch(args, torch, bn, inputs)
            out["batched"] = {k: b[k] for k in ("workload", "value", "unit", "ms_per_step",
                                                "steps", "pixels", "tiles", "workgroups",
                                                "grid_shape", "grid_shape_from", "roofline",
                                                "same_frames_plain_launches")}
            if not args.no_serve:
                out["serving"] = run_serve(args, torch, bn, inputs, b["value"])
        if not args.quick:
            out["differentiation"] = run_diff(args, torch, bn, inputs)
    line = {
        "metric": out["metric"],
        "value": out["value"],
        "unit": out["unit"],
        "n_gpus": 1,
        "steps": out["steps"],
        "warmup": out["warmup"],
        "ms_per_step": out["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": out["config"],
        "roofline": out["roofline"],
        "cpu_baseline": out["cpu_baseline"],
    }
    if not args.quick and args.workload == "plain1080":
        ach = achievable_rates(torch, bn)
        ach["plain_frac_of_pattern"] = out["roofline"]["achieved"] / ach["pattern_GBs"]
        if "batched" in out:
            ach["batched_frac_of_pattern"] = (out["batched"]["roofline"]["achieved"]
                                              / ach["pattern_GBs"])
        line["achievable"] = ach
    for k in ("alu_roofline", "launch_breakdown", "batched", "serving", "differentiation",
              "methods", "hot_cache", "plain640", "single_launch_us", "cpu_oracle_all_cores"):
        if k in out:
            line[k] = out[k]
    import multiprocessing
    left = multiprocessing.active_children()
    if left:
        log(f"child processes still alive at the end: {[c.pid for c in left]}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
