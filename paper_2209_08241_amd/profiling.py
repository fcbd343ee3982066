"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2209_08241_amd.profiling trace  <kernel_stats.csv> <out.md> [--cmd "..."]
    python -m paper_2209_08241_amd.profiling traffic --fetch <dir> --write <dir> \
        --kernel <substring> --pixels <per launch> --workload <name> --out <json> [--cmd "..."]
    python -m paper_2209_08241_amd.profiling launches [--reps N]
    python -m paper_2209_08241_amd.profiling rings [--reps N] [--calibration-mib M]
    python -m paper_2209_08241_amd.profiling diff [--reps N] [--calibration-mib M]
    python -m paper_2209_08241_amd.profiling valu <counter_collection dir> <out.md> [--cmd "..."]

`trace` turns a `--kernel-trace --stats` kernel_stats.csv into a short table.
`launches` runs each kernel of interest N times on synthetic frames (a
program for counter passes); `valu` tabulates a pass of VALU counters over it.
`diff` runs the stacked forward and adjoint on 16 x 640x480 over six distinct
buffer sets in turn (as bench.py times them), after a calibration copy.
`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into HBM bytes
per launch of one kernel.  Each counter is calibrated against the copy
kernel that bench.py runs first (`--calibration-mib`): its bytes read and
written are known exactly, so the factor is known bytes / counter reading.
The record carries the hash of the kernel sources it was measured on;
bench.py reports it only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _csv_rows(path_or_dir: str, pattern: str):
    if os.path.isdir(path_or_dir):
        files = glob.glob(os.path.join(path_or_dir, "**", pattern), recursive=True)
    else:
        files = [path_or_dir]
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def trace_summary(stats_csv: str, out_md: str, cmd: str = "") -> str:
    """The kernel statistics of a rocprofv3 run, with each kernel's median
    duration from the kernel trace beside them when the trace is there."""
    rows = _csv_rows(stats_csv, "*kernel_stats.csv")
    base = stats_csv if os.path.isdir(stats_csv) else os.path.dirname(stats_csv)
    med: dict = {}
    if glob.glob(os.path.join(base, "*kernel_trace.csv")):
        for r in _csv_rows(base, "*kernel_trace.csv"):
            med.setdefault(r["Kernel_Name"], []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# rocprofv3 kernel statistics", ""]
    if cmd:
        lines += ["Command:", "", "```", cmd, "```", ""]
    lines += ["| kernel | calls | avg us | median us | min us | max us | share % |",
              "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"] if len(r["Name"]) <= 160 else r["Name"][:100] + " ..."
        m = f"{statistics.median(med[r['Name']]):.3f}" if r["Name"] in med else ""
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.3f} | {m} | "
                     f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | "
                     f"{float(r['Percentage']):.2f} |")
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as fh:
        fh.write(text)
    return text


def trace_by_grid(trace_dir: str, out_md: str, cmd: str = "", pixels=None) -> str:
    """Per (kernel, grid size) durations of the library's kernels from a
    rocprofv3 kernel trace: one kernel run on frames of several sizes, or in
    several tile shapes, shows up as separate rows.  `pixels` maps a grid
    size (threads) to the pixels one launch covers, for the Mpix/s and
    GB/s columns (17 algorithmic bytes per pixel)."""
    rows = _csv_rows(trace_dir, "*kernel_trace.csv")
    agg: dict = {}
    meta: dict = {}
    for r in rows:
        k = r["Kernel_Name"]
        if "bn::" not in k:
            continue
        short = k.replace("(anonymous namespace)::", "").split("(")[0]
        short = short.replace("void ", "").replace("bn::", "")
        key = (short, int(r["Grid_Size_X"]))
        agg.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        meta[key] = (r["Workgroup_Size_X"], r["VGPR_Count"], r["LDS_Block_Size"])
    lines = ["# rocprofv3 kernel trace by kernel and grid size", ""]
    if cmd:
        lines += ["Command:", "", "```", cmd, "```", ""]
    lines += ["Durations between each dispatch's start and end timestamps, per kernel and "
              "grid size (threads).", "",
              "| kernel | grid | workgroup | VGPRs | LDS bytes | calls | median us | avg us | "
              "min us | max us | GB/s at median (17 B/px) |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
    for key in sorted(agg, key=lambda k: (-k[1], k[0])):
        d = sorted(agg[key])
        med = statistics.median(d)
        wg, vg, lds = meta[key]
        px = (pixels or {}).get(key[1])
        gbs = f"{17 * px / (med * 1e-6) / 1e9:.0f}" if px else ""
        lines.append(f"| `{key[0]}` | {key[1]} | {wg} | {vg} | {lds} | {len(d)} | {med:.3f} | "
                     f"{sum(d) / len(d):.3f} | {d[0]:.3f} | {d[-1]:.3f} | {gbs} |")
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as fh:
        fh.write(text)
    return text


def _per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, value)} for one counter."""
    out = {}
    for r in rows:
        name = r.get("Counter_Name") or r.get("Counter-Name")
        if name != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id")
        val = float(r.get("Counter_Value") or r.get("Counter-Value"))
        k = r.get("Kernel_Name") or r.get("Kernel-Name")
        g = int(r.get("Grid_Size") or r.get("Grid-Size") or 0)
        prev = out.get(did)
        out[did] = (k, val + (prev[1] if prev else 0.0), g)
    return out


def _kernel_values(disp, needle: str, grid: int = 0):
    return [v for (k, v, g) in disp.values() if needle in k and (not grid or g == grid)]


def _calibration_values(disp, needle: str, count: int):
    """The `count` largest readings of the calibration kernel: bench.py runs
    its calibration copy `count` times; smaller dispatches of the same
    kernel are unrelated host-to-device copies."""
    return sorted(_kernel_values(disp, needle), reverse=True)[:count]


def tile_shape_of_kernel(kernel: str):
    """The library's name of the tile shape ("variant") a single-frame kernel
    runs, from its template name; None for kernels without a choice of shape
    (the batch and stack kernels, the adjoint)."""
    m = re.match(r"k_(scalar|vec4|vec4p|vec4w)<([^>]*)>", kernel)
    if not m:
        return None
    kind, targs = m.group(1), [t.strip() for t in m.group(2).split(",")]
    if kind == "scalar":
        return "scalar"
    if kind == "vec4p":
        return "vec4p2"
    if kind == "vec4w":
        return f"vec4w{targs[2]}"
    return {"1": "vec4", "2": "vec4x2", "4": "vec4x4"}[targs[1]]


def traffic(fetch_dir: str, write_dir: str, kernel: str, pixels: int, workload: str,
            out_json: str, calib_bytes: int, calib_kernel: str, cmd: str = "",
            calib_count: int = 4, bytes_per_pixel: int = 17, adjoint: bool = False,
            grid: int = 0) -> dict:
    sys.path.insert(0, ROOT)
    import bench   # noqa: E402  (the hash bench.py checks)
    f_rows = _csv_rows(fetch_dir, "*counter_collection.csv")
    w_rows = _csv_rows(write_dir, "*counter_collection.csv")
    f = _per_dispatch(f_rows, "FETCH_SIZE")
    w = _per_dispatch(w_rows, "WRITE_SIZE")
    fc = _calibration_values(f, calib_kernel, calib_count)
    wc = _calibration_values(w, calib_kernel, calib_count)
    fk = _kernel_values(f, kernel, grid)
    wk = _kernel_values(w, kernel, grid)
    if not (fc and wc and fk and wk):
        raise SystemExit(f"missing dispatches: calib {len(fc)}/{len(wc)}, kernel {len(fk)}/{len(wk)}")
    # copy kernel: reads and writes calib_bytes each
    f_factor = calib_bytes / statistics.median(fc)
    w_factor = calib_bytes / statistics.median(wc)
    rb = statistics.median(fk) * f_factor
    wb = statistics.median(wk) * w_factor
    rec = {
        "workload": workload,
        "kernel": kernel,
        "variant": tile_shape_of_kernel(kernel),
        "grid_size": grid or None,
        "pixels_per_launch": pixels,
        "algorithmic_bytes_per_launch": bytes_per_pixel * pixels,
        "hbm_read_bytes_per_launch": rb,
        "hbm_write_bytes_per_launch": wb,
        "hbm_bytes_per_launch": rb + wb,
        "read_bytes_per_pixel": rb / pixels,
        "write_bytes_per_pixel": wb / pixels,
        "fetch_factor": f_factor,
        "write_factor": w_factor,
        "calibration": f"{calib_kernel} (largest {calib_count} dispatches): {calib_bytes} bytes "
                       f"read and written each",
        "dispatches": {"fetch": len(fk), "write": len(wk)},
        "kernel_hash": bench.kernel_hash(bench.ADJOINT_SOURCES if adjoint else None),
        "command": cmd,
    }
    # one file per workload: the first record written (the library's default
    # tile shape) at the top, the other tile shapes of the same sources under
    # "other_tile_shapes"
    old = None
    if os.path.exists(out_json):
        try:
            old = json.load(open(out_json))
        except ValueError:
            old = None
    if (old and old.get("workload") == workload and old.get("kernel_hash") == rec["kernel_hash"]
            and old.get("variant") != rec["variant"]):
        shape = {k: rec[k] for k in ("kernel", "grid_size", "hbm_read_bytes_per_launch",
                                     "hbm_write_bytes_per_launch", "hbm_bytes_per_launch",
                                     "read_bytes_per_pixel", "write_bytes_per_pixel",
                                     "dispatches")}
        old.setdefault("other_tile_shapes", {})[rec["variant"]] = shape
        rec = old
    elif old and old.get("kernel_hash") == rec["kernel_hash"] and "other_tile_shapes" in old:
        rec["other_tile_shapes"] = old["other_tile_shapes"]
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def launches(reps: int = 20) -> None:
    """Each kernel of interest `reps` times: the three methods on one
    1920x1080 frame, then the stacked forward and adjoint (vector kernel, and
    scalar tiles on a padded copy) on 16 x 640x480."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    import paper_2209_08241_amd as bn
    from synth import scenes
    s = scenes.frame_1920x1080(seed=2)
    d = torch.from_numpy(s.depth).cuda()
    for method, alpha, K in (("four_pair", 2, 0), ("pair_removal", 2, 0), ("multiscale", 1, 3)):
        for _ in range(reps):
            bn.estimate_normals(d, *s.intrinsics, alpha, method=method, scales=K)
    scs = [scenes.frame_640x480(seed=2000 + i) for i in range(16)]
    intr = [x.intrinsics for x in scs]
    st = torch.from_numpy(np.stack([x.depth for x in scs])).cuda()
    g = torch.randn((16, 480, 640, 3), device="cuda")
    # the same stack with a row stride of 641: the adjoint's scalar tiles
    pad = torch.zeros((16, 480, 641), device="cuda")
    pad[:, :, :640] = st
    for _ in range(reps):
        bn.estimate_normals_stack(st, intr, want_stats=False)
        bn.normals_vjp_stack(st, intr, g)
        bn.normals_vjp_stack(pad[:, :, :640], intr, g)
    torch.cuda.synchronize()
    print("launches done", flush=True)


def rings(reps: int = 64, calibration_mib: int = 1024) -> None:
    """The benchmark's single-frame and batched configurations as a program
    for counter passes: a calibration copy (4 times), then `reps` launches
    over a ring of distinct buffers for each of: four-pair, pair removal,
    multi-scale (alpha 1, K 3) and (alpha 3, K 3) on 1920x1080, each in the
    library's default tile shape and then in every other shape the autotuner
    may choose for it (the autotuner itself cannot time anything under a
    counter profiler, which serialises every dispatch); four-pair on 640x480
    in each shape (a ring of 256); then three runs of the 256-frame mixed
    batch (flat grid)."""
    sys.path.insert(0, ROOT)
    import concurrent.futures as cf
    from synth import scenes
    # host frames first, on threads (under a profiler the GPU runtime may be
    # initialised before this program starts, so nothing here forks)
    shapes = scenes.batch_shapes()
    jobs = [(H, W, 1000 + i, {}) for i, (H, W) in enumerate(shapes)]
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        batch_h = list(ex.map(scenes._sized_job, jobs))
    f1080 = [scenes.frame_1920x1080(seed=2 + i) for i in range(8)]
    f640 = [scenes.frame_640x480(seed=1 + i) for i in range(8)]
    import torch
    import paper_2209_08241_amd as bn
    if calibration_mib:
        src = torch.ones(calibration_mib * (1 << 20) // 4, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def ring_of(frames, n):
        H, W = frames[0].depth.shape
        d = [torch.from_numpy(frames[i % len(frames)].depth).cuda() for i in range(n)]
        nm = [torch.empty((H, W, 3), device="cuda") for _ in range(n)]
        mk = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(n)]
        st = bn.new_stats(n, device="cuda")
        return d, nm, mk, st

    # the library's default tile shapes first, then every other shape the
    # autotuner may choose for the configuration
    names = dict(bn.variants())
    runs = [("four_pair", 2, 0, 0), ("pair_removal", 2, 0, 0), ("multiscale", 1, 3, 0),
            ("multiscale", 3, 3, 0)]
    runs += [("four_pair", 2, 0, v) for v in (1, 3, 4, 5, 6, 7)]
    runs += [("pair_removal", 2, 0, v) for v in (1, 3, 4, 5, 6, 7)]
    runs += [("multiscale", a, 3, v) for a in (1, 3) for v in (1, 3, 4)]
    d, nm, mk, st = ring_of(f1080, 32)
    s0 = f1080[0]
    for method, alpha, K, v in runs:
        print(f"1920x1080 {method} alpha {alpha} K {K} {names.get(v, 'default')}", flush=True)
        for r in range(reps):
            j = r % 32
            bn.estimate_normals(d[j], *s0.intrinsics, alpha, method=method, scales=K, variant=v,
                                normals=nm[j], mask=mk[j], stats=st[j])
        torch.cuda.synchronize()
    del d, nm, mk, st
    d, nm, mk, st = ring_of(f640, 256)
    for v in (0, 2, 3, 4, 5, 6, 7):
        print(f"640x480 four_pair alpha 2 {names.get(v, 'default')}", flush=True)
        for r in range(max(reps, 256)):
            j = r % 256
            bn.estimate_normals(d[j], *f640[0].intrinsics, 2, variant=v, normals=nm[j],
                                mask=mk[j], stats=st[j])
        torch.cuda.synchronize()
    del d, nm, mk, st
    frames = [bn.BatchFrame(torch.from_numpy(s.depth).cuda(), s.fx, s.fy, s.cx, s.cy)
              for s in batch_h]
    with bn.BatchPlan(frames) as plan:
        for _ in range(3):
            plan.run()
        torch.cuda.synchronize()
    print("rings done", flush=True)


class _Request:
    """A device depth frame offered to the server (its outputs live in the
    server's slots)."""

    def __init__(self, depth, fx, fy, cx, cy):
        self.depth, self.fx, self.fy, self.cx, self.cy = depth, fx, fy, cx, cy

    def _c(self):
        import paper_2209_08241_amd as bn
        H, W = self.depth.shape
        return bn.Frame(self.depth.data_ptr(), H, W, self.depth.stride(0), self.fx, self.fy,
                        self.cx, self.cy, 0, 0, 0)


def serve_launches(requests: int = 4000, rate_hz: float = 50000.0) -> None:
    """The benchmark's serving workload under a profiler: the five serving
    sizes (320x240 to 4096x3072, seeds 3000..3004), 16 depth-scaled device
    copies of each, offered to a server (16 GiB budget, batches of up to 16
    requests, 2 in flight) as an open-loop Poisson stream of `requests` at
    `rate_hz`, then `requests` / 4 at once (a backlog: full batches)."""
    sys.path.insert(0, ROOT)
    import concurrent.futures as cf
    from synth import scenes
    jobs = [(H, W, 3000 + k, {}) for k, (H, W) in enumerate(scenes.SERVE_SIZES)]
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        frames_h = list(ex.map(scenes._sized_job, jobs))
    import torch
    import paper_2209_08241_amd as bn
    gen = torch.Generator(device="cuda").manual_seed(3000)
    pool = []
    for s in frames_h:
        d = torch.from_numpy(s.depth).cuda()
        H, W = s.depth.shape
        for _ in range(16):
            f = 1.0 + 0.02 * (2.0 * float(torch.rand((), device="cuda", generator=gen)) - 1.0)
            pool.append(_Request(d * f, s.fx, s.fy, s.cx, s.cy))
    with bn.Server(16 << 30, max_batch=16, max_batches_in_flight=2) as srv:
        r = srv.run_poisson(pool, rate_hz, requests, seed=3000)
        print(f"poisson {requests} requests at {rate_hz:.0f}/s: {r['wall_s'] * 1e3:.1f} ms",
              flush=True)
        r = srv.run_poisson(pool, 1e12, requests // 4, seed=3100)
        print(f"backlog {requests // 4} requests: {r['wall_s'] * 1e3:.1f} ms", flush=True)
        print(json.dumps(srv.stats()), flush=True)
    torch.cuda.synchronize()
    print("serve done", flush=True)


# kernel -> (workload, pixels or outputs per dispatch)
def diff_launches(reps: int = 12, calibration_mib: int = 1024) -> None:
    """The differentiation workload of bench.py under a profiler: a
    calibration copy (4 times), then the stacked forward and adjoint on
    16 x 640x480, `reps` calls each, cycling over six buffer sets."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    import paper_2209_08241_amd as bn
    from synth import scenes
    if calibration_mib:
        src = torch.ones(calibration_mib * (1 << 20) // 4, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sets = 6
    scs = [scenes.frame_640x480(seed=2000 + i) for i in range(16)]
    intr = [x.intrinsics for x in scs]
    d0 = torch.from_numpy(np.stack([x.depth for x in scs])).cuda()
    g0 = torch.randn((16, 480, 640, 3), device="cuda")
    D = [d0.clone() for _ in range(sets)]
    G = [g0.clone() for _ in range(sets)]
    GD = [torch.empty((16, 480, 640), device="cuda") for _ in range(sets)]
    N = [torch.empty((16, 480, 640, 3), device="cuda") for _ in range(sets)]
    M = [torch.empty((16, 480, 640), dtype=torch.uint8, device="cuda") for _ in range(sets)]
    for r in range(reps):
        i = r % sets
        bn.estimate_normals_stack(D[i], intr, normals=N[i], mask=M[i], want_stats=False)
    for r in range(reps):
        i = r % sets
        bn.normals_vjp_stack(D[i], intr, G[i], grad_depth=GD[i])
    torch.cuda.synchronize()
    print("diff launches done", flush=True)


_VALU_WHAT = {
    "bn::k_vec4<2, 1, 0>": ("four-pair, 1920x1080, alpha 2", 2073600),
    "bn::k_vec4<2, 1, 1>": ("pair removal, 1920x1080, alpha 2", 2073600),
    "bn::k_vec4<1, 1, 2>": ("multi-scale K=3, 1920x1080, alpha 1", 2073600),
    "bn::k_stack<2, 0>": ("four-pair stack, 16 x 640x480", 16 * 307200),
    "bn::k_vjp4_stack<2, 4, 8>": ("adjoint stack, 16 x 640x480, vector kernel", 16 * 307200),
    "bn::k_vjp_stack<2, 64, 16>": ("adjoint stack, 16 x 640x480, scalar tiles (row stride 641)",
                                   16 * 307200),
}


def valu_summary(pmc_dir: str, out_md: str, cmd: str = "") -> str:
    rows = _csv_rows(pmc_dir, "*counter_collection.csv")
    agg: dict = {}
    for r in rows:
        k = r.get("Kernel_Name") or r.get("Kernel-Name")
        if "bn::" not in k:
            continue
        short = k.split("(")[0].replace("void ", "")
        if short not in _VALU_WHAT:
            continue  # set-up kernels (work-area clears)
        c = agg.setdefault(short, {})
        name = r.get("Counter_Name") or r.get("Counter-Name")
        c.setdefault(name, []).append(float(r.get("Counter_Value") or r.get("Counter-Value")))
        c.setdefault("_dur", []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["# VALU counters of the main kernels (rocprofv3 --pmc)", ""]
    if cmd:
        lines += ["Command:", "", "```", cmd, "```", ""]
    lines += ["Medians over each kernel's dispatches.  Instruction counts are per wavefront; "
              "VALU / pixel is the lane-instructions per pixel (or output) of the dispatch, "
              "SQ_INSTS_VALU x 64 / pixels; VALUBusy is rocprofv3's derived share of the "
              "kernel's time in which the vector ALUs issue; durations are under the "
              "profiler.", "",
              "| kernel | workload | wavefronts | VALU / wavefront | VALU / pixel | "
              "SALU / wavefront | LDS / wavefront | VMEM reads / wavefront | VALUBusy | "
              "VALUUtilization | duration (profiled) |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, c in agg.items():
        med = {n: statistics.median(v) for n, v in c.items()}
        w = med.get("SQ_WAVES", 1.0) or 1.0
        what, npx = _VALU_WHAT.get(k, ("", 0))
        per_px = f"{med['SQ_INSTS_VALU'] * 64 / npx:.0f}" if npx else ""
        lines.append(f"| `{k}` | {what} | {w:.0f} | "
                     f"{med['SQ_INSTS_VALU'] / w:.0f} | {per_px} | "
                     f"{med['SQ_INSTS_SALU'] / w:.0f} | {med['SQ_INSTS_LDS'] / w:.1f} | "
                     f"{med['SQ_INSTS_VMEM_RD'] / w:.1f} | {med['VALUBusy']:.1f}% | "
                     f"{med['VALUUtilization']:.1f}% | {med['_dur']:.1f} us |")
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as fh:
        fh.write(text)
    return text


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    t.add_argument("out_md")
    t.add_argument("--cmd", default="")
    p = sub.add_parser("traffic")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--pixels", type=int, required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--out", required=True)
    p.add_argument("--calib-bytes", type=int, required=True)
    p.add_argument("--calib-kernel", default="copyBuffer")
    p.add_argument("--calib-count", type=int, default=4)
    p.add_argument("--cmd", default="")
    p.add_argument("--bytes-per-pixel", type=int, default=17)
    p.add_argument("--adjoint", action="store_true",
                   help="hash the adjoint's sources (bench.ADJOINT_SOURCES)")
    p.add_argument("--grid", type=int, default=0,
                   help="only dispatches of this grid size (threads), 0: any")
    rg = sub.add_parser("rings")
    rg.add_argument("--reps", type=int, default=64)
    rg.add_argument("--calibration-mib", type=int, default=1024)
    ln = sub.add_parser("launches")
    ln.add_argument("--reps", type=int, default=20)
    df = sub.add_parser("diff")
    df.add_argument("--reps", type=int, default=12)
    df.add_argument("--calibration-mib", type=int, default=1024)
    sv = sub.add_parser("serve")
    sv.add_argument("--requests", type=int, default=4000)
    sv.add_argument("--rate", type=float, default=50000.0)
    tg = sub.add_parser("tracegrid")
    tg.add_argument("trace_dir")
    tg.add_argument("out_md")
    tg.add_argument("--cmd", default="")
    tg.add_argument("--pixels-of", action="append", default=[], metavar="GRID=PIXELS",
                    help="pixels one launch of this grid size covers (repeatable)")
    v = sub.add_parser("valu")
    v.add_argument("pmc_dir")
    v.add_argument("out_md")
    v.add_argument("--cmd", default="")
    a = ap.parse_args()
    if a.what == "launches":
        launches(a.reps)
    elif a.what == "rings":
        rings(a.reps, a.calibration_mib)
    elif a.what == "diff":
        diff_launches(a.reps, a.calibration_mib)
    elif a.what == "serve":
        serve_launches(a.requests, a.rate)
    elif a.what == "valu":
        print(valu_summary(a.pmc_dir, a.out_md, a.cmd))
    elif a.what == "trace":
        print(trace_summary(a.stats_csv, a.out_md, a.cmd))
    elif a.what == "tracegrid":
        px = {int(g): int(n) for g, n in (x.split("=") for x in a.pixels_of)}
        print(trace_by_grid(a.trace_dir, a.out_md, a.cmd, px))
    else:
        print(json.dumps(traffic(a.fetch, a.write, a.kernel, a.pixels, a.workload, a.out,
                                 a.calib_bytes, a.calib_kernel, a.cmd, a.calib_count,
                                 a.bytes_per_pixel, a.adjoint, a.grid), indent=1))


if __name__ == "__main__":
    main()
