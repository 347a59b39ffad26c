#!/usr/bin/env python3
"""Throughput of E_s E_s^* (matern_cov_apply) on one MI355X.

Workload: 64 images of 1024x1024 FP32 (20-disc phantoms plus N(0, 0.05) noise), periodic
db8, 7 levels, s = 1.5, forward E_s E_s^* = W^T D_2s W x over the whole batch in one call.
One step = one such call; inputs are resident in HBM before timing starts.

Printed (one JSON line on stdout):
  value        voxels/s of the whole batch (64 * 1024^2 voxels per step)
  roofline     the dominant kernel of the launch sequence: its algorithmic HBM bytes per launch
               divided by its average duration, timed live here with HIP events on the stream
               it is launched on, against the 8 TB/s HBM peak
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same images (1 core)
  plain        the same op through the plain per-image, per-axis, per-level launches
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E_s E_s^* voxels/s + HBM GB/s, batched/autograd vs plain; FP32 err vs FP64"
HBM_PEAK_GBPS = 8000.0
IMAGES, SIDE, ORDER, LEVELS, S = 64, 1024, 8, 7, 1.5


def kernel_bytes(name, level, batch, side, ndim=2):
    """Algorithmic HBM bytes of one launch: every array it must read or write, once."""
    def n(i):
        return (side >> i) ** ndim
    kind = name.split("_")[0] + "_" + name.split("_")[1]
    if kind == "lp_down":  # a_{i-1} -> a_i, i = level + 1 (level = input level)
        return 4 * batch * (n(level) + n(level + 1))
    if kind == "lp_up":  # z_{i+1}, same_i -> out_i
        return 4 * batch * (n(level + 1) + 2 * n(level))
    if kind.startswith("tail"):
        return 4 * batch * 2 * n(level)
    return 4 * batch * 2 * n(level)  # full-bank level: read and write the level block


def trace_summary(path):
    """Per-dispatch-shape summary of a `rocprofv3 --kernel-trace --output-format csv` trace.

    Dispatches are grouped by kernel name and grid size (the same kernel template serves
    several pyramid levels); durations are End - Start of each dispatch.
    """
    import csv
    groups = {}
    for r in csv.DictReader(open(path)):
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["| kernel | work-groups | dispatches | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for (name, wg), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {wg} | {len(d)} | {statistics.mean(d):.2f} | {min(d):.2f} | {max(d):.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--trace-summary", metavar="CSV", help="summarise a rocprofv3 kernel trace and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: this build runs on one MI355X only "
              "(--gpus must be 1; multi-GPU sharding is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_2507_02401_amd as es
    from paper_2507_02401_amd import _lib

    lib = _lib.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print(f"[bench] generating {IMAGES} x {SIDE}^2 phantoms", file=sys.stderr, flush=True)
    data = inputs.image_batch(count=IMAGES, side=SIDE)
    x = torch.from_numpy(data["x"]).to(dev)
    y = torch.empty_like(x)
    grid = (SIDE, SIDE)
    ws = torch.empty(max(1, es.workspace_bytes(es.OP_COV, grid, IMAGES, ORDER, LEVELS)), dtype=torch.uint8, device=dev)
    voxels = IMAGES * SIDE * SIDE

    def step():
        es.matern_cov_apply(x, 2, ORDER, LEVELS, S, out=y, workspace=ws)

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    value = voxels / (elapsed / args.steps)

    # per-kernel durations: the same launch sequence, one launch at a time between HIP events
    stream = torch.cuda.current_stream(dev)
    shp = _lib.shape_arg(grid)
    nsteps = lib.es_schedule_length(es.OP_COV, 2, shp, IMAGES, ORDER, LEVELS)
    names, levels, wgs = [], [], []
    import ctypes
    for j in range(nsteps):
        buf = ctypes.create_string_buffer(128)
        wg = ctypes.c_int64()
        lv = ctypes.c_int32()
        _lib.check(lib.es_schedule_describe(es.OP_COV, 2, shp, IMAGES, ORDER, LEVELS, j, buf, 128, ctypes.byref(wg),
                                            ctypes.byref(lv)))
        names.append(buf.value.decode())
        levels.append(lv.value)
        wgs.append(wg.value)
    reps = max(3, min(args.steps, 10))
    per = [[] for _ in range(nsteps)]
    for _ in range(reps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nsteps + 1)]
        evs[0].record(stream)
        for j in range(nsteps):
            _lib.check(lib.es_schedule_run_step(es.OP_COV, 2, shp, IMAGES, ORDER, LEVELS, S, x.data_ptr(), y.data_ptr(),
                                                ws.data_ptr(), ws.numel(), j, stream.cuda_stream))
            evs[j + 1].record(stream)
        torch.cuda.synchronize()
        for j in range(nsteps):
            per[j].append(evs[j].elapsed_time(evs[j + 1]))
    kernels = []
    for j in range(nsteps):
        mean_ms = statistics.mean(per[j])
        b = kernel_bytes(names[j], levels[j], IMAGES, SIDE)
        kernels.append(dict(name=names[j], level=levels[j], work_groups=wgs[j], avg_us=round(1e3 * mean_ms, 2),
                            algorithmic_bytes=b, GBps=round(b / (mean_ms * 1e-3) / 1e9, 1)))
    dom = max(kernels, key=lambda k: k["avg_us"])
    achieved = dom["algorithmic_bytes"] / (dom["avg_us"] * 1e-6) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=None, kernel=dom["name"],
                    level=dom["level"])

    # parity on one sampled image
    i_s = 5
    import oracle
    ref = oracle.matern_cov_apply(data["x"][i_s].astype(np.float64), ORDER, LEVELS, S)
    got = y[i_s].double().cpu().numpy()
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"matern_cov_apply E_s E_s^*: {IMAGES} images {SIDE}x{SIDE}, db{ORDER}, {LEVELS} levels, "
                               f"s={S}, periodic, 20-disc phantoms + N(0,0.05)",
                   "images": IMAGES, "side": SIDE, "order": ORDER, "levels": LEVELS, "s": S, "op": "matern_cov_apply"},
        "hbm_GBps_effective": round(8.0 * value / 1e9, 1),
        "frac_of_hbm_peak_whole_op": round(8.0 * value / 1e9 / HBM_PEAK_GBPS, 4),
        "rel_l2_vs_fp64_oracle_image5": rel,
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_plain:
        print("[bench] plain per-image path", file=sys.stderr, flush=True)
        es.plain_op(es.OP_COV, x, 2, ORDER, LEVELS, S, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es.plain_op(es.OP_COV, x, 2, ORDER, LEVELS, S, out=y)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        result["plain"] = {"ms_per_step": round(1e3 * tp, 3), "value": round(voxels / tp, 1), "unit": "voxels/s",
                           "speedup_of_fused": round(tp / (elapsed / args.steps), 2)}

    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        done, t0 = 0, time.perf_counter()
        while True:
            oracle.matern_cov_apply(data["x"][done % IMAGES].astype(np.float64), ORDER, LEVELS, S)
            done += 1
            if time.perf_counter() - t0 >= args.cpu_seconds or done >= IMAGES:
                break
        tc = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(done * SIDE * SIDE / tc, 1), "unit": "voxels/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"{done} of the {IMAGES} images, FP64 numpy oracle, single process"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
