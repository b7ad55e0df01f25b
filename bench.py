#!/usr/bin/env python3
"""Pack + unpack throughput of MPI-style derived datatypes on one MI355X.

A step is one pass of the hot path over one batch of synthetic input: every
face of the 3-D halo workload (float64 512^3 array, ghost widths 1 and 4,
6 faces each) is packed from the array into contiguous buffers and then
unpacked into a zeroed copy, through the library's C ABI.  The value is
whole-step HBM throughput counted in algorithmic bytes (each packed byte is
read once and written once by pack, and again by unpack: 4 x packed bytes
per step), with all inputs resident in device memory before timing starts.

Other workloads (--workload): particles (struct records x 4M), hindexed (1M
irregular blocks in 2 GiB), contig (1 GiB contiguous), small (the 1024-
element vector).  --mode batched runs each direction of a step as one
persistent batched launch instead of one launch per face.

Prints one JSON line.  Run with no flags for the default single-GPU run.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2402_12274_amd import inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
METRIC = "pack+unpack HBM GB/s vs peak; p50/p99 latency, batched vs per-request"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="halo", choices=["halo", "particles", "hindexed", "contig", "small"])
    ap.add_argument("--mode", default="plain", choices=["plain", "batched"])
    ap.add_argument("--rotate", type=int, default=4,
                    help="rotate over this many copies of the arrays so every step reads cold data")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    return ap.parse_args()


# ---------------------------------------------------------------------------
# workloads: lists of (label, spec, count, source bytes) requests


def workload(name):
    if name == "halo":
        n = 512
        reqs = [(label, spec, 1) for label, spec in inputs.halo_faces(n)]
        return dict(desc="3-D halo faces: float64 512^3 array (1 GiB), ghost widths 1 and 4, all 6 faces "
                         "packed then unpacked into a zeroed copy per step",
                    src_bytes=n ** 3 * 8, reqs=reqs, seed=inputs.DEFAULT_SEED)
    if name == "particles":
        return dict(desc="particle records: struct {int32, float64[3], char[5]} (extent 40) x 4,000,000, "
                         "packed then unpacked per step",
                    src_bytes=4_000_000 * 40, reqs=[("records", inputs.particle_struct(), 4_000_000)],
                    seed=inputs.DEFAULT_SEED + 2)
    if name == "hindexed":
        lens, disps = inputs.hindexed_blocks()
        return dict(desc="hindexed: 1,000,000 blocks, geometric lengths mean 24 B clipped 1..256, random "
                         "non-overlapping displacements in 2 GiB, permuted order; packed then unpacked",
                    src_bytes=1 << 31, reqs=[("hindexed", inputs.hindexed_type(lens, disps), 1)],
                    seed=inputs.DEFAULT_SEED + 1)
    if name == "contig":
        return dict(desc="contiguous: 2^27 float64 (1 GiB), packed then unpacked per step",
                    src_bytes=1 << 30, reqs=[("contig", ("contiguous", 1 << 27, inputs.DOUBLE), 1)],
                    seed=inputs.DEFAULT_SEED + 3)
    if name == "small":
        return dict(desc="small vector: vector(1024, 1, 2, float64), 8 KiB packed from 16 KiB, packed then "
                         "unpacked per step", src_bytes=16384, reqs=[("vector", inputs.vector_small(), 1)],
                    seed=inputs.DEFAULT_SEED)
    raise ValueError(name)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample


def cpu_baseline(W, budget_s):
    import oracle

    host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
    otypes = [(label, oracle.build_type(spec), count) for label, spec, count in W["reqs"]]
    dst = np.zeros_like(host)
    done_bytes = 0
    passes = 0
    t0 = time.perf_counter()
    while True:
        for label, o, count in otypes:
            p = o.pack(host, 0, count)
            o.unpack(p, dst, 0, count)
            done_bytes += 4 * p.size
        passes += 1
        if time.perf_counter() - t0 >= budget_s or passes >= 50:
            break
    dt = time.perf_counter() - t0
    return dict(value=round(done_bytes / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample=f"{passes} full pass(es) of the step's pack+unpack requests on the host "
                       f"({dt:.1f} s, single thread, {platform.processor() or platform.machine()}, "
                       f"nproc={os.cpu_count()})")


def copy_ceiling_gbs(torch, dev, nbytes=1 << 30, reps=10):
    """Measured device-to-device copy rate (read + write bytes) of 1 GiB."""
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    a.fill_(1)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    del a, b
    return round(2 * nbytes / times[len(times) // 2] / 1e9, 1)


# ---------------------------------------------------------------------------


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported on this build "
              "(the single-GPU kernel is the measured unit; see the design notes on sharding)",
              file=sys.stderr)
        return 2
    import torch

    from paper_2402_12274_amd import mdt

    W = workload(args.workload)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)

    host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
    R = max(1, args.rotate if W["src_bytes"] >= (1 << 28) else 1)
    srcs = [torch.from_numpy(host).to(dev) for _ in range(R)]
    dsts = [torch.zeros(W["src_bytes"], dtype=torch.uint8, device=dev) for _ in range(R)]
    del host
    types = [(label, mdt.build_type(spec), count) for label, spec, count in W["reqs"]]
    sizes = [t.size() * count for _, t, count in types]
    packed = [[torch.empty(max(1, s), dtype=torch.uint8, device=dev) for s in sizes] for _ in range(R)]
    step_bytes = 4 * sum(sizes)

    batches = None
    if args.mode == "batched":
        batches = []
        for r in range(R):
            bp = mdt.Batch()
            bu = mdt.Batch()
            for (label, t, count), out in zip(types, packed[r]):
                bp.add_pack(srcs[r].data_ptr(), count, t, 0, out.data_ptr(), -1)
                bu.add_unpack(out.data_ptr(), t.size() * count, dsts[r].data_ptr(), count, t, 0)
            batches.append((bp, bu))
        bp0, bu0 = batches[0]
        bp0.autotune(ms)
        bu0.autotune(ms)
        for bp, bu in batches[1:]:
            bp.set_config(bp0.get_config())
            bu.set_config(bu0.get_config())

    # per-kernel event timing of the pack direction and the unpack direction
    ev_log = {"pack": [], "unpack": []}

    def step(r, timed):
        if batches is not None:
            bp, bu = batches[r]
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            bp.launch(ms)
            e1.record(stream)
            bu.launch(ms)
            e2.record(stream)
            if timed:
                ev_log["pack"].append((e0, e1, sum(sizes)))
                ev_log["unpack"].append((e1, e2, sum(sizes)))
            return
        for (label, t, count), out, s in zip(types, packed[r], sizes):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mdt.mdt_pack_enqueue(srcs[r].data_ptr(), count, t, 0, out.data_ptr(), -1, ms)
            e1.record(stream)
            if timed:
                ev_log["pack"].append((e0, e1, s))
        for (label, t, count), out, s in zip(types, packed[r], sizes):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mdt.mdt_unpack_enqueue(out.data_ptr(), s, dsts[r].data_ptr(), count, t, 0, ms)
            e1.record(stream)
            if timed:
                ev_log["unpack"].append((e0, e1, s))

    for i in range(args.warmup):
        step(i % R, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i % R, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    value = step_bytes * args.steps / dt / 1e9
    copy_ceiling = copy_ceiling_gbs(torch, dev)
    # dominant direction: the one with the larger total kernel time
    per = {}
    for k, lst in ev_log.items():
        durs = [a.elapsed_time(b) * 1e-3 for a, b, _ in lst]
        per[k] = dict(total=sum(durs), n=len(durs), bytes=sum(2 * s for _, _, s in lst))
    dom = max(per, key=lambda k: per[k]["total"])
    d = per[dom]
    avg_dur = d["total"] / max(1, d["n"])
    bytes_per_launch = d["bytes"] / max(1, d["n"])
    achieved = bytes_per_launch / avg_dur / 1e9 if avg_dur > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": W["desc"], "mode": args.mode, "requests_per_step": 2 * len(types),
                   "packed_bytes_per_step": sum(sizes), "rotating_copies": R,
                   "frac_of_peak_value": round(value / PEAK_HBM_GBS, 4),
                   "device_copy_ceiling_GBps": copy_ceiling},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": f"{dom} ({'batched launch' if batches else 'one launch per request'})",
                     "avg_launch_us": round(avg_dur * 1e6, 2), "bytes_per_launch": int(bytes_per_launch)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
