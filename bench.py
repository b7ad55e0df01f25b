#!/usr/bin/env python3
"""Pack + unpack throughput of MPI-style derived datatypes on one MI355X.

A step is one pass of the hot path over one batch of synthetic input: every
face of the 3-D halo workload (float64 512^3 array, ghost widths 1 and 4,
6 faces each) is packed from the array into contiguous buffers and then
unpacked into a zeroed copy, through the library's C ABI.  The value is
whole-step HBM throughput counted in algorithmic bytes (each packed byte is
read once and written once by pack, and again by unpack: 4 x packed bytes
per step), with all inputs resident in device memory before timing starts.

The default run also measures the metric's second half and attaches it to
the same JSON line:
  "batch4096": 4096 pack requests (sizes log-uniform 64 B..16 MiB over
      strided vectors, halo faces and the 1M-block hindexed layout) as one
      batched launch (autotuned, and the best persistent graph-replayed
      configuration) against 4096 plain launches, with its own roofline;
  "serve": the open-loop serving trace (Poisson arrivals, 20,000/s for 60 s,
      mixed pack/unpack, Zipf sizes, 500 resident types) replayed through
      the server and as one plain launch per request: p50/p99 latency and
      aggregate GB/s, then a short saturating replay; sampled requests write
      to their own buffers and the served bytes are compared with the
      per-request bytes.

Other workloads (--workload): particles (struct records x 4M), hindexed (1M
irregular blocks in 2 GiB), contig (1 GiB contiguous), rows (an interior
block of an 8192^2 float64 matrix), darray (one rank's block-cyclic share of
a 512^3 float64 array), small (the 1024-element vector), serve, batch4096,
chunked (1 MiB byte ranges of the particle records and of the hindexed
layout, batched and one launch per range, beside the whole transfer; also
part of the default run as "chunked_1MiB") and copy (periodic halo
self-exchange by typed copy).  --mode batched (the
default) runs each direction of a step as one batched launch (autotuned);
--mode plain launches once per request.

roofline: the launches are queued back to back between one pair of HIP
events on the launch stream; the region's device time over its launch count
is the average launch duration, and achieved = algorithmic bytes per launch
over it.  traffic: measured HBM bytes per launch from the committed counter
summary (profiles/hbm_traffic.md) when it was taken on the current sources.

cpu_baseline: the oracle as it stands, on the host's cores (all of them,
each task a 1 MiB byte range of a request's packed stream; and single
threaded, each request whole), over whole passes of the step's requests;
its packed and unpacked bytes are compared with the GPU's.

Prints one JSON line.  Run with no flags for the default single-GPU run.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from paper_2402_12274_amd import inputs  # noqa: E402

PEAK_HBM_GBS = 8000.0
TRAFFIC_TABLE = os.path.join(HERE, "profiles", "hbm_traffic.md")
MiB = 1 << 20
GiB = 1 << 30


# the sources that decide what the kernels execute: kernel bodies, the
# layout program and its tables, launch selection and the batch kernels
KERNEL_SOURCES = ("batch.hip", "batch_kernel.h", "batch_variants.hip", "compile.cpp", "device.h", "device.hip",
                  "layout_dev.h", "xfer.h")


def kernel_sources_sha():
    """sha256 over what decides the work the GPU does for a transfer: the
    kernels, their launch and batching code, and the layout compiler (not the
    host-only constructors or the API header).  A measured HBM traffic figure
    holds only for the sources it was measured on."""
    import hashlib

    h = hashlib.sha256()
    src = os.path.join(HERE, "paper_2402_12274_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy's readings), or None when there is none for the current sources."""
    if not os.path.exists(TRAFFIC_TABLE):
        return None
    sha = kernel_sources_sha()
    with open(TRAFFIC_TABLE) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 6 and cells[0] == workload and cells[1] == kernel and cells[-1] == sha:
                try:
                    return int(cells[4])
                except ValueError:
                    return None
    return None


METRIC = "pack+unpack HBM GB/s vs peak; p50/p99 latency, batched vs per-request"


def log(msg):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="halo",
                    choices=["halo", "particles", "hindexed", "contig", "rows", "darray", "small", "serve", "batch4096",
                             "copy", "chunked"])
    ap.add_argument("--no-extras", action="store_true",
                    help="halo: skip the batch4096 and serve blocks of the default run")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of trace per replay")
    ap.add_argument("--rate", type=float, default=20000.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--sat-rate", type=float, default=150000.0,
                    help="serve: a second, saturating arrival rate replayed after the first (0: skip)")
    ap.add_argument("--sat-duration", type=float, default=2.0, help="serve: seconds of the saturating trace")
    ap.add_argument("--ring-gib", type=float, default=64.0,
                    help="serve: device ring the in-flight requests' destinations are taken from")
    ap.add_argument("--mode", default="batched", choices=["plain", "batched"])
    ap.add_argument("--rotate", type=int, default=4,
                    help="rotate over this many copies of the arrays so every step reads cold data")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="batched mode: skip the per-request comparison (profiling runs: the timed launches are then "
                         "the trace's last ones)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="seconds of each CPU-baseline leg")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the copy-ceiling measurement (profiling runs: the timed launches stay the trace's last)")
    return ap.parse_args(argv)


# ---------------------------------------------------------------------------
# workloads: lists of (label, spec, count) requests over one source buffer


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
    if name == "rows":
        n, w = 8192, 64
        spec = ("subarray", [n, n], [n - 2 * w, n - 2 * w], [w, w], "C", inputs.DOUBLE)
        return dict(desc="row-dominated subarray: interior [64, 8128)^2 block of a float64 8192x8192 array "
                         "(512 MiB): 8064 rows of 64,512 B, packed then unpacked per step",
                    src_bytes=n * n * 8, reqs=[("rows", spec, 1)], seed=inputs.DEFAULT_SEED + 4)
    if name == "darray":
        n = 512
        spec = ("darray", 8, 5, [n, n, n], ["cyclic"] * 3, [16] * 3, [2, 2, 2], "C", inputs.DOUBLE)
        return dict(desc="distributed array: rank 5's share of a float64 512^3 array (1 GiB) distributed "
                         "cyclic(16) x cyclic(16) x cyclic(16) over a 2 x 2 x 2 process grid (128 MiB in "
                         "128-byte runs), packed then unpacked per step",
                    src_bytes=n ** 3 * 8, reqs=[("darray", spec, 1)], seed=inputs.DEFAULT_SEED + 5)
    if name == "small":
        return dict(desc="small vector: vector(1024, 1, 2, float64), 8 KiB packed from 16 KiB, packed then "
                         "unpacked per step", src_bytes=16384, reqs=[("vector", inputs.vector_small(), 1)],
                    seed=inputs.DEFAULT_SEED)
    raise ValueError(name)


# ---------------------------------------------------------------------------
# the timed step: setup shared with the full-size parity tests


def step_setup(torch, mdt, W, rotate, batched, ms, autotune=True):
    """Device buffers, types and (batched) the two batches per rotating copy
    of workload W, exactly as the timed step runs them: source copies
    (identical bytes), zeroed destinations, one packed buffer per request;
    the pack and unpack batches of copy 0 are autotuned and the others take
    the same configuration."""
    dev = torch.device("cuda:0")
    host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
    R = max(1, rotate if W["src_bytes"] >= (1 << 28) else 1)
    srcs = [torch.from_numpy(host).to(dev) for _ in range(R)]
    dsts = [torch.zeros(W["src_bytes"], dtype=torch.uint8, device=dev) for _ in range(R)]
    del host
    types = [(label, mdt.build_type(spec), count) for label, spec, count in W["reqs"]]
    sizes = [t.size() * count for _, t, count in types]
    packed = [[torch.empty(max(1, s), dtype=torch.uint8, device=dev) for s in sizes] for _ in range(R)]
    S = dict(R=R, srcs=srcs, dsts=dsts, types=types, sizes=sizes, packed=packed, batches=None, tuned=None)
    if batched:
        batches = []
        for r in range(R):
            bp = mdt.Batch()
            bu = mdt.Batch()
            for (label, t, count), out in zip(types, packed[r]):
                bp.add_pack(srcs[r].data_ptr(), count, t, 0, out.data_ptr(), -1)
                bu.add_unpack(out.data_ptr(), t.size() * count, dsts[r].data_ptr(), count, t, 0)
            batches.append((bp, bu))
        S["batches"] = batches
        if autotune:
            # each direction tuned over all rotating copies (inputs as the timed steps see them)
            cp = mdt.autotune_set([bp for bp, _ in batches], ms)
            cu = mdt.autotune_set([bu for _, bu in batches], ms)
            S["tuned"] = {"pack": mdt.config_dict(cp), "unpack": mdt.config_dict(cu)}
    return S


def set_step_config(S, cfg_pack, cfg_unpack):
    for bp, bu in S["batches"]:
        bp.set_config(cfg_pack)
        bu.set_config(cfg_unpack)


def run_step(S, r, batched, ms, mdt):
    """One step on rotating copy r: pack every request, then unpack them."""
    if batched:
        bp, bu = S["batches"][r]
        bp.launch(ms)
        bu.launch(ms)
        return
    src, dst = S["srcs"][r].data_ptr(), S["dsts"][r].data_ptr()
    for (label, t, count), out in zip(S["types"], S["packed"][r]):
        mdt.mdt_pack_enqueue(src, count, t, 0, out.data_ptr(), -1, ms)
    for (label, t, count), out, s in zip(S["types"], S["packed"][r], S["sizes"]):
        mdt.mdt_unpack_enqueue(out.data_ptr(), s, dst, count, t, 0, ms)


def timed_steps(torch, S, batched, ms, stream, steps, warmup, mdt):
    """Warm-up (every rotating copy runs at least once: its first launch
    uploads descriptors or captures a graph), then exactly `steps` timed
    steps bracketed by synchronisation.  Returns wall seconds, device seconds
    (one event pair around the region) and host-side timestamps."""
    R = S["R"]
    for i in range(max(warmup, R)):
        run_step(S, i % R, batched, ms, mdt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)  # created here, outside the region (the first record creates the event)
    e1.record(stream)
    torch.cuda.synchronize()
    marks = []
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        run_step(S, i % R, batched, ms, mdt)
        marks.append(time.perf_counter())
    e1.record(stream)
    t_issued = time.perf_counter()
    while not e1.query():  # poll: a blocking wait can sleep past the completion
        pass
    t_done = time.perf_counter()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    host = {"enqueue_us_per_step": round((marks[-1] - t0) / steps * 1e6, 2) if steps else 0.0,
            "max_step_enqueue_us": round(max(b - a for a, b in zip([t0] + marks[:-1], marks)) * 1e6, 2)
            if steps else 0.0,
            "issue_done_us": round((t_issued - t0) * 1e6, 1), "device_done_seen_us": round((t_done - t0) * 1e6, 1),
            "sync_after_done_us": round((t_end - t_done) * 1e6, 1)}
    return t_end - t0, e0.elapsed_time(e1) * 1e-3, host


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample; its results are
# compared with the GPU's


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(W, budget_s, gpu_packed=None, gpu_dst=None):
    """The oracle over whole passes of the step's requests: all cores (each
    task a 1 MiB byte range of one request's packed stream, packed and then
    unpacked by the oracle's partial pack/unpack; ctypes releases the GIL, so
    the tasks run in parallel), then single threaded (each request packed
    and unpacked whole).  gpu_packed / gpu_dst:
    the GPU's packed buffers (one per request) and unpacked array, compared
    with the oracle's (equal bytes expected)."""
    import concurrent.futures as cf

    import oracle

    model, ncores = host_cpu()
    host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
    otypes = [(label, oracle.build_type(spec), count) for label, spec, count in W["reqs"]]
    totals = [o.attrs()["size"] * count for _, o, count in otypes]
    packed = [np.zeros(max(1, n), np.uint8) for n in totals]
    dst = np.zeros_like(host)
    tasks = [(k, off) for k, n in enumerate(totals) for off in range(0, n, MiB)]

    def pack_task(kt):
        k, off = kt
        _, o, count = otypes[k]
        p = o.pack(host, 0, count, off, MiB)
        packed[k][off:off + p.size] = p

    def unpack_task(kt):
        k, off = kt
        _, o, count = otypes[k]
        o.unpack(packed[k][off:min(totals[k], off + MiB)], dst, 0, count, off)

    def run_pass(pool):
        if pool is None:
            # one thread: each request packed and unpacked whole
            for k, (_, o, count) in enumerate(otypes):
                p = o.pack(host, 0, count)
                packed[k][:p.size] = p
                o.unpack(p, dst, 0, count)
        else:
            list(pool.map(pack_task, tasks))
            list(pool.map(unpack_task, tasks))

    step_bytes = 4 * sum(totals)
    legs = {}
    for name, threads in (("all_cores", ncores), ("single_thread", 1)):
        pool = cf.ThreadPoolExecutor(threads) if threads > 1 else None
        passes = 0
        t0 = time.perf_counter()
        while True:
            run_pass(pool)
            passes += 1
            if time.perf_counter() - t0 >= budget_s or passes >= 50:
                break
        dt = time.perf_counter() - t0
        if pool is not None:
            pool.shutdown()
        legs[name] = dict(value=round(passes * step_bytes / dt / 1e9, 4), threads=threads, passes=passes,
                          seconds=round(dt, 2))
    out = dict(value=legs["all_cores"]["value"], unit="GB/s", cores=ncores, kind="oracle",
               sample=f"{legs['all_cores']['passes']} full pass(es) of the step's pack+unpack requests on "
                      f"{ncores} host threads, 1 MiB byte ranges per task ({legs['all_cores']['seconds']} s); "
                      f"CPU: {model}",
               single_thread=legs["single_thread"], cpu_model=model)
    if gpu_packed is not None:
        bad = sum(int(not np.array_equal(g[:n], p[:n])) for g, p, n in zip(gpu_packed, packed, totals))
        check = {"requests": len(totals), "packed_mismatching_requests": bad,
                 "packed_bytes_compared": int(sum(totals))}
        if gpu_dst is not None:
            d = np.nonzero(gpu_dst != dst)[0]
            check.update(unpacked_bytes_compared=int(dst.size), unpacked_bytes_differing=int(d.size))
        out["agrees_with_gpu"] = check
    return out


def hip_lib():
    return C.CDLL("libamdhip64.so")


def copy_ceiling(torch, mdt, nbytes=4 * GiB, reps=8):
    """Measured device copy rates (read + write bytes) of 4 GiB: the HIP
    runtime's device-to-device memcpy, and this library's own streaming copy
    (the pack of a contiguous type, which runs the chunk kernel's whole-tile
    copy path)."""
    dev = torch.device("cuda:0")
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    a.fill_(1)
    stream = torch.cuda.current_stream()
    hip = hip_lib()
    hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    hip.hipMemcpyAsync.restype = C.c_int
    ms = mdt.Stream(stream.cuda_stream)
    t = mdt.build_type(("contiguous", nbytes // 8, inputs.DOUBLE))

    def memcpy():
        rc = hip.hipMemcpyAsync(C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()), nbytes, 3,
                                C.c_void_p(stream.cuda_stream))
        assert rc == 0, rc

    def own():
        mdt.mdt_pack_enqueue(a.data_ptr(), 1, t, 0, b.data_ptr(), -1, ms)

    out = {}
    for name, fn in (("hipMemcpyDtoD", memcpy), ("library_streaming_copy", own)):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        times.sort()
        out[name + "_GBps"] = round(2 * nbytes / times[len(times) // 2] / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


# ---------------------------------------------------------------------------
# pipelined partial transfers: 1 MiB byte ranges of one request


def chunked_block(args, torch, mdt, budget=1 << 20, reps=10):
    """The particle records and the hindexed layout packed and unpacked in
    1 MiB byte ranges of their packed streams (126 and 23 ranges: the pieces
    a pipelined transfer hands on one at a time), as one autotuned batch per
    direction and as one launch per range, beside the whole transfer in one
    launch.  Sources of 256 MiB or more rotate over 4 copies.  The ranges'
    packed bytes are checked equal to the whole pack's and the ranges'
    unpack equal to the whole unpack's; times are medians of `reps`."""
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    dev = torch.device("cuda:0")
    out = {"budget_bytes": budget}
    for name in ("particles", "hindexed"):
        W = workload(name)
        (_, spec, count), = W["reqs"]
        t = mdt.build_type(spec)
        total = t.size() * count
        host = inputs.random_bytes(W["src_bytes"], seed=W["seed"])
        R = 4 if W["src_bytes"] >= (1 << 28) else 1
        srcs = [torch.from_numpy(host).to(dev) for _ in range(R)]
        del host
        whole_p = torch.empty(total, dtype=torch.uint8, device=dev)
        parts_p = [torch.empty(total, dtype=torch.uint8, device=dev) for _ in range(R)]
        whole_d = torch.zeros(W["src_bytes"], dtype=torch.uint8, device=dev)
        parts_d = [torch.zeros(W["src_bytes"], dtype=torch.uint8, device=dev) for _ in range(R)]
        ranges = [(o, min(budget, total - o)) for o in range(0, total, budget)]
        bps, bus = [], []
        for r in range(R):
            bp, bu = mdt.Batch(), mdt.Batch()
            for o, n in ranges:
                bp.add_pack(srcs[r].data_ptr(), count, t, o, parts_p[r].data_ptr() + o, n)
                bu.add_unpack(parts_p[r].data_ptr() + o, n, parts_d[r].data_ptr(), count, t, o)
            bps.append(bp)
            bus.append(bu)
        log(f"chunked {name}: autotune")
        cp = mdt.autotune_set(bps, ms)
        cu = mdt.autotune_set(bus, ms)
        for bp in bps:
            bp.set_config(cp)
        for bu in bus:
            bu.set_config(cu)
        it = {"p": 0, "u": 0}

        def nxt(k):
            it[k] += 1
            return it[k] % R

        def whole_pack():
            mdt.mdt_pack_enqueue(srcs[nxt("p")].data_ptr(), count, t, 0, whole_p.data_ptr(), -1, ms)

        def whole_unpack():
            mdt.mdt_unpack_enqueue(whole_p.data_ptr(), total, whole_d.data_ptr(), count, t, 0, ms)

        def batch_pack():
            bps[nxt("p")].launch(ms)

        def batch_unpack():
            bus[nxt("u")].launch(ms)

        def plain_pack():
            r = nxt("p")
            for o, n in ranges:
                mdt.mdt_pack_enqueue(srcs[r].data_ptr(), count, t, o, parts_p[r].data_ptr() + o, n, ms)

        def plain_unpack():
            r = nxt("u")
            for o, n in ranges:
                mdt.mdt_unpack_enqueue(parts_p[r].data_ptr() + o, n, parts_d[r].data_ptr(), count, t, o, ms)

        res = {"workload": W["desc"], "packed_bytes": total, "ranges": len(ranges),
               "last_range_bytes": ranges[-1][1], "autotuned": {"pack": mdt.config_dict(cp),
                                                               "unpack": mdt.config_dict(cu)}}
        for form, fp, fu, launches in (("whole", whole_pack, whole_unpack, 1),
                                       ("batched_ranges", batch_pack, batch_unpack, 1),
                                       ("plain_ranges", plain_pack, plain_unpack, len(ranges))):
            log(f"chunked {name}: {form}")
            wp, dp = time_region(torch, stream, fp, reps, R)
            wu, du = time_region(torch, stream, fu, reps, R)
            res[form] = {"launches_per_direction": launches,
                         "pack_us": round(wp * 1e6, 2), "unpack_us": round(wu * 1e6, 2),
                         "pack_device_us": round(dp * 1e6, 2), "unpack_device_us": round(du * 1e6, 2),
                         "GBps": round(4 * total / (wp + wu) / 1e9, 2)}
        # equality of the range forms with the whole transfer (every copy ran)
        torch.cuda.synchronize()
        res["ranges_equal_whole"] = (all(bool(torch.equal(p, whole_p)) for p in parts_p) and
                                     all(bool(torch.equal(d, whole_d)) for d in parts_d))
        out[name] = res
        del srcs, whole_p, parts_p, whole_d, parts_d, bps, bus
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# batching: 4096 requests in one launch vs 4096 launches


def batch4096_setup(torch, mdt):
    """The 4096-request mix at its stated sizes: shared read-only source
    arenas (a 1 GiB vector arena, the 512^3 halo array, the 2 GiB hindexed
    buffer), one type per distinct spec, each request the partial pack
    [0, min(target, type size)) into its own 256-byte-aligned slice of one
    output buffer.  Returns the plan and an unconfigured batch."""
    dev = torch.device("cuda:0")
    reqs = inputs.batch_mix()
    lens, disps = inputs.hindexed_blocks()
    hspec = inputs.hindexed_type(lens, disps)
    arenas = batch4096_arenas()
    src = {k: torch.from_numpy(inputs.random_bytes(b, seed=seed)).to(dev) for k, (b, seed) in arenas.items()}
    cache = {}
    plan = []
    for r in reqs:
        key = r["spec_key"]
        if key not in cache:
            cache[key] = mdt.build_type(r["spec"] if r["spec"] is not None else hspec)
        t = cache[key]
        plan.append((t, src[r["kind"]], min(r["target"], t.size())))
    offs = np.concatenate([[0], np.cumsum([(n + 255) // 256 * 256 for _, _, n in plan])])
    out = torch.empty(int(offs[-1]), dtype=torch.uint8, device=dev)
    b = mdt.Batch()
    for (t, s, n), o in zip(plan, offs):
        b.add_pack(s.data_ptr(), 1, t, 0, out.data_ptr() + int(o), n)
    return dict(reqs=reqs, hspec=hspec, src=src, plan=plan, offs=offs, out=out, batch=b,
                total=sum(n for _, _, n in plan), types=cache)


def batch4096_arenas():
    """Source arenas of the 4096-request mix: kind -> (bytes, seed)."""
    return {"vector": (((1 << 21) - 1) * 64 * 8 + 8, inputs.DEFAULT_SEED),
            "face": (512 ** 3 * 8, inputs.DEFAULT_SEED + 1),
            "hindexed": (1 << 31, inputs.DEFAULT_SEED + 2)}


# persistent, graph-replayed configurations reported beside the autotuner's
# choice (static and dynamic tile split at 2, 4 and 8 workgroups per CU)
PERSISTENT_GRAPH = [(tc, w, pol, 1, 0) for pol in (0, 1) for w in (2, 4, 8) for tc in (1024, 4096)]


def time_region(torch, stream, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        fn()
        e1.record(stream)
        while not e1.query():
            pass
        times.append((time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3))
    wall = sorted(t[0] for t in times)[len(times) // 2]
    dev_t = sorted(t[1] for t in times)[len(times) // 2]
    return wall, dev_t


def batch4096_block(args, torch, mdt, steps=10, warmup=2):
    B = batch4096_setup(torch, mdt)
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    b = B["batch"]
    total = B["total"]
    log("batch4096: autotune")
    cfg = b.autotune(ms)
    tuned = mdt.config_dict(cfg)

    def run_batched():
        b.launch(ms)

    def run_plain():
        for (t, s, n), o in zip(B["plan"], B["offs"]):
            mdt.mdt_pack_enqueue(s.data_ptr(), 1, t, 0, B["out"].data_ptr() + int(o), n, ms)

    res = {}
    wall, dev_t = time_region(torch, stream, run_batched, steps, warmup)
    launches = 4096 if tuned["policy"] == 3 else 1
    res["batched"] = {"makespan_ms": round(wall * 1e3, 3), "device_ms": round(dev_t * 1e3, 3),
                      "GBps": round(2 * total / wall / 1e9, 2), "config": tuned}
    achieved = 2 * total / launches / (dev_t / launches) / 1e9
    kernel = "batch_kernel (one pack launch)" if launches == 1 else "single-request kernels (4096 launches)"
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("batch4096/batched", kernel), "kernel": kernel,
                "avg_launch_us": round(dev_t / launches * 1e6, 2), "bytes_per_launch": int(2 * total / launches)}
    head = {"workload": "batching: 4096 pack requests, packed sizes log-uniform 64 B..16 MiB, types uniform over "
                        "vector(2^21, 1, s<=64, float64), 512^3 halo faces and the 1M-block hindexed layout",
            "packed_bytes": total}
    if args.no_compare:  # profiling runs: the timed launches stay the trace's last
        return {**head, **res, "roofline": roofline}
    best = None
    for c in PERSISTENT_GRAPH:
        b.set_config(mdt.BatchConfig(*c))
        w, d = time_region(torch, stream, run_batched, 3, 1)
        if best is None or w < best[0]:
            best = (w, d, c)
    res["persistent_graph"] = {"makespan_ms": round(best[0] * 1e3, 3), "device_ms": round(best[1] * 1e3, 3),
                               "GBps": round(2 * total / best[0] / 1e9, 2),
                               "config": mdt.config_dict(mdt.BatchConfig(*best[2]))}
    b.set_config(cfg)
    log("batch4096: 4096 plain launches")
    wall_p, dev_p = time_region(torch, stream, run_plain, max(3, steps // 2), 1)
    res["per_request"] = {"makespan_ms": round(wall_p * 1e3, 3), "device_ms": round(dev_p * 1e3, 3),
                          "GBps": round(2 * total / wall_p / 1e9, 2), "launches": 4096}
    return {**head, **res, "speedup_vs_per_request": round(wall_p / wall, 2), "roofline": roofline}


# ---------------------------------------------------------------------------
# serving: the open-loop trace through the server and as per-request launches

SERVE_ARENAS = {"vector": 1 << 30, "face": 512 ** 3 * 8, "hindexed": 1 << 28, "struct": 1 << 30}

LG_REQ = np.dtype([("t_arrive_us", "<f8"), ("unpack", "<i4"), ("type_index", "<i4"), ("count", "<i8"),
                   ("target", "<i8"), ("typed", "<u8"), ("packed", "<u8"), ("fixed", "<u8"), ("span", "<i8"),
                   ("origin_off", "<i8")], align=True)


class LgResult(C.Structure):
    _fields_ = [("completed", C.c_int64), ("failed", C.c_int64), ("bytes", C.c_int64), ("elapsed_s", C.c_double),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("max_us", C.c_double), ("mean_us", C.c_double),
                ("launches", C.c_int64), ("late_issues", C.c_int64), ("p50_queue_us", C.c_double),
                ("p99_queue_us", C.c_double), ("p50_run_us", C.c_double), ("p99_run_us", C.c_double),
                ("p50_issue_us", C.c_double), ("p99_issue_us", C.c_double), ("ring_waits", C.c_int64),
                ("ring_wait_us", C.c_double)]


def serve_setup(torch, mdt):
    """The serving workload's resident state: 500 committed types, a seeded
    source arena per type family (pack sources) and a 64 MiB packed input
    (unpack sources)."""
    dev = torch.device("cuda:0")
    fam_types = inputs.serving_types()
    types = [mdt.build_type(spec) for _, spec in fam_types]
    src = {f: torch.from_numpy(inputs.random_bytes(b, seed=inputs.DEFAULT_SEED + i)).to(dev)
           for i, (f, b) in enumerate(SERVE_ARENAS.items())}
    pk_in = torch.from_numpy(inputs.random_bytes(64 << 20, seed=5)).to(dev)
    return dict(fam_types=fam_types, types=types, src=src, pk_in=pk_in)


def serve_requests(V, rate, duration):
    """The trace as the load generator's request array: count = ceil(target /
    type size), capped so count x extent fits the family's source arena
    (target then truncated to count x size); span = the bytes a request
    writes (pack: its output; unpack: its typed span, whose first byte is at
    origin + true_lb)."""
    types, fam_types = V["types"], V["fam_types"]
    tr = inputs.serving_trace(rate, duration, len(types))
    n = tr["t_us"].size
    size = np.array([t.size() for t in types], np.int64)
    ext = np.array([t.extent()[1] for t in types], np.int64)
    tlb = np.array([t.true_extent()[0] for t in types], np.int64)
    tex = np.array([t.true_extent()[1] for t in types], np.int64)
    fam_names = list(SERVE_ARENAS)
    fam_of_type = np.array([fam_names.index(f) for f, _ in fam_types], np.int64)
    arena = np.array([SERVE_ARENAS[f] for f in fam_names], np.int64)
    ti = tr["type_index"].astype(np.int64)
    want = tr["target"].astype(np.int64)
    cnt = -(-want // size[ti])
    cap = 1 + (arena[fam_of_type[ti]] - tlb[ti] - tex[ti]) // np.maximum(1, ext[ti])
    truncated = int((cnt > cap).sum())
    cnt = np.minimum(cnt, cap)
    tgt = np.minimum(want, cnt * size[ti])
    up = tr["unpack"].astype(np.int32)
    reqs = np.zeros(n, LG_REQ)
    reqs["t_arrive_us"] = tr["t_us"]
    reqs["unpack"] = up
    reqs["type_index"] = ti
    reqs["count"] = cnt
    reqs["target"] = tgt
    src_ptr = np.array([V["src"][f].data_ptr() for f in fam_names], np.uint64)
    reqs["typed"] = src_ptr[fam_of_type[ti]]
    reqs["packed"] = V["pk_in"].data_ptr()
    span = np.where(up == 1, (cnt - 1) * ext[ti] + tex[ti], tgt)
    reqs["span"] = span
    reqs["origin_off"] = np.where(up == 1, -tlb[ti], 0)
    return reqs, dict(truncated=truncated, fam=np.array(fam_names)[fam_of_type[ti]], target=tgt)


def pick_samples(reqs, nsample=240, budget=6 * GiB, max_span=256 * MiB):
    """Requests whose destinations are kept for comparison: evenly spaced
    ones plus the largest pack and unpack requests, within a memory budget."""
    n = reqs.size
    order = list(range(0, n, max(1, n // nsample)))
    pk = np.nonzero(reqs["unpack"] == 0)[0]
    upk = np.nonzero((reqs["unpack"] == 1) & (reqs["span"] <= GiB))[0]
    big = list(pk[np.argsort(reqs["target"][pk])[-4:]]) + list(upk[np.argsort(reqs["target"][upk])[-2:]])
    out, used = [], 0
    for i in big + order:
        i = int(i)
        s = int(reqs["span"][i])
        if i in out or s == 0 or (i not in big and s > max_span) or used + s > budget:
            continue
        out.append(i)
        used += (s + 255) // 256 * 256
    return sorted(out)


def serve_replay(torch, mdt, V, rate, duration, ring, samples=True):
    """Replay one trace through the server and as per-request launches."""
    reqs, info = serve_requests(V, rate, duration)
    n = reqs.size
    lg = C.CDLL(os.path.join(HERE, "paper_2402_12274_amd", "libmdt_loadgen.so"))
    dp = C.POINTER(C.c_double)
    lg.mdt_lg_run_served.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(mdt.ServerConfig), C.c_void_p,
                                     C.c_int64, C.POINTER(LgResult), dp]
    lg.mdt_lg_run_plain.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                    C.POINTER(LgResult), dp]
    handles = (C.c_void_p * len(V["types"]))(*[t.handle for t in V["types"]])
    cfg = mdt.ServerConfig(8, 32 << 30, 256, 2, 0)
    sample = pick_samples(reqs) if samples else []
    res, lat, bufs = {}, {}, {}
    for mode in ("served", "per_request"):
        run = reqs.copy()
        keep = []
        for i in sample:
            buf = torch.zeros(int(run["span"][i]), dtype=torch.uint8, device="cuda")
            run["fixed"][i] = buf.data_ptr()
            keep.append(buf)
        bufs[mode] = keep
        torch.cuda.synchronize()
        r = LgResult()
        lt = np.zeros(n)
        log(f"serve: {mode} replay, {n} requests at {rate:.0f}/s")
        if mode == "served":
            rc = lg.mdt_lg_run_served(run.ctypes.data, n, handles, C.byref(cfg), C.c_void_p(ring.data_ptr()),
                                      ring.numel(), C.byref(r), lt.ctypes.data_as(dp))
        else:
            rc = lg.mdt_lg_run_plain(run.ctypes.data, n, handles, 8, C.c_void_p(ring.data_ptr()), ring.numel(),
                                     C.byref(r), lt.ctypes.data_as(dp))
        mdt.check(rc, f"{mode} run")
        torch.cuda.synchronize()
        res[mode], lat[mode] = r, lt
    bad = [i for i, a, b in zip(sample, bufs["served"], bufs["per_request"]) if not torch.equal(a, b)]
    check = {"requests": len(sample), "bytes": int(sum(int(reqs["span"][i]) for i in sample)),
             "mismatching_requests": len(bad), "packs": int(sum(1 for i in sample if reqs["unpack"][i] == 0))}
    return reqs, info, res, lat, check


def serve_summary(r):
    return {"completed": r.completed, "failed": r.failed, "GBps": round(2 * r.bytes / r.elapsed_s / 1e9, 2),
            "p50_us": round(r.p50_us, 1), "p99_us": round(r.p99_us, 1), "max_us": round(r.max_us, 1),
            "launches": r.launches, "late_issues": r.late_issues, "elapsed_s": round(r.elapsed_s, 3),
            "server_p50_queue_us": round(r.p50_queue_us, 1), "server_p99_queue_us": round(r.p99_queue_us, 1),
            "server_p50_run_us": round(r.p50_run_us, 1), "server_p99_run_us": round(r.p99_run_us, 1),
            "p50_issue_us": round(r.p50_issue_us, 2), "p99_issue_us": round(r.p99_issue_us, 2),
            "ring_waits": r.ring_waits, "ring_wait_ms": round(r.ring_wait_us * 1e-3, 2)}


def serve_block(args, torch, mdt):
    V = serve_setup(torch, mdt)
    ring = torch.empty(int(args.ring_gib * GiB), dtype=torch.uint8, device="cuda")
    reqs, info, res, lat, check = serve_replay(torch, mdt, V, args.rate, args.duration, ring)
    fam = info["fam"]
    tgt = info["target"]

    def pct(l, sel):
        v = l[sel & (l >= 0)]
        return [round(float(np.percentile(v, 50)), 1), round(float(np.percentile(v, 99)), 1), int(v.size)] \
            if v.size else None

    breakdown = {}
    for key, sel in [(f, fam == f) for f in SERVE_ARENAS] + \
                    [("<64KiB", tgt < (64 << 10)), ("64KiB-4MiB", (tgt >= (64 << 10)) & (tgt < (4 << 20))),
                     (">=4MiB", tgt >= (4 << 20))]:
        breakdown[key] = {"served_p50_p99_n": pct(lat["served"], sel),
                          "per_request_p50_p99_n": pct(lat["per_request"], sel)}
    out = {"workload": f"serving: Poisson arrivals {args.rate:.0f}/s for {args.duration:.0f} s, 50/50 pack/unpack, "
                       "sizes 256 B x Zipf(1.2) up to 64 MiB, 500 resident types, 8 streams, 32 GiB admission "
                       "budget",
           "requests": int(reqs.size), "offered_bytes": int(tgt.sum()), "truncated_requests": info["truncated"],
           "served": serve_summary(res["served"]), "per_request": serve_summary(res["per_request"]),
           "latency_breakdown_us": breakdown, "sample_check_served_vs_per_request": check,
           "ring_GiB": args.ring_gib}
    if args.sat_rate > 0:
        r2, _, res2, _, check2 = serve_replay(torch, mdt, V, args.sat_rate, args.sat_duration, ring, samples=False)
        out["saturation"] = {"rate_per_s": args.sat_rate, "duration_s": args.sat_duration, "requests": int(r2.size),
                             "served": serve_summary(res2["served"]),
                             "per_request": serve_summary(res2["per_request"])}
    del ring
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# halo self-exchange by typed copy


def copy_bench(args, torch, mdt):
    """Periodic halo self-exchange on a float64 512^3 array: for each dim and
    ghost width 1 and 4, the interior layer next to each side is copied into
    the ghost layer on the opposite side (12 copies per step), as typed
    copies (one pass, no staging) and as pack + unpack through a staging
    buffer (plain launches, and one batched launch per direction)."""
    dev = torch.device("cuda:0")
    n = 512
    D = inputs.DOUBLE
    R = max(1, args.rotate)
    arrs = [torch.from_numpy(inputs.random_bytes(n ** 3 * 8, seed=inputs.DEFAULT_SEED + r)).to(dev) for r in range(R)]
    pairs = []
    for w in (1, 4):
        for dim in (0, 1, 2):
            for side in ("lo", "hi"):
                src = inputs.halo_face(n, w, dim, side)
                sub = [n - 2 * w] * 3
                st = [w] * 3
                sub[dim] = w
                st[dim] = n - w if side == "lo" else 0  # ghost layer on the opposite side
                pairs.append((mdt.build_type(src), mdt.build_type(("subarray", [n, n, n], sub, st, "C", D))))
    sizes = [a.size() for a, _ in pairs]
    stage = [torch.empty(s, dtype=torch.uint8, device=dev) for s in sizes]
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    useful = 2 * sum(sizes)  # algorithmic bytes of the exchange: each byte read once, written once

    def copies(r):
        a = arrs[r].data_ptr()
        for (ta, tb), _ in zip(pairs, sizes):
            mdt.mdt_typed_copy_enqueue(a, 1, ta, a, 1, tb, 0, -1, ms)

    def staged(r):
        a = arrs[r].data_ptr()
        for (ta, _), buf in zip(pairs, stage):
            mdt.mdt_pack_enqueue(a, 1, ta, 0, buf.data_ptr(), -1, ms)
        for (_, tb), buf, s in zip(pairs, stage, sizes):
            mdt.mdt_unpack_enqueue(buf.data_ptr(), s, a, 1, tb, 0, ms)

    batches = []
    for r in range(R):
        bp, bu = mdt.Batch(), mdt.Batch()
        for (ta, tb), buf, s in zip(pairs, stage, sizes):
            bp.add_pack(arrs[r].data_ptr(), 1, ta, 0, buf.data_ptr(), -1)
            bu.add_unpack(buf.data_ptr(), s, arrs[r].data_ptr(), 1, tb, 0)
        batches.append((bp, bu))
    batches[0][0].autotune(ms)
    batches[0][1].autotune(ms)
    for bp, bu in batches[1:]:
        bp.set_config(batches[0][0].get_config())
        bu.set_config(batches[0][1].get_config())

    def batched(r):
        bp, bu = batches[r]
        bp.launch(ms)
        bu.launch(ms)

    def timed(fn, launches):
        for i in range(max(args.warmup, R)):
            fn(i % R)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for i in range(args.steps):
            fn(i % R)
        e1.record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dev_s = e0.elapsed_time(e1) * 1e-3
        return {"GBps": round(useful * args.steps / dt / 1e9, 2), "ms_per_step": round(dt / args.steps * 1e3, 4),
                "avg_launch_us": round(dev_s / (launches * args.steps) * 1e6, 2)}

    cbatches = []
    for r in range(R):
        b = mdt.Batch()
        for ta, tb in pairs:
            b.add_copy(arrs[r].data_ptr(), 1, ta, arrs[r].data_ptr(), 1, tb, 0, -1)
        cbatches.append(b)
    cbatches[0].autotune(ms)
    for b in cbatches[1:]:
        b.set_config(cbatches[0].get_config())

    def copies_batched(r):
        cbatches[r].launch(ms)

    res_copy = timed(copies, len(pairs))
    res_copy_batched = timed(copies_batched, 1)
    res_staged = timed(staged, 2 * len(pairs))
    res_batched = timed(batched, 2)
    achieved = useful / (res_copy_batched["avg_launch_us"] * 1e-6) / 1e9
    out = {
        "metric": METRIC, "value": res_copy_batched["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res_copy_batched["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "periodic halo self-exchange: float64 512^3 array, ghost widths 1 and 4, each "
                               "interior layer copied into the opposite ghost layer (12 typed copies per step)",
                   "bytes_per_step": useful, "rotating_copies": R,
                   "autotuned": mdt.config_dict(cbatches[0].get_config())},
        "typed_copy_batched": res_copy_batched, "typed_copy_plain": res_copy, "pack_unpack_plain": res_staged,
        "pack_unpack_batched": res_batched,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "batch_kernel (typed copies, one launch per step)",
                     "avg_launch_us": res_copy_batched["avg_launch_us"], "bytes_per_launch": int(useful)},
    }
    print(json.dumps(out), flush=True)
    return 0


def standalone(block, args, name):
    """A serve or batch4096 block as its own JSON line."""
    head = {"metric": METRIC, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic"}
    if name == "serve":
        head.update(value=block["served"]["GBps"], ms_per_step=round(block["served"]["elapsed_s"] * 1e3, 3),
                    steps=1, warmup=0)
        head["config"] = {"workload": block["workload"]}
    elif name == "chunked":
        b = block["particles"]["batched_ranges"]
        head.update(value=b["GBps"], ms_per_step=round((b["pack_us"] + b["unpack_us"]) * 1e-3, 4))
        head["config"] = {"workload": "1 MiB byte ranges of the particle records, packed then unpacked as one "
                                      "batch per direction"}
    else:
        head.update(value=block["batched"]["GBps"], ms_per_step=block["batched"]["makespan_ms"],
                    roofline=block["roofline"])
        head["config"] = {"workload": block["workload"]}
    head[name] = block
    print(json.dumps(head), flush=True)
    return 0


# ---------------------------------------------------------------------------


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs one GPU's "
              "share of the work, and splitting a transfer across GPUs (by packed byte range) is not built",
              file=sys.stderr)
        return 2
    import torch

    from paper_2402_12274_amd import mdt

    if args.workload == "serve":
        return standalone(serve_block(args, torch, mdt), args, "serve")
    if args.workload == "batch4096":
        return standalone(batch4096_block(args, torch, mdt, steps=args.steps, warmup=args.warmup), args,
                          "batch4096")
    if args.workload == "copy":
        return copy_bench(args, torch, mdt)
    if args.workload == "chunked":
        return standalone(chunked_block(args, torch, mdt), args, "chunked")
    W = workload(args.workload)
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    batched = args.mode == "batched"
    log(f"{args.workload}: setup and autotune")
    S = step_setup(torch, mdt, W, args.rotate, batched, ms)
    types, sizes = S["types"], S["sizes"]
    step_bytes = 4 * sum(sizes)

    dt, dev_s, host_t = timed_steps(torch, S, batched, ms, stream, args.steps, args.warmup, mdt)
    value = step_bytes * args.steps / dt / 1e9
    tuned = S["tuned"]
    if batched:
        # a direction tuned to policy 3 runs each request's own kernel
        single = [tuned[d]["policy"] == 3 for d in ("pack", "unpack")]
        launches_per_step = sum(len(types) if x else 1 for x in single)
        dom = ("batch_kernel" if not any(single) else "single-request kernels" if all(single)
               else "batch_kernel and single-request kernels") + " (pack and unpack launches)"
    else:
        launches_per_step = 2 * len(types)
        dom = "pack and unpack launches"
    avg_dur = dev_s / (launches_per_step * args.steps)
    bytes_per_launch = step_bytes / launches_per_step
    achieved = bytes_per_launch / avg_dur / 1e9 if avg_dur > 0 else 0.0
    extra = {}
    if batched and not args.no_compare:
        # the persistent, graph-replayed form beside the autotuner's choice
        keep = (S["batches"][0][0].get_config(), S["batches"][0][1].get_config())
        best = None
        for c in PERSISTENT_GRAPH:
            cfg = mdt.BatchConfig(*c)
            set_step_config(S, cfg, cfg)
            d, dv, _ = timed_steps(torch, S, True, ms, stream, args.steps, 1, mdt)
            if best is None or d < best[0]:
                best = (d, dv, c)
        set_step_config(S, *keep)
        extra["persistent_graph"] = {"config": mdt.config_dict(mdt.BatchConfig(*best[2])),
                                     "value": round(step_bytes * args.steps / best[0] / 1e9, 2),
                                     "ms_per_step": round(best[0] / args.steps * 1e3, 4),
                                     "device_ms_per_step": round(best[1] / args.steps * 1e3, 4)}
        dt_plain, dev_plain, _ = timed_steps(torch, S, False, ms, stream, args.steps, 1, mdt)
        extra["per_request"] = {"mode": "plain (one launch per request)",
                                "value": round(step_bytes * args.steps / dt_plain / 1e9, 2),
                                "ms_per_step": round(dt_plain / args.steps * 1e3, 4),
                                "device_ms_per_step": round(dev_plain / args.steps * 1e3, 4)}
    # the outputs of one more step, for the CPU baseline's comparison
    gpu_packed = gpu_dst = None
    if not args.no_cpu_baseline:
        r_last = (args.steps - 1) % S["R"]
        run_step(S, r_last, batched, ms, mdt)
        torch.cuda.synchronize()
        gpu_packed = [p.cpu().numpy() for p in S["packed"][r_last]]
        gpu_dst = S["dsts"][r_last].cpu().numpy()
    del S
    torch.cuda.empty_cache()
    ceiling = None
    if not args.no_ceiling:
        log("copy ceiling")
        ceiling = copy_ceiling(torch, mdt)
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
                   "packed_bytes_per_step": sum(sizes), "rotating_copies": max(1, args.rotate),
                   "frac_of_peak_value": round(value / PEAK_HBM_GBS, 4), "autotuned": tuned},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(args.workload + "/" + args.mode, dom),
                     "kernel": dom,
                     "avg_launch_us": round(avg_dur * 1e6, 2), "bytes_per_launch": int(bytes_per_launch),
                     "launches_per_step": launches_per_step},
        "timing": {"device_ms_per_step": round(dev_s / args.steps * 1e3, 4), **host_t},
        "copy_ceiling": ceiling,
        **extra,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds, gpu_packed, gpu_dst)
    del gpu_packed, gpu_dst
    if args.workload == "halo" and not args.no_extras:
        log("batch4096 block")
        out["batch4096"] = batch4096_block(args, torch, mdt)
        torch.cuda.empty_cache()
        log("chunked block")
        out["chunked_1MiB"] = chunked_block(args, torch, mdt)
        torch.cuda.empty_cache()
        log("serve block")
        out["serve"] = serve_block(args, torch, mdt)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
