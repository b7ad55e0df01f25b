"""Stream order, requests, batched launches and the serving loop on the GPU.

- enqueue semantics: an enqueued pack is visible to later work on the same
  stream with no host synchronisation in between, and to another stream
  after it waits on an event recorded behind the pack; requests complete;
- batches: every request of a mixed batch (vectors, halo faces, hindexed;
  sizes log-uniform) gives the bytes of the same request run alone, for both
  split policies, with and without graph capture, across graph replays with
  eager work in between and after the descriptors change; a batch refilled
  and relaunched on another stream while its last launch is still queued;
  the autotuner returns a valid configuration;
- serving: mixed pack/unpack requests served with continuous batching equal
  the same requests run alone; four client threads at once get the oracle's
  bytes; a tiny budget defers but does not fail;
  injected arena failures fail exactly those requests; shutdown drains.
"""
import numpy as np
import pytest

from gpu_util import first_diff, note, to_dev, to_host, zeros_dev
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    return torch, mdt


def test_enqueue_stream_order(env):
    torch, mdt = env
    note("enqueue stream order")
    spec = inputs.halo_face(128, 2, 2, "lo")
    t = mdt.build_type(spec)
    o = obuild(spec)
    host = inputs.random_bytes(128 ** 3 * 8, seed=31)
    side = torch.cuda.Stream()
    ms = mdt.Stream(side.cuda_stream)
    src = torch.zeros(host.size, dtype=torch.uint8, device="cuda")
    pinned = torch.from_numpy(host).pin_memory()
    out = torch.zeros(t.size(), dtype=torch.uint8, device="cuda")
    with torch.cuda.stream(side):
        src.copy_(pinned, non_blocking=True)          # producer on the stream
        n, req = mdt.mdt_pack_enqueue(src.data_ptr(), 1, t, 0, out.data_ptr(), -1, ms, want_request=True)
        snap = out.clone()                             # consumer on the same stream
        back = torch.zeros_like(src)
        m, req2 = mdt.mdt_unpack_enqueue(snap.data_ptr(), n, back.data_ptr(), 1, t, 0, ms, want_request=True)
    assert n == m == t.size()
    req.wait()
    while not req2.test():
        pass
    side.synchronize()
    ref = o.pack(host, 0, 1)
    assert first_diff(to_host(snap), ref) is None
    exp = np.zeros_like(host)
    o.unpack(ref, exp, 0, 1)
    assert first_diff(to_host(back), exp) is None


def test_cross_stream_order_through_an_event(env):
    """A pack enqueued on stream A behind about a millisecond of copies, an
    event recorded after it, and the unpack of its output enqueued on stream B
    after B waits on that event: the unpack sees the packed bytes.  A third
    stream packs another layout meanwhile, untouched by either."""
    torch, mdt = env
    note("cross-stream order through an event")
    spec_a = inputs.halo_face(128, 4, 2, "lo")
    spec_c = ("vector", 1 << 16, 3, 11, inputs.DOUBLE)
    ta, tc = mdt.build_type(spec_a), mdt.build_type(spec_c)
    oa, oc = obuild(spec_a), obuild(spec_c)
    host = inputs.random_bytes(128 ** 3 * 8, seed=57)
    host_c = inputs.random_bytes(sum(tc.extent()), seed=58)
    src, src_c = to_dev(host), to_dev(host_c)
    packed = zeros_dev(ta.size(), 0)
    back = zeros_dev(host.size, 0)
    out_c = zeros_dev(tc.size(), 0)
    hold_src = torch.ones(1 << 29, dtype=torch.uint8, device="cuda")
    hold_dst = torch.empty_like(hold_src)
    sa, sb, sc = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        for _ in range(4):
            hold_dst.copy_(hold_src)
    n, _ = mdt.mdt_pack_enqueue(src.data_ptr(), 1, ta, 0, packed.data_ptr(), -1, mdt.Stream(sa.cuda_stream))
    ev = torch.cuda.Event()
    ev.record(sa)
    sb.wait_event(ev)
    m, _ = mdt.mdt_unpack_enqueue(packed.data_ptr(), n, back.data_ptr(), 1, ta, 0, mdt.Stream(sb.cuda_stream))
    k, _ = mdt.mdt_pack_enqueue(src_c.data_ptr(), 1, tc, 0, out_c.data_ptr(), -1, mdt.Stream(sc.cuda_stream))
    assert n == m == ta.size() and k == tc.size()
    sb.synchronize()
    sc.synchronize()
    ref = oa.pack(host, 0, 1)
    exp = np.zeros_like(host)
    oa.unpack(ref, exp, 0, 1)
    assert first_diff(to_host(back), exp) is None
    assert first_diff(to_host(packed), ref) is None
    assert first_diff(to_host(out_c), oc.pack(host_c, 0, 1)) is None


def _mix(nreq, seed, n_face=128, vec_count=1 << 14, hi=1 << 20):
    reqs = inputs.batch_mix(nreq=nreq, seed=seed, hi=hi, n_face=n_face, vec_count=vec_count)
    lens, disps = inputs.hindexed_blocks(nblocks=20000, span=1 << 24, seed=seed + 1)
    hspec = inputs.hindexed_type(lens, disps)
    return reqs, hspec


def _arena_bytes(kind, n_face, vec_count):
    if kind == "vector":
        return vec_count * 64 * 8
    if kind == "face":
        return n_face ** 3 * 8
    return 1 << 24


def test_batch_equals_alone(env):
    torch, mdt = env
    n_face, vec_count = 128, 1 << 14
    reqs, hspec = _mix(300, 77, n_face, vec_count)
    arenas = {k: to_dev(inputs.random_bytes(_arena_bytes(k, n_face, vec_count), seed=40 + i))
              for i, k in enumerate(("vector", "face", "hindexed"))}
    cache = {}

    def ty(r):
        key = r["spec_key"]
        if key not in cache:
            cache[key] = mdt.build_type(r["spec"] if r["spec"] is not None else hspec)
        return cache[key]

    plan = []
    for r in reqs:
        t = ty(r)
        n = min(r["target"], t.size())
        plan.append((t, arenas[r["kind"]], n))
    total = sum(n for _, _, n in plan)
    offs = np.concatenate([[0], np.cumsum([n + 16 for _, _, n in plan])])
    alone = zeros_dev(int(offs[-1]), 0)
    for (t, src, n), o in zip(plan, offs):
        mdt.mdt_pack(src.data_ptr(), 1, t, 0, alone.data_ptr() + int(o) + 3, n)
    ref = to_host(alone)
    # every request against the oracle as well
    hosts = {k: to_host(v) for k, v in arenas.items()}
    otypes = {}
    for i in range(len(plan)):
        t, src, n = plan[i]
        key = reqs[i]["spec_key"]
        if key not in otypes:
            otypes[key] = obuild(reqs[i]["spec"] if reqs[i]["spec"] is not None else hspec)
        exp = otypes[key].pack(hosts[reqs[i]["kind"]], 0, 1, 0, n)
        assert first_diff(ref[int(offs[i]) + 3:int(offs[i]) + 3 + n], exp) is None, i
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    out = zeros_dev(int(offs[-1]), 0)
    b = mdt.Batch()
    for (t, src, n), o in zip(plan, offs):
        assert b.add_pack(src.data_ptr(), 1, t, 0, out.data_ptr() + int(o) + 3, n) == n
    for policy, wgs, order in ((0, 4, 0), (1, 4, 0), (0, 0, 0), (0, 4, 1), (1, 2, 1), (0, 0, 1), (2, 0, 0), (2, 0, 1),
                               (3, 0, 0)):
        for graph in (1, 0):
            for tc in (256, 4096):
                note(f"batch policy={policy} wgs={wgs} order={order} graph={graph} tile={tc}")
                b.set_config(mdt.BatchConfig(tc, wgs, policy, graph, order))
                for rep in range(3):
                    out.fill_(0)
                    b.launch(ms)
                    torch.cuda.synchronize()
                    _ = (out[:1024].sum().item())  # eager work between replays
                    assert first_diff(to_host(out), ref) is None, (policy, graph, tc, rep)
    cfg = b.autotune(ms)
    assert cfg.tile_chunks in (256, 512, 1024, 2048, 4096) and 0 <= cfg.wgs_per_cu <= 16
    out.fill_(0)
    b.launch(ms)
    assert first_diff(to_host(out), ref) is None
    assert total > 0
    # change the descriptors: same batch object, new requests (unpack back)
    b.clear()
    back = {k: zeros_dev(v.numel(), 0) for k, v in arenas.items()}
    exp_back = {k: np.zeros(v.numel(), np.uint8) for k, v in arenas.items()}
    seen = set()
    for i, ((t, src, n), o) in enumerate(zip(plan, offs)):
        if reqs[i]["kind"] == "vector" or i % 3:
            continue
        spec = reqs[i]["spec"] if reqs[i]["spec"] is not None else hspec
        key = reqs[i]["spec_key"]
        if key in seen:
            continue  # one request per type: faces of one array only meet where they carry equal bytes
        seen.add(key)
        b.add_unpack(out.data_ptr() + int(o) + 3, n, back[reqs[i]["kind"]].data_ptr(), 1, t, 0)
        obuild(spec).unpack(ref[int(o) + 3:int(o) + 3 + n], exp_back[reqs[i]["kind"]], 0, 1)
    note("batch after descriptor change")
    for rep in range(2):
        b.launch(ms)
        torch.cuda.synchronize()
    for k in back:
        assert first_diff(to_host(back[k]), exp_back[k]) is None, k


def test_batch_relaunch_on_another_stream(env):
    """One batch launched on stream A behind a long copy, then refilled and
    launched on stream B, then refilled again and launched back on A: each
    launch writes what its own requests say.  Without the device-side wait on
    a stream change, B's descriptor upload would land before A's delayed
    kernel reads the descriptors and A's requests would be lost."""
    torch, mdt = env
    D = ("basic", "DOUBLE")
    specs = [("vector", 4096, 2, 5, D), inputs.halo_face(96, 2, 1, "hi")]
    types = [mdt.build_type(s) for s in specs]
    otypes = [obuild(s) for s in specs]
    span = max(sum(t.extent()) for t in types)
    host = inputs.random_bytes(span, seed=91)
    src = to_dev(host)
    nreq = 48
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    msa, msb = mdt.Stream(sa.cuda_stream), mdt.Stream(sb.cuda_stream)
    hold_src = torch.ones(1 << 29, dtype=torch.uint8, device="cuda")
    hold_dst = torch.empty_like(hold_src)
    for cfg in (mdt.BatchConfig(256, 4, 1, 0, 0), mdt.BatchConfig(4096, 0, 0, 1, 1)):
        note(f"relaunch on another stream cfg={mdt.config_dict(cfg)}")
        b = mdt.Batch()
        b.set_config(cfg)
        outs = [zeros_dev(nreq * t.size(), 0) for t in types]
        ext0 = sum(types[0].extent())
        back = zeros_dev(nreq * ext0, 0)
        for i in range(nreq):
            b.add_pack(src.data_ptr(), 1, types[0], 0, outs[0].data_ptr() + i * types[0].size(), -1)
        b.launch(msa)  # sizes the batch's buffers, whose first allocation waits for the device
        torch.cuda.synchronize()
        outs[0].fill_(0)
        torch.cuda.synchronize()
        # launch 1 on A, queued behind about a millisecond of copies
        with torch.cuda.stream(sa):
            for _ in range(4):
                hold_dst.copy_(hold_src)
        b.launch(msa)
        # launch 2 on B with other requests, at once from the host
        b.clear()
        for i in range(nreq):
            b.add_pack(src.data_ptr(), 1, types[1], 0, outs[1].data_ptr() + i * types[1].size(), -1)
        b.launch(msb)
        # launch 3 back on A: unpack what launch 1 packed
        b.clear()
        for i in range(nreq):
            b.add_unpack(outs[0].data_ptr() + i * types[0].size(), types[0].size(), back.data_ptr() + i * ext0, 1,
                         types[0], 0)
        b.launch(msa)
        sa.synchronize()
        sb.synchronize()
        for k in range(2):
            exp = otypes[k].pack(host, 0, 1)
            got = to_host(outs[k]).reshape(nreq, -1)
            for i in range(nreq):
                assert first_diff(got[i], exp) is None, (k, i)
        exp = np.zeros(ext0, dtype=np.uint8)
        otypes[0].unpack(otypes[0].pack(host, 0, 1), exp, 0, 1)
        got = to_host(back).reshape(nreq, ext0)
        for i in range(nreq):
            assert first_diff(got[i], exp) is None, ("unpack", i)
        del b
    del types


def test_batch_mixed_directions(env):
    # pack and unpack requests added in interleaved order run as two launches
    # (pack first); every request gives the oracle's bytes
    torch, mdt = env
    specs = [inputs.particle_struct(), inputs.halo_face(64, 2, 1, "hi"), ("vector", 3000, 3, 7, inputs.DOUBLE)]
    types = [mdt.build_type(sp) for sp in specs]
    orc = [obuild(sp) for sp in specs]
    counts = [5000, 1, 1]
    srcs, outs, exps, pks, dsts, dexp = [], [], [], [], [], []
    for i, (sp, o, c) in enumerate(zip(specs, orc, counts)):
        a = o.attrs()
        nb = (c - 1) * a["extent"] + a["true_ub"] + 8
        h = inputs.random_bytes(nb, seed=50 + i)
        srcs.append(to_dev(h))
        full = o.pack(h, 0, c)
        exps.append(full)
        outs.append(zeros_dev(full.size, 0))
        pks.append(to_dev(full))
        canary = np.full(nb, 0x33, np.uint8)
        e = canary.copy()
        o.unpack(full, e, 0, c)
        dexp.append(e)
        dsts.append(to_dev(canary))
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for wgs, order, pol in ((0, 0, 0), (2, 0, 0), (0, 1, 0), (4, 1, 0), (0, 0, 2), (0, 1, 2), (0, 0, 3)):
        note(f"mixed-direction batch wgs={wgs} order={order} policy={pol}")
        for d, o in zip(dsts, orc):
            d.fill_(0x33)
        for x in outs:
            x.fill_(0)
        b = mdt.Batch()
        for i, (t, c) in enumerate(zip(types, counts)):
            b.add_unpack(pks[i].data_ptr(), exps[i].size, dsts[i].data_ptr(), c, t, 0)
            b.add_pack(srcs[i].data_ptr(), c, t, 0, outs[i].data_ptr(), -1)
        b.set_config(mdt.BatchConfig(1024, wgs, pol, 1, order))
        b.launch(ms)
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert first_diff(to_host(outs[i]), exps[i]) is None, (wgs, i)
            assert first_diff(to_host(dsts[i]), dexp[i]) is None, (wgs, i)


def test_batch_single_body_kernels(env):
    # batches whose requests all take one tile body run a kernel compiled for
    # that body only: run tables (hindexed of bytes), chunk path (faces),
    # record path (particles); pack and unpack must equal the oracle
    torch, mdt = env
    lens, disps = inputs.hindexed_blocks(nblocks=30000, span=1 << 22, seed=21)
    groups = {
        "runs": [inputs.hindexed_type(lens, disps)],
        "chunk": [inputs.halo_face(64, 1, 2, "lo"), inputs.halo_face(64, 4, 0, "hi"), inputs.halo_face(64, 2, 1, "lo")],
        "records": [inputs.particle_struct()],
    }
    counts = {"runs": 2, "chunk": 1, "records": 7001}
    expect_body = {"runs": (3, 0), "chunk": (2, 0), "records": (2, 1)}
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for name, specs in groups.items():
        types = [mdt.build_type(sp) for sp in specs]
        kind, rec = expect_body[name]
        assert all(t.layout_info()["kind"] == kind and t.layout_info()["records"] == rec for t in types), name
        for wgs, order, pol in ((0, 0, 0), (4, 1, 0), (0, 0, 2), (0, 0, 3)):
            note(f"single-body batch {name} wgs={wgs} order={order} policy={pol}")
            bp, bu = mdt.Batch(), mdt.Batch()
            keep = []
            for i, (sp, t) in enumerate(zip(specs, types)):
                o = obuild(sp)
                a = o.attrs()
                c = counts[name]
                nb = (c - 1) * a["extent"] + a["true_ub"] + 8
                h = inputs.random_bytes(nb, seed=70 + i)
                full = o.pack(h, 0, c)
                src, out = to_dev(h), zeros_dev(full.size, 0)
                canary = np.full(nb, 0x21, np.uint8)
                exp_u = canary.copy()
                o.unpack(full, exp_u, 0, c)
                pk, dst = to_dev(full), to_dev(canary)
                bp.add_pack(src.data_ptr(), c, t, 0, out.data_ptr(), -1)
                bu.add_unpack(pk.data_ptr(), full.size, dst.data_ptr(), c, t, 0)
                keep.append((src, out, full, pk, dst, exp_u))
            for b in (bp, bu):
                b.set_config(mdt.BatchConfig(1024, wgs, pol, 1, order))
                b.launch(ms)
            torch.cuda.synchronize()
            for src, out, full, pk, dst, exp_u in keep:
                assert first_diff(to_host(out), full) is None, name
                assert first_diff(to_host(dst), exp_u) is None, name


def test_server_mix_equals_alone(env):
    torch, mdt = env
    n_face, vec_count = 96, 1 << 13
    reqs, hspec = _mix(400, 91, n_face, vec_count, hi=1 << 19)
    arenas = {k: to_dev(inputs.random_bytes(_arena_bytes(k, n_face, vec_count), seed=60 + i))
              for i, k in enumerate(("vector", "face", "hindexed"))}
    cache = {}
    for r in reqs:
        if r["spec_key"] not in cache:
            cache[r["spec_key"]] = mdt.build_type(r["spec"] if r["spec"] is not None else hspec)
    srv = mdt.Server(nstreams=8, budget_bytes=1 << 30, max_batch=64, max_inflight=2)
    srv.start()
    note("server pack mix")
    handles = []
    for r in reqs:
        t = cache[r["spec_key"]]
        n = min(r["target"], t.size())
        handles.append((srv.submit_pack(arenas[r["kind"]].data_ptr(), 1, t, 0, n), t, r, n))
    outs = []
    for h, t, r, n in handles:
        srv.wait(h)
        st, pk, nb, lat = srv.result(h)
        assert st == 0 and nb == n and lat > 0
        got = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        if n:
            torch.cuda.synchronize()
            hip_copy(torch, got, pk, n)
        alone = zeros_dev(n + 16, 0)
        mdt.mdt_pack(arenas[r["kind"]].data_ptr(), 1, t, 0, alone.data_ptr(), n)
        assert first_diff(to_host(got)[:n], to_host(alone)[:n]) is None
        outs.append((h, t, r, n, got))
    # unpack requests: scatter packed faces back through the server
    note("server unpack mix")
    seen = {}
    ups = []
    for h, t, r, n, got in outs:
        if r["kind"] != "face" or r["spec_key"] in seen or n == 0:
            continue
        dst = zeros_dev(n_face ** 3 * 8, 0)
        seen[r["spec_key"]] = dst
        ups.append((srv.submit_unpack(got.data_ptr(), n, dst.data_ptr(), 1, t, 0), t, r, n, got, dst))
    for h, t, r, n, got, dst in ups:
        srv.wait(h)
        assert srv.result(h)[0] == 0
        exp = zeros_dev(n_face ** 3 * 8, 0)
        mdt.mdt_unpack(got.data_ptr(), n, exp.data_ptr(), 1, t, 0)
        assert torch.equal(dst, exp)
        srv.release(h)
    for h, *_ in outs:
        srv.release(h)
    s = srv.stats()
    assert s["completed"] == len(handles) + len(ups) and s["failed"] == 0
    assert s["p99_us"] >= s["p50_us"] > 0
    srv.stop()
    srv.close()


def test_server_concurrent_clients(env):
    """Four client threads submit to one server at once (the library's calls
    run without the interpreter lock): two submit packs of a mix of faces,
    vectors and hindexed ranges, two submit unpacks of face streams into
    destinations of their own, while the progress thread runs.  Every
    request completes with the oracle's bytes."""
    import threading

    torch, mdt = env
    n_face, vec_count = 96, 1 << 13
    reqs, hspec = _mix(240, 123, n_face, vec_count, hi=1 << 19)
    hosts = {k: inputs.random_bytes(_arena_bytes(k, n_face, vec_count), seed=80 + i)
             for i, k in enumerate(("vector", "face", "hindexed"))}
    arenas = {k: to_dev(v) for k, v in hosts.items()}
    types, otypes = {}, {}
    for r in reqs:
        if r["spec_key"] not in types:
            spec = r["spec"] if r["spec"] is not None else hspec
            types[r["spec_key"]] = mdt.build_type(spec)
            otypes[r["spec_key"]] = obuild(spec)
    faces = [(label, spec) for label, spec in inputs.halo_faces(n_face)][:6]
    ftypes = [mdt.build_type(spec) for _, spec in faces]
    ofaces = [obuild(spec) for _, spec in faces]
    fpacked = [o.pack(hosts["face"], 0, 1) for o in ofaces]
    fsrc = [to_dev(p) for p in fpacked]
    nup = 30
    dsts = [[zeros_dev(n_face ** 3 * 8, 0) for _ in range(nup)] for _ in range(2)]
    torch.cuda.synchronize()
    srv = mdt.Server(nstreams=8, budget_bytes=1 << 30, max_batch=32, max_inflight=2)
    srv.start()
    note("server, four client threads")
    got = [[] for _ in range(4)]
    errors = []

    def packer(w):
        try:
            for i in range(w, len(reqs), 2):
                r = reqs[i]
                t = types[r["spec_key"]]
                n = min(r["target"], t.size())
                got[w].append((srv.submit_pack(arenas[r["kind"]].data_ptr(), 1, t, 0, n), i, n))
            for h, _, _ in got[w]:
                srv.wait(h)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    def unpacker(w):
        try:
            for j in range(nup):
                k = (j + w) % len(faces)
                h = srv.submit_unpack(fsrc[k].data_ptr(), fpacked[k].size, dsts[w - 2][j].data_ptr(), 1, ftypes[k], 0)
                got[w].append((h, k, j))
            for h, _, _ in got[w]:
                srv.wait(h)
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=packer, args=(w,)) for w in (0, 1)] + \
              [threading.Thread(target=unpacker, args=(w,)) for w in (2, 3)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    assert not errors, errors
    torch.cuda.synchronize()
    for w in (0, 1):
        for h, i, n in got[w]:
            st, pk, nb, _ = srv.result(h)
            assert st == 0 and nb == n, (w, i)
            out = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
            if n:
                hip_copy(torch, out, pk, n)
            exp = otypes[reqs[i]["spec_key"]].pack(hosts[reqs[i]["kind"]], 0, 1, 0, n)
            assert first_diff(to_host(out)[:n], exp) is None, (w, i)
            srv.release(h)
    expu = []
    for k, o in enumerate(ofaces):
        e = np.zeros(n_face ** 3 * 8, np.uint8)
        o.unpack(fpacked[k], e, 0, 1)
        expu.append(e)
    for w in (2, 3):
        for h, k, j in got[w]:
            assert srv.result(h)[0] == 0
            assert first_diff(to_host(dsts[w - 2][j]), expu[k]) is None, (w, k, j)
            srv.release(h)
    st = srv.stats()
    assert st["completed"] == len(reqs) + 2 * nup and st["failed"] == 0
    srv.stop()
    srv.close()


def hip_copy(torch, dst_tensor, src_ptr, n):
    """Device-to-device copy from a raw pointer (the server's arena)."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(ctypes.c_void_p(dst_tensor.data_ptr()), ctypes.c_void_p(src_ptr), n, 3)
    assert rc == 0


def test_server_budget_defers_and_failures_are_isolated(env):
    torch, mdt = env
    note("server budget / injected failures")
    t = mdt.build_type(("vector", 1 << 16, 1, 2, inputs.DOUBLE))
    src = to_dev(inputs.random_bytes(1 << 20, seed=71))
    srv = mdt.Server(nstreams=2, budget_bytes=3 << 19, max_batch=4, max_inflight=1, arena_bytes=1 << 22)
    srv.inject_alloc_failures(2)
    hs = [srv.submit_pack(src.data_ptr(), 1, t, 0, -1) for _ in range(10)]
    done = []
    for h in hs:
        srv.wait(h)
        done.append(srv.result(h))
        srv.release(h)  # frees its budget so queued requests can be admitted
    codes = [d[0] for d in done]
    assert codes[:2] == [mdt.ERR_NO_MEM, mdt.ERR_NO_MEM] and all(c == 0 for c in codes[2:])
    s = srv.stats()
    assert s["failed"] == 2 and s["completed"] == 8
    assert s["deferred"] > 0 and s["peak_inflight_bytes"] <= 3 << 19
    # shutdown drains requests still queued
    more = [srv.submit_pack(src.data_ptr(), 1, t, 0, -1) for _ in range(5)]
    srv.close()
    assert all(h for h in more)


def test_single_request_policy_graph_follows_requests(env):
    """Policy 3 captures each request's own kernel launch (its arguments
    are in the graph), so a graph replay after the batch's requests change
    must be a new capture: the new destination is written, the old one is
    left alone."""
    torch, mdt = env
    from gpu_util import first_diff, note, to_dev, to_host, zeros_dev

    note("policy 3 graph after the requests change")
    spec = inputs.particle_struct()
    t = mdt.build_type(spec)
    o = obuild(spec)
    count = 3001
    h = inputs.random_bytes(count * 40, seed=91)
    full = o.pack(h, 0, count)
    src = to_dev(h)
    out1, out2 = zeros_dev(full.size, 0), zeros_dev(full.size, 0)
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    b = mdt.Batch()
    b.set_config(mdt.BatchConfig(1024, 0, 3, 1, 0))
    b.add_pack(src.data_ptr(), count, t, 0, out1.data_ptr(), -1)
    b.launch(ms)
    torch.cuda.synchronize()
    assert first_diff(to_host(out1), full) is None
    out1.fill_(0)
    b.clear()
    b.add_pack(src.data_ptr(), count, t, 0, out2.data_ptr(), -1)
    for _ in range(2):
        b.launch(ms)
        torch.cuda.synchronize()
    assert first_diff(to_host(out2), full) is None
    assert not to_host(out1).any()


def test_autotune_set_and_cache(env, tmp_path, monkeypatch):
    """One configuration tuned over rotating copies is applied to all of
    them and stored in the cache file under the batch shape; a later tuning
    of a batch of the same shape reads it back (no timing); the bytes stay
    the oracle's."""
    import json
    import time

    torch, mdt = env
    note("autotune over rotating copies, cache file")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MDT_AUTOTUNE_CACHE", str(cache))
    spec = inputs.halo_face(128, 2, 2, "lo")
    t = mdt.build_type(spec)
    host = inputs.random_bytes(128 ** 3 * 8, seed=81)
    ref = obuild(spec).pack(host, 0, 1)
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    srcs = [to_dev(host) for _ in range(3)]
    outs = [zeros_dev(t.size(), 0) for _ in range(3)]

    def batches():
        bs = []
        for s, o in zip(srcs, outs):
            b = mdt.Batch()
            b.add_pack(s.data_ptr(), 1, t, 0, o.data_ptr(), -1)
            bs.append(b)
        return bs

    bs = batches()
    cfg = mdt.autotune_set(bs, ms)
    assert all(mdt.config_dict(b.get_config()) == mdt.config_dict(cfg) for b in bs)
    entries = json.loads(cache.read_text())
    assert len(entries) == 1 and list(entries.values())[0] == [cfg.tile_chunks, cfg.wgs_per_cu, cfg.policy,
                                                               cfg.use_graph, cfg.order]
    bs2 = batches()
    t0 = time.perf_counter()
    cfg2 = bs2[0].autotune(ms)  # same shape: read back
    assert time.perf_counter() - t0 < 0.05
    assert mdt.config_dict(cfg2) == mdt.config_dict(cfg)
    for o in outs:
        o.fill_(0)
    for b in bs2[:1] + bs[1:]:
        b.launch(ms)
    torch.cuda.synchronize()
    for o in outs:
        assert first_diff(to_host(o), ref) is None
    # a different shape gets its own entry
    b3 = mdt.Batch()
    b3.add_pack(srcs[0].data_ptr(), 1, t, 0, outs[0].data_ptr(), 1000)
    b3.autotune(ms)
    assert len(json.loads(cache.read_text())) == 2
